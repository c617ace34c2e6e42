"""Adjoint of the shape-weighted force field (the differentiable form):
the HIP backward kernel against FP64 central finite differences of the
oracle (step 1e-6) and against the oracle's analytic FP64 adjoint at the
8 192 x 8 192 size, and the autograd wrapper against the direct call."""
import numpy as np
import pytest
import torch

from oracle import ref as O
from synth import random_pair

pytestmark = pytest.mark.gpu

G = 2500.0


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_01061_amd as sg
    return sg


@pytest.fixture(scope="module")
def ctx(sg):
    c = sg.Context(0)
    yield c
    c.close()


def _mom(P):
    c, S, lam = O.moments(P)
    return np.array([c[0], c[1], c[2], S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2], lam])


def _dt(x, dtype=torch.float32):
    return torch.as_tensor(np.asarray(x)).to(device="cuda", dtype=dtype).contiguous()


def _loss_oracle(Y, m, sigma, eps, X, aX, aY, wX, p, g_mode, gf, gF, gK):
    prm = O.Params(p=p, g_mode=g_mode, sigma=sigma, eps=eps)
    S = O.make_setup(X, Y, prm, aX=aX, aY=aY, wX=wX, mY=m)
    f, _ = O.forces(Y, S, G)
    F = (m[:, None] * f).sum(0)
    K = f.T @ (Y - Y.mean(0))
    return float(np.sum(gf * f) + gF @ F + np.sum(gK * K))


@pytest.mark.parametrize("p,g_mode,eps", [(1.0, 0, 0.0), (2.0, 0, 0.05), (2.0, 1, 0.02), (1.5, 0, 0.1),
                                        (-2.0, 2, 0.05)])
def test_force_adjoint_matches_fp64_finite_differences(sg, ctx, p, g_mode, eps):
    pr = random_pair(150, 700, seed=31)
    rng = np.random.default_rng(5)
    X = pr.ref.astype(np.float64)
    Y32 = pr.tmpl.astype(np.float32)
    Y = Y32.astype(np.float64)
    aX = rng.uniform(0.01, 0.3, pr.N).astype(np.float32).astype(np.float64)
    aY = rng.uniform(0.01, 0.3, pr.M).astype(np.float32).astype(np.float64)
    wX = rng.uniform(0.5, 2.0, pr.N).astype(np.float32).astype(np.float64)
    m = rng.uniform(0.5, 2.0, pr.M).astype(np.float32).astype(np.float64)
    sigma = 0.08
    gf = rng.normal(size=(pr.M, 3)).astype(np.float32).astype(np.float64)
    gF = rng.normal(size=3)
    gK = rng.normal(size=(3, 3))

    tm = sg.Cloud(Y32, masses=m)
    rf = sg.Cloud(pr.ref, masses=wX)
    prm = sg.Params(p=p, g_mode=g_mode, sigma=sigma, eps=eps)
    f, _ = ctx.force_fwd(tm, _dt(aY), rf, _dt(aX), _dt(_mom(pr.ref), torch.float64), prm, G)
    gw = _dt(np.concatenate([gF, gK.reshape(-1)]), torch.float64)
    gy, gm, gse = ctx.force_bwd(tm, _dt(aY), rf, _dt(aX), _dt(_mom(pr.ref), torch.float64), prm, G, f,
                                _dt(gf), gw)
    gy, gm, gse = gy.cpu().numpy(), gm.cpu().numpy(), gse.cpu().numpy()

    L = lambda Yv=Y, mv=m, sv=sigma, ev=eps: _loss_oracle(Yv, mv, sv, ev, X, aX, aY, wX, p, g_mode, gf, gF, gK)
    h = 1e-6
    coords = [(int(i), int(c)) for i, c in zip(rng.choice(pr.M, 60, replace=False), rng.integers(0, 3, 60))]
    fd_y = np.zeros(len(coords))
    for n, (i, c) in enumerate(coords):
        Yp, Ym = Y.copy(), Y.copy()
        Yp[i, c] += h
        Ym[i, c] -= h
        fd_y[n] = (L(Yv=Yp) - L(Yv=Ym)) / (2 * h)
    g_sel = np.array([gy[i, c] for i, c in coords])
    assert np.linalg.norm(g_sel - fd_y) / np.linalg.norm(fd_y) <= 1e-4
    idx = np.arange(0, pr.M, 7)
    fd_m = np.array([(L(mv=m + h * (np.arange(pr.M) == i)) - L(mv=m - h * (np.arange(pr.M) == i))) / (2 * h)
                     for i in idx])
    np.testing.assert_allclose(gm[idx], fd_m, rtol=1e-4, atol=1e-4 * np.abs(fd_m).max())
    fd_s = (L(sv=sigma + h) - L(sv=sigma - h)) / (2 * h)
    assert gse[0] == pytest.approx(fd_s, rel=1e-4, abs=1e-6 * abs(L()))
    if eps > 0 and p != 1.0:
        fd_e = (L(ev=eps + h) - L(ev=eps - h)) / (2 * h)
        assert gse[1] == pytest.approx(fd_e, rel=1e-4)
    else:
        assert gse[1] == 0.0


def test_force_adjoint_matches_analytic_oracle_gradient_full_size(sg, ctx):
    """The 8 192 x 8 192 differentiation workload (p = 2, eps = 0.05 L,
    masses): every coordinate, mass, sigma and eps gradient against the
    oracle's analytic FP64 adjoint (finite differences of every coordinate
    would cost 5e4 force evaluations).  The FP32 pair terms of the kernel
    carry about 1e-7 relative error per term; the gate is 1e-4 relative in
    norm (measured errors printed)."""
    from synth import config1
    pr = config1(n=8192)
    rng = np.random.default_rng(12)
    X = pr.ref.astype(np.float64)
    Y32 = pr.tmpl.astype(np.float32)
    aX = O.descriptors(pr.ref, 16).astype(np.float32)
    aY = O.descriptors(pr.tmpl, 16).astype(np.float32)
    m = rng.uniform(0.5, 2.0, pr.M).astype(np.float32)
    wX = rng.uniform(0.5, 2.0, pr.N).astype(np.float32)
    lamX = np.linalg.eigvalsh(np.cov(X.T, bias=True))[-1]
    eps = 0.05 * float(np.sqrt(lamX))
    sigma = float(np.std(aX.astype(np.float64)))
    gf = rng.normal(size=(pr.M, 3)).astype(np.float32).astype(np.float64)
    gF, gK = rng.normal(size=3), rng.normal(size=(3, 3))
    tm = sg.Cloud(Y32, masses=m)
    rf = sg.Cloud(pr.ref, masses=wX)
    prm = sg.Params(p=2.0, g_mode=0, sigma=sigma, eps=eps)
    f, _ = ctx.force_fwd(tm, _dt(aY), rf, _dt(aX), _dt(_mom(pr.ref), torch.float64), prm, G)
    gw = _dt(np.concatenate([gF, gK.reshape(-1)]), torch.float64)
    gy, gm, gse = ctx.force_bwd(tm, _dt(aY), rf, _dt(aX), _dt(_mom(pr.ref), torch.float64), prm, G, f, _dt(gf), gw)
    S = O.make_setup(X, Y32, O.Params(p=2.0, g_mode=0, sigma=sigma, eps=eps), aX=aX.astype(np.float64),
                     aY=aY.astype(np.float64), wX=wX.astype(np.float64), mY=m.astype(np.float64))
    oY, om, osig, oeps = O.force_vjp(Y32.astype(np.float64), S, G, gf, gF, gK)
    gy, gm, gse = gy.cpu().numpy().astype(np.float64), gm.cpu().numpy().astype(np.float64), gse.cpu().numpy()
    e = (np.linalg.norm(gy - oY) / np.linalg.norm(oY), np.linalg.norm(gm - om) / np.linalg.norm(om),
         abs(gse[0] - osig) / abs(osig), abs(gse[1] - oeps) / abs(oeps))
    print(f"adjoint 8192^2 vs analytic FP64: y {e[0]:.1e}, m {e[1]:.1e}, sigma {e[2]:.1e}, eps {e[3]:.1e}")
    assert max(e) <= 1e-4


def test_autograd_function_matches_direct_adjoint(sg, ctx):
    pr = random_pair(2100, 2600, seed=33)      # several tiles and chunks, ragged tails
    rng = np.random.default_rng(6)
    aX = _dt(rng.uniform(0.01, 0.3, pr.N))
    aY = _dt(rng.uniform(0.01, 0.3, pr.M))
    rf = sg.Cloud(pr.ref)
    mom_r = _dt(_mom(pr.ref), torch.float64)
    prm = sg.Params(p=2.0, g_mode=0, sigma=0.1, eps=0.05)
    Y = _dt(pr.tmpl).requires_grad_(True)
    m = torch.ones(pr.M, device="cuda", requires_grad=True)
    sig = torch.tensor(0.1, dtype=torch.float64, device="cuda", requires_grad=True)
    eps = torch.tensor(0.05, dtype=torch.float64, device="cuda", requires_grad=True)
    f, w = sg.ForceField.apply(ctx, Y, m, sig, eps, aY, rf, aX, mom_r, prm, G)
    wt = _dt(rng.normal(size=(pr.M, 3)))
    loss = (f * wt).sum() + w[0:3].sum() + w[3:12].pow(2).sum() * 1e-12
    loss.backward()
    # the same upstream gradients through the direct call
    gw = torch.zeros(12, dtype=torch.float64, device="cuda")
    gw[0:3] = 1.0
    gw[3:12] = 2e-12 * w[3:12].detach()
    tm = sg.Cloud(pr.tmpl, masses=np.ones(pr.M, np.float32))
    gy, gm, gse = ctx.force_bwd(tm, aY, rf, aX, mom_r, prm, G, f.detach(), wt, gw)
    torch.testing.assert_close(Y.grad, gy, rtol=1e-6, atol=1e-6 * gy.abs().max().item())
    torch.testing.assert_close(m.grad, gm, rtol=1e-6, atol=1e-6 * gm.abs().max().item())
    assert sig.grad.item() == pytest.approx(gse[0].item(), rel=1e-9)
    assert eps.grad.item() == pytest.approx(gse[1].item(), rel=1e-9)
