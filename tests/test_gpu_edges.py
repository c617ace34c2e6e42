"""Edge cases of the registration path against the oracle: clouds smaller
than one wave and than one block (every tile ragged), a single reference
tile, degenerate clouds (one point, non-finite coordinates) that must come
back as errors, and the largest workload (the 250 000 x 307 200 depth-frame
scene) on sampled rows along a registration's trajectory."""
import os

import numpy as np
import pytest
import torch

from oracle import ref as O
from parity_bars import F_TOL, row_error
from synth import config5, random_pair, rot_axis_angle

TILES = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1902_01061_amd",
                     "tiles_gfx950.json")

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("M,N,k,p", [(17, 23, 8, 1.0), (63, 65, 16, 2.0), (5, 300, 4, 1.0), (300, 5, 4, 1.0)])
def test_tiny_clouds_step_and_register_match_oracle(sg, ctx, M, N, k, p):
    pr = random_pair(M, N, seed=M * 100 + N)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    a_t, m_t = ctx.descriptors(tm, k)
    a_r, m_r = ctx.descriptors(rf, k)
    aY, aX = a_t.cpu().numpy().astype(np.float64), a_r.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(aY, O.descriptors(pr.tmpl, k), rtol=2e-6, atol=1e-9)
    prm = O.Params(p=p, k=k, E=12)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX, aY=aY)
    pose = O.Pose(0.9, rot_axis_angle([1, 0, 1], 10.0), np.array([0.1, 0.0, -0.1]))
    Y = pose.apply(pr.tmpl)
    so = O.step(Y, S, 5)
    gp = sg.Params(p=p, k=k, E=12)
    pout, wr, f = ctx.step(tm, a_t, rf, a_r, _dt(_mom(pr.tmpl), torch.float64), _dt(_mom(pr.ref), torch.float64),
                           gp, 5, sg.pose_from_srt(pose.s, pose.R, pose.t), want_wrench=True, want_f=True)
    f = f.cpu().numpy().astype(np.float64)
    assert row_error(f, so.f, O.force_scale(Y, S, so.G)) <= F_TOL
    po, _, _ = O.register(pr.tmpl, S)
    # p = 1 also with the pair sums formed once (flags bit 3)
    for flags in ((0, 8) if p == 1.0 else (0,)):
        pg, _ = ctx.register(tm, rf, sg.Params(p=p, k=k, E=12, flags=flags))
        s, R, t = sg.pose_to_srt(pg)
        d = O.Pose(s, R, t).apply(pr.tmpl) - po.apply(pr.tmpl)
        assert np.sqrt(np.mean(np.sum(d * d, axis=1))) <= 1e-4 * O.diameter(pr.ref), flags


def test_degenerate_clouds_are_errors(sg, ctx):
    pr = random_pair(50, 60, seed=4)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    one = sg.Cloud(pr.tmpl[:1].copy())
    with pytest.raises(sg.SgrError) as e:             # one template point: no spread, no rotation
        ctx.register(one, rf, sg.Params(k=1, E=3))
    assert e.value.code in (-2, -5)
    bad = pr.tmpl.copy()
    bad[7, 1] = np.nan
    with pytest.raises(sg.SgrError) as e:             # a non-finite coordinate
        ctx.register(sg.Cloud(bad), rf, sg.Params(k=8, E=3))
    assert e.value.code in (-2, -5)
    bad = pr.ref.copy()
    bad[3, 0] = np.inf
    with pytest.raises(sg.SgrError) as e:
        ctx.register(tm, sg.Cloud(bad), sg.Params(k=8, E=3))
    assert e.value.code in (-2, -5)
    # the context stays usable after errors
    ctx.register(tm, rf, sg.Params(k=8, E=3))


def test_empty_clouds_are_rejected(sg, ctx):
    """A cloud with no points is an argument error (code -1) at every entry
    point that takes one, before any kernel runs; the context stays
    usable."""
    pr = random_pair(40, 50, seed=6)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    empty = sg.Cloud(np.zeros((0, 3), np.float32))
    prm = sg.Params(k=4, E=3)
    calls = [
        ("register, empty template", lambda: ctx.register(empty, rf, prm)),
        ("register, empty reference", lambda: ctx.register(tm, empty, prm)),
        ("descriptors", lambda: ctx.descriptors(empty, 4)),
        ("knn", lambda: ctx.knn(empty, 4)),
        ("residual", lambda: ctx.residual(empty, rf, sg.pose_identity())),
        ("batch with an empty member", lambda: ctx.register_batch([tm, empty], [rf, rf], prm)),
        ("vector registration", lambda: ctx.register_vec(empty, _dt(np.zeros((0, 4))), rf,
                                                         _dt(np.random.rand(50, 4)), sg.Params(p=1.0, E=3))),
        ("batched descriptors", lambda: ctx.descriptors_batch([tm, empty], 4)),
    ]
    for name, call in calls:
        with pytest.raises(sg.SgrError) as e:
            call()
        assert e.value.code == -1, name
    pose, _ = ctx.register(tm, rf, prm)
    assert np.isfinite(pose.cpu().numpy()).all()


@pytest.mark.parametrize("p,flags,tol", [(1.0, 0, F_TOL), (1.0, 2, 2e-3), (2.0, 0, F_TOL)])
def test_largest_workload_force_along_trajectory(sg, ctx, p, flags, tol):
    """The depth-frame scene (250 000 x 307 200, g = a a s): the force at the
    poses the FP32 registration reaches before iterations 0-4, 10, 50 and 99,
    on 256 sampled rows against the C oracle by the per-point bar, in the
    launch shapes of the committed tile table (the shapes the bench times):
    the FP32 kernel at p = 1 and p = 2, and the mixed-precision one (whose
    gate, 2e-3, is derived in test_gpu_mixed.py from the bf16 rounding of the
    pair weights)."""
    pr = config5()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    E = 100
    _, st = ctx.register(tm, rf, sg.Params(p=1.0, g_mode=1, k=16, E=E), stats=True)
    traj = st.cpu().numpy()
    a_t, mom_t = ctx.descriptors(tm, 16)
    a_r, mom_r = ctx.descriptors(rf, 16)
    S = O.make_setup(pr.ref, pr.tmpl, O.Params(p=p, g_mode=1, k=16, E=E),
                     aX=a_r.cpu().numpy().astype(np.float64), aY=a_t.cpu().numpy().astype(np.float64))
    ctx_t = sg.Context(0)
    ctx_t.load_tiles(TILES)
    plan = sg.Plan(ctx_t, tm, a_t, rf, a_r, mom_t, mom_r, sg.Params(p=p, g_mode=1, k=16, E=E, flags=flags))
    rows = np.random.default_rng(5).choice(pr.M, 256, replace=False)
    errs = []
    for t in (0, 1, 2, 3, 4, 10, 50, 99):
        P = np.concatenate([[1.0], np.eye(3).reshape(-1), np.zeros(3)]) if t == 0 else traj[t - 1][14:27]
        _, f = plan.force(_dt(P, torch.float64), t=t, want_wrench=False, want_f=True)
        f = f.cpu().numpy().astype(np.float64)[rows]
        Yt = P[0] * pr.tmpl.astype(np.float64) @ P[1:10].reshape(3, 3).T + P[10:13]
        f_o, _, sc = O.forces_c(Yt, S, O.G_schedule(t, E), rows=rows, want_scale=True)
        errs.append(row_error(f, f_o, sc))
    plan.close()
    ctx_t.close()
    print(f"scene force along the trajectory (p {p:g}, flags {flags}): " + ", ".join(f"{e:.1e}" for e in errs))
    assert max(errs) <= tol


@pytest.mark.parametrize("flags", [0, 4])
def test_tiny_clouds_vector_step_matches_oracle(sg, ctx, flags):
    """Vector descriptors with fewer points than one row tile and one LDS
    stage (both product forms)."""
    pr = random_pair(19, 37, seed=8)
    rng = np.random.default_rng(8)
    aX = rng.random((37, 7)).astype(np.float32)
    aY = rng.random((19, 7)).astype(np.float32)
    prm = O.Params(p=1.0, k=16, E=10)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX.astype(np.float64), aY=aY.astype(np.float64))
    so = O.step(pr.tmpl.astype(np.float64), S, 3)
    sc = O.force_scale(pr.tmpl.astype(np.float64), S, so.G)
    gp = sg.Params(p=1.0, k=16, E=10, flags=flags)
    _, wr, f = ctx.step_vec(sg.Cloud(pr.tmpl), _dt(aY), sg.Cloud(pr.ref), _dt(aX), _dt(_mom(pr.tmpl), torch.float64),
                            _dt(_mom(pr.ref), torch.float64), gp, 3, sg.pose_identity(), want_wrench=True,
                            want_f=True)
    f = f.cpu().numpy().astype(np.float64)
    assert row_error(f, so.f, sc) <= F_TOL
    assert np.linalg.norm(wr.cpu().numpy()[0:3] - so.F) <= F_TOL * np.abs(so.f).sum()
    # the registration, per-iteration kernel and pair sums formed once
    po, _, _ = O.register(pr.tmpl, S)
    for fl in (flags, flags | 8):
        pg, _ = ctx.register_vec(sg.Cloud(pr.tmpl), _dt(aY), sg.Cloud(pr.ref), _dt(aX),
                                 sg.Params(p=1.0, k=16, E=10, flags=fl))
        s_, R_, t_ = sg.pose_to_srt(pg)
        d = O.Pose(s_, R_, t_).apply(pr.tmpl) - po.apply(pr.tmpl)
        assert np.sqrt(np.mean(np.sum(d * d, axis=1))) <= 1e-4 * O.diameter(pr.ref), fl


@pytest.mark.parametrize("p", [1.0, 2.0])
def test_step_beyond_32bit_pair_count_sampled(sg, ctx, p):
    """2 097 159 template x 2 097 161 reference points (4.4e12 pairs per
    step, past 32-bit pair counts), curvatures from the GPU (k = 16, shared
    with the oracle): one step's per-point forces on 128 sampled rows meet
    the per-point bar, and the wrench equals the FP64 sum of the step's own
    per-point forces (F = sum f, K = sum f (y - ybar)^T) to 1e-5 of the
    absolute-sum scales."""
    M, N = (1 << 21) + 7, (1 << 21) + 9
    pr = random_pair(M, N, seed=31)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    a_t, mom_t = ctx.descriptors(tm, 16)
    a_r, mom_r = ctx.descriptors(rf, 16)
    eps = 0.0 if p == 1.0 else 0.01
    prm = O.Params(p=p, k=16, E=100, eps=eps)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=a_r.cpu().numpy().astype(np.float64),
                     aY=a_t.cpu().numpy().astype(np.float64))
    t = 3
    _, wr, f = ctx.step(tm, a_t, rf, a_r, mom_t, mom_r, sg.Params(p=p, k=16, E=100, eps=eps), t,
                        sg.pose_identity(), want_wrench=True, want_f=True)
    f = f.cpu().numpy().astype(np.float64)
    wr = wr.cpu().numpy()
    rows = np.random.default_rng(2).choice(M, 128, replace=False)
    G = O.G_schedule(t, 100)
    Y = pr.tmpl.astype(np.float64)
    f_o, _, sc = O.forces_c(Y, S, G, rows=rows, want_scale=True)   # the C loops: same definition
    e = row_error(f[rows], f_o, sc)
    Yc = Y - Y.mean(axis=0)
    nf = np.linalg.norm(f, axis=1)
    e_F = np.linalg.norm(wr[0:3] - f.sum(axis=0)) / nf.sum()
    e_K = np.linalg.norm(wr[3:12].reshape(3, 3) - f.T @ Yc) / np.sum(nf * np.linalg.norm(Yc, axis=1))
    print(f"p = {p:g}, {M} x {N}: sampled force error {e:.1e}, wrench vs own forces F {e_F:.1e} K {e_K:.1e}")
    assert e <= F_TOL
    assert e_F <= 1e-5 and e_K <= 1e-5
