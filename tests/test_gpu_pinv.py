"""Registration with the pose-independent pair sums of the p = 1 law (flags
bit 3): the sums over the reference are formed once and every iteration is
O(M).  Compared with the oracle, which evaluates every pair at every
iteration as eq. 5 is written (pose parity within 1e-4 of the diameter, the
registration bar), and with the per-iteration all-pairs kernel on the same
inputs, which computes the same FP32 pair terms in another order (pose
difference within 1e-6 of the diameter, per-iteration statistics within
1e-5 relative)."""
import numpy as np
import pytest
import torch

from oracle import ref as O
from synth import config1, config2, config4, super_fibonacci_rotations

pytestmark = pytest.mark.gpu

PINV = 8


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


def _pose(sg, p):
    s, R, t = sg.pose_to_srt(p)
    return O.Pose(s, R, t)


def _rmse(pa, pb, P):
    d = pa.apply(P) - pb.apply(P)
    return float(np.sqrt(np.mean(np.sum(d * d, axis=1))))


@pytest.mark.parametrize("g_mode,masses,eps", [(0, False, 0.0), (1, False, 0.0), (0, True, 0.02)])
def test_register_pinv_matches_oracle(sg, ctx, g_mode, masses, eps):
    pr = config1()
    rng = np.random.default_rng(5)
    wX = rng.uniform(0.5, 2.0, pr.N).astype(np.float32) if masses else None
    mY = rng.uniform(0.5, 2.0, pr.M).astype(np.float32) if masses else None
    prm = O.Params(p=1.0, g_mode=g_mode, k=16, eps=eps, E=100)
    S = O.make_setup(pr.ref, pr.tmpl, prm, wX=wX, mY=mY)
    po, _, _ = O.register(pr.tmpl, S)
    tm, rf = sg.Cloud(pr.tmpl, mY), sg.Cloud(pr.ref, wX)
    D = O.diameter(pr.ref)
    poses = {}
    for flags in (0, PINV):
        gp = sg.Params(p=1.0, g_mode=g_mode, k=16, eps=eps, E=100, flags=flags)
        pose, _ = ctx.register(tm, rf, gp)
        poses[flags] = _pose(sg, pose)
    e_o = _rmse(poses[PINV], po, pr.tmpl) / D
    e_k = _rmse(poses[PINV], poses[0], pr.tmpl) / D
    print(f"pose-independent sums, g_mode {g_mode}, masses {masses}: vs oracle {e_o:.1e} D, "
          f"vs all-pairs kernel {e_k:.1e} D")
    assert e_o <= 1e-4
    assert e_k <= 1e-6


def test_register_pinv_stats_follow_all_pairs_kernel(sg, ctx):
    """G, F, K, U, the pose and the scale at every iteration."""
    pr = config1(n=2000)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    out = []
    for flags in (0, PINV):
        pose, st = ctx.register(tm, rf, sg.Params(p=1.0, k=16, E=40, flags=flags), stats=True)
        out.append(st.cpu().numpy())
    a, b = out
    assert np.array_equal(a[:, 0], b[:, 0])                              # G_t
    for t in range(40):
        for lo, hi in ((1, 4), (4, 13), (13, 14)):                      # F, K, U
            scale = np.abs(a[t, lo:hi]).max()
            assert np.abs(b[t, lo:hi] - a[t, lo:hi]).max() <= 1e-5 * scale, (t, lo)
    assert np.abs(b[:, 14:28] - a[:, 14:28]).max() <= 1e-6              # pose after the update, scale c
    assert np.array_equal(b[:, 28], a[:, 28])                            # status words


def test_register_pinv_scan_sized(sg, ctx):
    """The scan-sized pair (32 400 x 36 000, k = 24, 300 iterations) against
    the all-pairs kernel."""
    pr = config2()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    poses = {}
    for flags in (0, PINV):
        pose, _ = ctx.register(tm, rf, sg.Params(p=1.0, k=24, E=300, flags=flags))
        poses[flags] = _pose(sg, pose)
    e = _rmse(poses[PINV], poses[0], pr.tmpl) / O.diameter(pr.ref)
    print(f"scan-sized registration, pose-independent sums vs all-pairs kernel: {e:.1e} D")
    assert e <= 1e-6


def test_register_pyramid_pinv(sg, ctx):
    pr = config1()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    levels = [sg.Level(1.0, 1.0, 20), sg.Level(0.0, 1.0, 30, 16)]
    poses = {}
    for flags in (0, PINV):
        pose, _ = ctx.register_pyramid(tm, rf, sg.Params(p=1.0, k=16, E=50, flags=flags), levels)
        poses[flags] = _pose(sg, pose)
    assert _rmse(poses[PINV], poses[0], pr.tmpl) / O.diameter(pr.ref) <= 1e-6


def test_batch_pinv_matches_all_pairs_batch(sg, ctx):
    """Uneven registrations in one batched call: poses, final energies and
    per-iteration statistics against the persistent all-pairs batch."""
    pairs = config4(B=7, nmin=300, nmax=6000, iters=25)
    tms = [sg.Cloud(p.tmpl) for p in pairs]
    rfs = [sg.Cloud(p.ref) for p in pairs]
    out = {}
    for flags in (0, PINV):
        poses, energy, st = ctx.register_batch(tms, rfs, sg.Params(p=1.0, k=16, E=25, flags=flags), stats=True)
        out[flags] = (poses.cpu().numpy(), energy.cpu().numpy(), st.cpu().numpy())
    for r, pr in enumerate(pairs):
        pa, pb = _pose(sg, torch.as_tensor(out[0][0][r])), _pose(sg, torch.as_tensor(out[PINV][0][r]))
        assert _rmse(pa, pb, pr.tmpl) <= 1e-6 * O.diameter(pr.ref), r
    np.testing.assert_allclose(out[PINV][1], out[0][1], rtol=1e-5)
    np.testing.assert_allclose(out[PINV][2][..., 0], out[0][2][..., 0], rtol=0, atol=0)   # G_t
    # one registration of the batch against the oracle
    pr = pairs[3]
    S = O.make_setup(pr.ref, pr.tmpl, O.Params(p=1.0, k=16, E=25))
    po, _, _ = O.register(pr.tmpl, S)
    assert _rmse(_pose(sg, torch.as_tensor(out[PINV][0][3])), po, pr.tmpl) <= 1e-4 * O.diameter(pr.ref)


def test_multistart_pinv_matches_all_pairs_multistart(sg, ctx):
    pr = config1(n=1500)
    R0 = super_fibonacci_rotations(6)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    out = {}
    for flags in (0, PINV):
        poses, energy, best = ctx.multistart(tm, rf, sg.Params(p=1.0, k=16, E=20, flags=flags), R0)
        out[flags] = (poses.cpu().numpy(), energy.cpu().numpy(), int(best))
    for s in range(len(R0)):
        pa, pb = _pose(sg, torch.as_tensor(out[0][0][s])), _pose(sg, torch.as_tensor(out[PINV][0][s]))
        assert _rmse(pa, pb, pr.tmpl) <= 1e-6 * O.diameter(pr.ref), s
    np.testing.assert_allclose(out[PINV][1], out[0][1], rtol=1e-5)
    assert out[PINV][2] == out[0][2]


@pytest.mark.parametrize("flags", [0, 4])
def test_register_vec_pinv(sg, ctx, flags):
    """Vector descriptors (16-bin histograms of normals): the sums come from
    one pass of the matrix-core kernel (split f16, or FP32 products with
    flags bit 2); against the oracle and the per-iteration kernel."""
    pr = config1()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    hX = ctx.descriptors_hn(rf, 16, 16)
    hY = ctx.descriptors_hn(tm, 16, 16)
    prm = O.Params(p=1.0, k=16, E=60)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=hX.cpu().numpy().astype(np.float64),
                     aY=hY.cpu().numpy().astype(np.float64))
    po, _, _ = O.register(pr.tmpl, S)
    poses = {}
    for f in (flags, flags | PINV):
        pose, _ = ctx.register_vec(tm, hY, rf, hX, sg.Params(p=1.0, k=16, E=60, flags=f))
        poses[f] = _pose(sg, pose)
    D = O.diameter(pr.ref)
    e_o = _rmse(poses[flags | PINV], po, pr.tmpl) / D
    e_k = _rmse(poses[flags | PINV], poses[flags], pr.tmpl) / D
    print(f"vector registration with pose-independent sums (flags {flags}): vs oracle {e_o:.1e} D, "
          f"vs per-iteration kernel {e_k:.1e} D")
    assert e_o <= 1e-4
    assert e_k <= 1e-6


def test_pinv_rejected_where_it_does_not_apply(sg, ctx):
    pr = config1(n=300)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    for bad in (sg.Params(p=2.0, k=16, E=5, flags=PINV),
                sg.Params(p=-2.0, g_mode=2, eps=0.1, k=16, E=5, flags=PINV),
                sg.Params(p=1.0, k=16, E=5, flags=PINV | 2)):
        with pytest.raises(sg.SgrError):
            ctx.register(tm, rf, bad)
        with pytest.raises(sg.SgrError):
            ctx.register_batch([tm], [rf], bad)
    # entry points without the O(M) iteration
    a, mom = ctx.descriptors(tm, 16)
    with pytest.raises(sg.SgrError):
        sg.Plan(ctx, tm, a, rf, ctx.descriptors(rf, 16)[0], mom, ctx.descriptors(rf, 16)[1],
                sg.Params(p=1.0, k=16, E=5, flags=PINV))
