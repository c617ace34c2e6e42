"""Vector shape descriptors (soft histograms of normals) and the force whose
similarity exponents are one dense contraction on the matrix cores, against
the oracle.

Tolerances.  Histograms: the GPU's Jacobi eigenvectors and the oracle's
LAPACK ones agree to about 1e-15 divided by the gap between the two smallest
eigenvalues, so points whose normal is determined (gap above 1e-3 of the
trace) are compared to 2e-6 absolute (float32 output of values <= 1); the
others have no unique normal and are excluded.  Forces: the exponent of a
pair is an FP32 dot product of K = 4 ceil((D + 2) / 4) terms of magnitude up
to about 4 kappa |a - abar|^2 (below 30 here), so it carries an absolute
error of order K 2^-24 30, i.e. 4e-5 relative in each pair weight at worst;
sums run in FP32 over at most 128 terms per lane before FP64.  The gate is
the force tolerance of the scalar path, 1e-4 relative per iteration (the
measured errors are printed)."""
import numpy as np
import pytest
import torch

from oracle import ref as O
from parity_bars import row_error
from synth import config1, config2, random_pair, rot_axis_angle
from synth.clouds import ellipsoid_patch

pytestmark = pytest.mark.gpu

F_TOL = 1e-4


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


@pytest.mark.parametrize("n,k,D", [(3001, 16, 16), (2000, 8, 5), (700, 24, 30)])
def test_normal_histograms_match_oracle(sg, ctx, n, k, D):
    P = ellipsoid_patch(n, 13).astype(np.float32)
    h = ctx.descriptors_hn(sg.Cloud(P), k, D).cpu().numpy()
    h_o, lam = O.normal_histograms(P, k, D)
    ok = (lam[:, 1] - lam[:, 0]) > 1e-3 * lam.sum(axis=1)
    assert ok.mean() > 0.9
    err = np.abs(h[ok] - h_o[ok]).max()
    print(f"normal histograms n={n} k={k} D={D}: max abs error {err:.1e} on {ok.mean():.1%} of the points")
    assert err <= 2e-6
    np.testing.assert_allclose(h.sum(axis=1), 1.0, rtol=1e-5)


@pytest.mark.parametrize("n,k", [(3001, 16), (2000, 8), (700, 24)])
def test_poly_descriptors_match_oracle(sg, ctx, n, k):
    """Local polynomial descriptors (quadric fit in the covariance frame)
    against the oracle on the points whose normal is determined.  The GPU
    solves the FP64 normal equations, the oracle an SVD least-squares
    problem; both round once to float32."""
    P = ellipsoid_patch(n, 17).astype(np.float32)
    d = ctx.descriptors_poly(sg.Cloud(P), k).cpu().numpy()
    d_o, lam = O.poly_descriptors(P, k)
    ok = (lam[:, 1] - lam[:, 0]) > 1e-3 * lam.sum(axis=1)
    assert ok.mean() > 0.9
    err = np.abs(d[ok] - d_o[ok]).max()
    scale = np.abs(d_o[ok]).max()
    print(f"poly descriptors n={n} k={k}: max abs error {err:.1e} (values up to {scale:.2f}) on {ok.mean():.1%}")
    np.testing.assert_allclose(d[ok], d_o[ok].astype(np.float32), rtol=1e-5, atol=1e-6)


def test_poly_descriptors_plane_full_size_and_bad_arguments(sg, ctx):
    g = np.stack(np.meshgrid(np.arange(30), np.arange(20)), -1).reshape(-1, 2).astype(np.float32)
    plane = np.concatenate([g, np.zeros((len(g), 1), np.float32)], axis=1)
    d = ctx.descriptors_poly(sg.Cloud(plane), 12).cpu().numpy()
    assert np.abs(d).max() <= 1e-6
    pr = config2()
    rows = np.random.default_rng(3).choice(pr.N, 80, replace=False)
    d = ctx.descriptors_poly(sg.Cloud(pr.ref), 24).cpu().numpy()[rows]
    d_o, lam = O.poly_descriptors(pr.ref, 24, rows)
    ok = (lam[:, 1] - lam[:, 0]) > 1e-3 * lam.sum(axis=1)
    np.testing.assert_allclose(d[ok], d_o[ok].astype(np.float32), rtol=1e-5, atol=1e-6)
    for k in (5, 33):
        with pytest.raises(sg.SgrError):
            ctx.descriptors_poly(sg.Cloud(pr.ref), k)


def test_register_vec_with_poly_descriptors_matches_oracle(sg, ctx):
    pr = config1()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    aX = ctx.descriptors_poly(rf, 16)
    aY = ctx.descriptors_poly(tm, 16)
    prm = O.Params(p=1.0, k=16, E=60)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX.cpu().numpy().astype(np.float64),
                     aY=aY.cpu().numpy().astype(np.float64))
    po, _, _ = O.register(pr.tmpl, S)
    pose, _ = ctx.register_vec(tm, aY, rf, aX, sg.Params(p=1.0, k=16, E=60))
    s, R, t = sg.pose_to_srt(pose)
    d = O.Pose(s, R, t).apply(pr.tmpl) - po.apply(pr.tmpl)
    err = np.sqrt(np.mean(np.sum(d * d, axis=1))) / O.diameter(pr.ref)
    gt = O.pose_rmse(po, pr.tmpl, pr.gt_s, pr.gt_R, pr.gt_t) / O.diameter(pr.ref)
    print(f"registration with polynomial descriptors: parity {err:.2e} D (oracle pose error {gt:.3f} D)")
    assert err <= 1e-4


def _vec_case(D, seed, kind):
    pr = random_pair(1300, 2900, seed=seed)         # several tiles and chunks, ragged tails
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        aX = rng.random((pr.N, D)).astype(np.float32)
        aY = rng.random((pr.M, D)).astype(np.float32)
    else:                                            # clustered, with far outliers
        cen = rng.random((6, D))
        aX = (cen[rng.integers(0, 6, pr.N)] + 0.05 * rng.normal(size=(pr.N, D))).astype(np.float32)
        aY = (cen[rng.integers(0, 6, pr.M)] + 0.05 * rng.normal(size=(pr.M, D))).astype(np.float32)
        aY[:20] += 2.0
        if kind == "extreme":                        # beyond the f16 range of the split form
            sd = np.sqrt(np.mean(np.sum((aX - aX.mean(0)) ** 2, axis=1)))
            aY[20:23] = aX.mean(0) + 500.0 * sd / np.sqrt(D)
            aX[:2] = aY[20]
        elif kind == "far":                          # far rows within the f16 range, with close partners
            sd = np.sqrt(np.mean(np.sum((aX - aX.mean(0)) ** 2, axis=1)))
            u = rng.normal(size=(10, D))
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            aY[20:30] = aX.mean(0) + 20.0 * sd * u
            aX[:10] = aY[20:30] + 0.1 * sd * rng.normal(size=(10, D))
    return pr, aX, aY


def _step_both(sg, ctx, pr, aX, aY, prm, pose, t, wX=None, mY=None, flags=0):
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX.astype(np.float64), aY=aY.astype(np.float64), wX=wX, mY=mY)
    Y = pose.apply(pr.tmpl)
    so = O.step(Y, S, t)
    so.scale = O.force_scale(Y, S, so.G)
    ora_pose = O.compose(pose, so, Y.mean(axis=0))
    tm = sg.Cloud(pr.tmpl, masses=mY)
    rf = sg.Cloud(pr.ref, masses=wX)
    gp = sg.Params(p=prm.p, g_mode=prm.g_mode, k=prm.k, sigma=prm.sigma, eps=prm.eps, E=prm.E, flags=flags)
    pout, wr, f = ctx.step_vec(tm, _dt(aY), rf, _dt(aX), _dt(_mom(pr.tmpl), torch.float64),
                               _dt(_mom(pr.ref), torch.float64), gp, t, sg.pose_from_srt(pose.s, pose.R, pose.t),
                               want_wrench=True, want_f=True)
    return so, ora_pose, pout.cpu().numpy(), wr.cpu().numpy(), f.cpu().numpy().astype(np.float64), Y


def _errors(so, wr, f, Y, mY=None):
    """Per-point bar (parity_bars) on every row; F, K against their
    absolute-sum scales; U relatively."""
    m = np.ones(len(f)) if mY is None else np.asarray(mY, np.float64)
    e_f = row_error(f, so.f, so.scale)
    e_F = np.linalg.norm(wr[0:3] - so.F) / np.sum(m * np.linalg.norm(so.f, axis=1))
    Yc = Y - Y.mean(axis=0)
    e_K = np.linalg.norm(wr[3:12].reshape(3, 3) - so.K) / np.sum(np.linalg.norm(so.f, axis=1) *
                                                                 np.linalg.norm(Yc, axis=1))
    e_U = abs(wr[12] - so.U) / abs(so.U)
    return e_f, e_F, e_K, e_U


@pytest.mark.parametrize("D,kind,masses,eps,flags", [
    (16, "uniform", False, 0.0, 0), (30, "clustered", True, 0.02, 0), (5, "uniform", True, 0.0, 0),
    (1, "clustered", False, 0.0, 0), (14, "clustered", False, 0.0, 0),
    (16, "uniform", False, 0.0, 4), (30, "clustered", True, 0.02, 4), (5, "uniform", True, 0.0, 4),
    (9, "extreme", True, 0.0, 0), (19, "uniform", True, 0.0, 0), (20, "clustered", False, 0.01, 0),
    (5, "far", True, 0.0, 0), (5, "far", False, 0.0, 4)])
def test_step_vec_matches_oracle(sg, ctx, D, kind, masses, eps, flags):
    """flags 0: split-f16 products (the default), except for "extreme", whose
    descriptors lie 500 spreads from the mean and select FP32 products by
    themselves; flags 4: FP32 products.  Template rows more than 8 spreads
    from the mean ("extreme": 3 rows at 500 spreads; "far": 10 rows at 20
    spreads, each with a close reference partner) are evaluated exactly
    outside the contraction, so every row meets the per-point bar.  The split form takes
    ceil(3 (D + 2) / 32) 16x16x32 instructions: one for D = 1, 5; two for
    D = 14, 16 and 19 (63 of 64 slots); three for D = 20 and 30."""
    pr, aX, aY = _vec_case(D, 40 + D, kind)
    rng = np.random.default_rng(D)
    wX = rng.uniform(0.5, 2.0, pr.N).astype(np.float32).astype(np.float64) if masses else None
    mY = rng.uniform(0.5, 2.0, pr.M).astype(np.float32).astype(np.float64) if masses else None
    prm = O.Params(p=1.0, k=16, eps=eps, E=40)
    pose = O.Pose(1.1, rot_axis_angle([1, 2, 3], 20.0), np.array([0.1, -0.2, 0.05]))
    for t in (0, 39):
        so, ora_pose, pout, wr, f, Y = _step_both(sg, ctx, pr, aX, aY, prm, pose, t, wX, mY, flags)
        e = _errors(so, wr, f, Y, mY)
        print(f"vector step D={D} {kind} flags={flags} t={t}: e_f={e[0]:.1e} e_F={e[1]:.1e} e_K={e[2]:.1e} "
              f"e_U={e[3]:.1e}")
        assert max(e) <= F_TOL, e
        gp = O.Pose(pout[0], pout[1:10].reshape(3, 3), pout[10:13])
        d = gp.apply(pr.tmpl) - ora_pose.apply(pr.tmpl)
        assert np.sqrt(np.mean(np.sum(d * d, axis=1))) <= 1e-4 * O.diameter(pr.ref)


def test_step_vec_with_one_dimension_is_the_scalar_step(sg, ctx):
    """D = 1 through the matrix cores and the scalar kernel agree (both
    against the same oracle step) on the same curvatures."""
    pr = random_pair(2100, 2600, seed=9)
    rng = np.random.default_rng(9)
    aX = rng.uniform(0.0, 0.3, pr.N).astype(np.float32)
    aY = rng.uniform(0.0, 0.3, pr.M).astype(np.float32)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    gp = sg.Params(p=1.0, k=16, E=40)
    pin = sg.pose_from_srt(0.9, rot_axis_angle([0, 1, 1], 15.0), np.array([0.05, 0.1, -0.1]))
    mt, mr = _dt(_mom(pr.tmpl), torch.float64), _dt(_mom(pr.ref), torch.float64)
    _, w1, f1 = ctx.step(tm, _dt(aY), rf, _dt(aX), mt, mr, gp, 7, pin, want_wrench=True, want_f=True)
    _, w2, f2 = ctx.step_vec(tm, _dt(aY[:, None]), rf, _dt(aX[:, None]), mt, mr, gp, 7, pin, want_wrench=True,
                             want_f=True)
    f1, f2 = f1.cpu().numpy().astype(np.float64), f2.cpu().numpy().astype(np.float64)
    e = np.linalg.norm(f2 - f1) / np.linalg.norm(f1)
    print(f"D = 1 vector path vs scalar path: force difference {e:.1e}")
    assert e <= 2e-5
    w1, w2 = w1.cpu().numpy(), w2.cpu().numpy()
    assert np.linalg.norm(w2[:12] - w1[:12]) <= 2e-5 * np.linalg.norm(w1[:12])


def test_register_vec_with_normal_histograms_matches_oracle(sg, ctx):
    pr = config1()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    hX = ctx.descriptors_hn(rf, 16, 16)
    hY = ctx.descriptors_hn(tm, 16, 16)
    prm = O.Params(p=1.0, k=16, E=60)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=hX.cpu().numpy().astype(np.float64),
                     aY=hY.cpu().numpy().astype(np.float64))
    po, _, _ = O.register(pr.tmpl, S)
    pose, _ = ctx.register_vec(tm, hY, rf, hX, sg.Params(p=1.0, k=16, E=60))
    s, R, t = sg.pose_to_srt(pose)
    d = O.Pose(s, R, t).apply(pr.tmpl) - po.apply(pr.tmpl)
    err = np.sqrt(np.mean(np.sum(d * d, axis=1))) / O.diameter(pr.ref)
    gt = O.pose_rmse(po, pr.tmpl, pr.gt_s, pr.gt_R, pr.gt_t) / O.diameter(pr.ref)
    print(f"vector registration parity RMSE / diameter = {err:.2e} (oracle pose error {gt:.3f} D)")
    assert err <= 1e-4


def test_step_vec_full_size_sampled(sg, ctx):
    """The scan-sized pair (32 400 x 36 000) with 16-bin normal histograms:
    forces on sampled rows against the oracle."""
    pr = config2()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    hX = ctx.descriptors_hn(rf, 24, 16)
    hY = ctx.descriptors_hn(tm, 24, 16)
    gp = sg.Params(p=1.0, k=24, E=300)
    mt, mr = _dt(_mom(pr.tmpl), torch.float64), _dt(_mom(pr.ref), torch.float64)
    _, wr, f = ctx.step_vec(tm, hY, rf, hX, mt, mr, gp, 0, sg.pose_identity(), want_wrench=True, want_f=True)
    prm = O.Params(p=1.0, k=24, E=300)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=hX.cpu().numpy().astype(np.float64),
                     aY=hY.cpu().numpy().astype(np.float64))
    rows = np.random.default_rng(1).choice(pr.M, 256, replace=False)
    f_o, _ = O.forces(pr.tmpl.astype(np.float64), S, O.G_schedule(0, 300), rows=rows, block=32)
    sc = O.force_scale(pr.tmpl.astype(np.float64), S, O.G_schedule(0, 300), rows=rows, block=32)
    f = f.cpu().numpy().astype(np.float64)[rows]
    e = row_error(f, f_o, sc)
    print(f"full-size vector step: sampled force error {e:.1e}")
    assert e <= F_TOL


def _far_case(M, N, D, seed):
    """Clustered descriptors with 40 % of the template rows 30 spreads (of
    the clustered part) from the mean, in groups around 1 % of the
    reference descriptors (at most 240): more than 8 spreads after
    standardisation."""
    pr = random_pair(M, N, seed=seed)
    rng = np.random.default_rng(seed)
    cen = rng.random((6, D))
    aX = cen[rng.integers(0, 6, N)] + 0.05 * rng.normal(size=(N, D))
    aY = cen[rng.integers(0, 6, M)] + 0.05 * rng.normal(size=(M, D))
    sd0 = np.sqrt(np.mean(np.sum((aX - aX.mean(0)) ** 2, axis=1)))
    u = rng.normal(size=(240, D))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    hubs = aX.mean(0) + 30.0 * sd0 * u
    far = rng.choice(M, int(0.4 * M), replace=False)
    n_hub = max(1, min(240, N // 100))   # 1 % of the reference, so sigma stays near 3 sd0
    aX[:n_hub] = hubs[:n_hub] + 0.1 * sd0 * rng.normal(size=(n_hub, D))
    aY[far] = hubs[rng.integers(0, n_hub, len(far))] + 0.3 * sd0 * rng.normal(size=(len(far), D))
    aX, aY = aX.astype(np.float32), aY.astype(np.float32)
    mu = aX.astype(np.float64).mean(0)
    sig = np.sqrt(np.mean(np.sum((aX - mu) ** 2, axis=1)))
    n_far = int(np.sum(np.sum(((aY - mu) / sig) ** 2, axis=1) > 64.0))
    assert n_far > 0.35 * M, n_far
    return pr, aX, aY, far, n_far, rng


@pytest.mark.parametrize("D", [3, 5, 20])
def test_step_vec_many_far_rows_sampled(sg, ctx, D):
    """24 000 x 24 000 with 40% of the template rows far (_far_case): the
    far-row kernels run on about 150 row tiles with several staged chunks
    per reference segment and a ragged last segment (register prefetch for
    D = 3 and 5; descriptors padded to 4, 8 and 20 entries).  Sampled rows,
    most of them far, meet the per-point bar with the energy sum (wrench
    asked for) and without it."""
    M = N = 24000
    pr, aX, aY, far, n_far, rng = _far_case(M, N, D, 70 + D)
    prm = O.Params(p=1.0, k=16, E=40)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX.astype(np.float64), aY=aY.astype(np.float64))
    pose = O.Pose(1.05, rot_axis_angle([1, -1, 2], 10.0), np.array([0.02, -0.03, 0.01]))
    Y = pose.apply(pr.tmpl)
    rows = np.concatenate([rng.choice(far, 200, replace=False),
                           rng.choice(np.setdiff1d(np.arange(M), far), 56, replace=False)])
    t = 5
    G = O.G_schedule(t, prm.E)
    f_o, _ = O.forces(Y, S, G, rows=rows, block=32)
    sc = O.force_scale(Y, S, G, rows=rows, block=32)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    gp = sg.Params(p=1.0, k=16, E=40)
    mt, mr = _dt(_mom(pr.tmpl), torch.float64), _dt(_mom(pr.ref), torch.float64)
    for want_wrench in (True, False):
        _, _, f = ctx.step_vec(tm, _dt(aY), rf, _dt(aX), mt, mr, gp, t, sg.pose_from_srt(pose.s, pose.R, pose.t),
                               want_wrench=want_wrench, want_f=True)
        e = row_error(f.cpu().numpy().astype(np.float64)[rows], f_o, sc)
        print(f"many far rows D={D} ({n_far} far) wrench={want_wrench}: sampled force error {e:.1e}")
        assert e <= F_TOL


@pytest.mark.parametrize("flags", [0, 4])
def test_register_vec_far_rows_with_pose_independent_sums(sg, ctx, flags):
    """A registration whose template has 40 % far rows (_far_case, 3 000 x
    3 000, D = 5): with the pair sums formed once (flags bit 3; the far rows'
    sums from the far-row kernels) against the per-iteration kernels and
    against the oracle's registration, in both product forms."""
    pr, aX, aY, _, n_far, _ = _far_case(3000, 3000, 5, 90)
    prm = O.Params(p=1.0, k=16, E=20)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX.astype(np.float64), aY=aY.astype(np.float64))
    po, _, _ = O.register(pr.tmpl, S)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    poses = {}
    for f in (flags, flags | 8):
        pose, _ = ctx.register_vec(tm, _dt(aY), rf, _dt(aX), sg.Params(p=1.0, k=16, E=20, flags=f))
        s, R, t = sg.pose_to_srt(pose)
        poses[f] = O.Pose(s, R, t)
    D = O.diameter(pr.ref)

    def rmse(a, b):
        d = a.apply(pr.tmpl) - b.apply(pr.tmpl)
        return float(np.sqrt(np.mean(np.sum(d * d, axis=1)))) / D
    e_o, e_k = rmse(poses[flags | 8], po), rmse(poses[flags | 8], poses[flags])
    print(f"far rows ({n_far}), flags {flags}: pose-independent sums vs oracle {e_o:.1e} D, "
          f"vs per-iteration kernels {e_k:.1e} D (per-iteration vs oracle {rmse(poses[flags], po):.1e} D)")
    assert e_o <= 1e-4 and rmse(poses[flags], po) <= 1e-4
    assert e_k <= 1e-6


def test_vec_rejects_bad_arguments(sg, ctx):
    pr = random_pair(100, 120, seed=2)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    a_t, a_r = _dt(np.random.rand(100, 8)), _dt(np.random.rand(120, 8))
    for prm in (sg.Params(p=2.0, E=3), sg.Params(p=1.0, g_mode=1, E=3), sg.Params(p=1.0, E=3, flags=2)):
        with pytest.raises(sg.SgrError):
            ctx.register_vec(tm, a_t, rf, a_r, prm)
    with pytest.raises(sg.SgrError):
        ctx.register_vec(tm, _dt(np.random.rand(100, 31)), rf, _dt(np.random.rand(120, 31)), sg.Params(p=1.0, E=3))
    with pytest.raises(sg.SgrError):
        ctx.descriptors_hn(tm, 16, 1)
    with pytest.raises(sg.SgrError):   # zero descriptor spread
        ctx.register_vec(tm, _dt(np.ones((100, 8))), rf, _dt(np.ones((120, 8))), sg.Params(p=1.0, E=3))
