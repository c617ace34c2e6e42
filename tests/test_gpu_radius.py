"""Radius-neighbourhood curvature and the pyramidal schedule (Sec. IV)
against the oracle.  Member counts are integer decisions taken on the
float32 key, compared bit for bit.  The curvature is FP64 arithmetic rounded
once to float32: the GPU forms the covariance from moments about the query
point, the oracle from the members' coordinates centred at their mean, so
the two agree to about 1e-15 relative before the rounding.  They are
compared to one float32 ulp (rtol 2.4e-7), with 1e-12 absolute for values
that are 0."""
import numpy as np
import pytest
import torch

from oracle import ref as O
from synth import config1, config2
from synth.clouds import ellipsoid_patch

pytestmark = pytest.mark.gpu

A_RTOL, A_ATOL = 2.4e-7, 1e-12


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


def _check(sg, ctx, P, r2, rows=None):
    P = np.ascontiguousarray(P, np.float32)
    a, cnt = ctx.descriptors_radius(sg.Cloud(P), float(np.float32(r2)))
    a, cnt = a.cpu().numpy(), cnt.cpu().numpy()
    rows = np.arange(len(P)) if rows is None else rows
    a_o, c_o = O.radius_descriptors(P, np.float32(r2), rows)
    assert np.array_equal(cnt[rows], c_o.astype(np.int32)), "member counts differ"
    nan = np.isnan(a_o)
    assert np.array_equal(np.isnan(a[rows]), nan)
    np.testing.assert_allclose(a[rows][~nan], a_o[~nan].astype(np.float32), rtol=A_RTOL, atol=A_ATOL)
    return a, cnt


@pytest.mark.parametrize("scale", [0.08, 0.3, 1.0])
def test_radius_descriptors_match_oracle(sg, ctx, scale):
    P = ellipsoid_patch(3001, 5).astype(np.float32)      # 47 blocks of 64 queries, ragged tail
    lam = O.moments(P)[2]
    a, cnt = _check(sg, ctx, P, np.float32(scale * scale * lam))
    assert cnt.min() >= 1 and cnt.max() > 10


def test_radius_descriptors_edge_cases(sg, ctx):
    rng = np.random.default_rng(3)
    # a plane grid: every curvature is exactly 0
    g = np.stack(np.meshgrid(np.arange(30), np.arange(20)), -1).reshape(-1, 2).astype(np.float32)
    plane = np.concatenate([g, np.zeros((len(g), 1), np.float32)], axis=1)
    a, cnt = _check(sg, ctx, plane, 2.0)
    assert (a == 0).all() and cnt.max() == 9
    # duplicates, a NaN point, an inf point, r2 = 0 (self and exact duplicates only)
    P = rng.normal(size=(700, 3)).astype(np.float32)
    P[10:15] = P[3]
    P[20] = [np.nan, 0, 0]
    P[21] = [np.inf, 1, 1]
    _check(sg, ctx, P, 0.0)
    _check(sg, ctx, P, 0.5)
    # radius covering the whole cloud: every finite point sees every finite point
    a, cnt = _check(sg, ctx, P, 1e30)
    assert (cnt[np.isfinite(P).all(axis=1)] == 698).all()
    # fewer points than one block
    _check(sg, ctx, P[:37], 1.0)


def test_radius_descriptors_tile_skipping(sg, ctx):
    """Cases aimed at the tile test, which skips a tile of 64 Morton-ordered
    points when its box is farther than r from the box of a block's queries:
    it must never skip a member."""
    rng = np.random.default_rng(11)
    # offsets of 1e-30: every key underflows to 0 in float32, so with r2 = 0
    # every point is a member of every neighbourhood, across all 16 tiles
    T = (rng.normal(size=(1024, 3)) * 1e-30).astype(np.float32)
    a, cnt = _check(sg, ctx, T, 0.0)
    assert (cnt == 1024).all()
    # a second such cluster 1e-20 away: keys of about 1e-40 are subnormal,
    # not 0, so the clusters stay apart
    T2 = np.concatenate([T, (rng.normal(size=(600, 3)) * 1e-30 + 1e-20).astype(np.float32)])
    _, cnt = _check(sg, ctx, T2, 0.0)
    assert sorted(set(cnt.tolist())) == [600, 1024]
    # eight separated blobs: most tiles are skipped; r2 reaches across a
    # blob but not between blobs
    ctr = np.array([[i, j, k] for i in (0, 50) for j in (0, 50) for k in (0, 50)], np.float32)
    B = (ctr[rng.integers(0, 8, 4000)] + rng.normal(size=(4000, 3)) * 2.0).astype(np.float32)
    _check(sg, ctx, B, 4.0)
    _check(sg, ctx, B, 400.0)
    # an integer lattice with r2 = 1 and 2: many members lie exactly on the
    # threshold, in other tiles than their query
    g = np.stack(np.meshgrid(np.arange(16), np.arange(16), np.arange(8)), -1).reshape(-1, 3).astype(np.float32)
    for r2 in (1.0, 2.0):
        a, cnt = _check(sg, ctx, g[rng.permutation(len(g))], r2)
        assert cnt.max() == (7 if r2 == 1.0 else 19)


def test_radius_descriptors_two_list_passes(sg, ctx):
    """70 000 points = 1 094 tiles of 64: the per-block list of tiles within
    r is built in two passes of 1 024 tiles; sampled rows, including the
    first and last points of the Morton order's extremes."""
    P = ellipsoid_patch(70000, 9).astype(np.float32)
    lam = O.moments(P)[2]
    rows = np.concatenate([np.random.default_rng(2).choice(len(P), 60, replace=False),
                           [int(np.argmin(P[:, 0])), int(np.argmax(P[:, 0])), len(P) - 1]])
    a, cnt = _check(sg, ctx, P, np.float32(0.3 * 0.3 * lam), rows)
    assert cnt[rows].min() >= 1


def test_radius_descriptors_full_size_sampled(sg, ctx):
    """The scan-sized reference (36 000 points) with the paper's radius
    sqrt(lambda_max): sampled rows against the oracle."""
    pr = config2()
    lam = O.moments(pr.ref)[2]
    rows = np.random.default_rng(0).choice(pr.N, 60, replace=False)
    a, cnt = _check(sg, ctx, pr.ref, np.float32(lam), rows)
    print(f"radius sqrt(lambda_max) on 36 000 points: members {cnt.min()}..{cnt.max()}, mean {cnt.mean():.0f}")


def _levels(sg, spec):
    return [sg.Level(*v) for v in spec], [O.Level(*v) for v in spec]


@pytest.mark.parametrize("spec", [
    [(1.0, 1.0, 20), (0.5, 0.5, 20), (0.25, 0.3, 20)],
    [(0.0, 1.0, 25, 16), (0.4, 0.6, 35)]])
def test_register_pyramid_matches_oracle(sg, ctx, spec):
    pr = config1()
    lv_g, lv_o = _levels(sg, spec)
    E = sum(v[2] for v in spec)
    po = O.register_pyramid(pr.ref, pr.tmpl, O.Params(p=1.0, k=16, E=E), lv_o)
    pose, _ = ctx.register_pyramid(sg.Cloud(pr.tmpl), sg.Cloud(pr.ref), sg.Params(p=1.0, k=16, E=E), lv_g)
    s, R, t = sg.pose_to_srt(pose)
    d = O.Pose(s, R, t).apply(pr.tmpl) - po.apply(pr.tmpl)
    err = np.sqrt(np.mean(np.sum(d * d, axis=1))) / O.diameter(pr.ref)
    print(f"pyramid {spec}: parity RMSE / diameter = {err:.2e}")
    assert err <= 1e-4


def test_register_pyramid_one_knn_level_is_register(sg, ctx):
    """A single kNN level runs the same launches as register(): bit-identical
    poses and per-iteration statistics."""
    pr = config1(n=1500)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    prm = sg.Params(p=1.0, k=16, E=30)
    p1, s1 = ctx.register(tm, rf, prm, stats=True)
    p2, s2 = ctx.register_pyramid(tm, rf, prm, [sg.Level(0.0, 1.0, 30, 16)], stats=True)
    assert torch.equal(p1, p2) and torch.equal(s1, s2)


def test_pyramid_and_radius_reject_bad_arguments(sg, ctx):
    pr = config1(n=300)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    prm = sg.Params(p=1.0, k=16, E=10)
    for bad in ([sg.Level(1.0, 1.0, 9)],              # iterations do not add up to E
                [sg.Level(1.0, 0.0, 10)],             # sigma_scale must be > 0
                [sg.Level(-1.0, 1.0, 10)],            # negative radius
                [sg.Level(0.0, 1.0, 10, 0)],          # kNN level without k
                [sg.Level(1.0, 1.0, 10), sg.Level(1.0, 1.0, 0)],
                []):
        with pytest.raises(sg.SgrError):
            ctx.register_pyramid(tm, rf, prm, bad)
    for r2 in (-1.0, float("inf"), float("nan")):
        with pytest.raises(sg.SgrError):
            ctx.descriptors_radius(tm, r2)


def test_pyramid_graph_cache_follows_the_workspace_layout(sg):
    """One context and one pose buffer reused across pyramids whose levels
    differ only in the neighbourhood (k nearest with k = 16, a radius level,
    k = 8): the workspace layout differs between them while clouds,
    parameters and pose address do not, so a cached graph must not be
    replayed.  Each result equals a fresh context's, bit for bit."""
    pr = config1(n=1200)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    prm = sg.Params(p=1.0, k=16, E=30)
    schedules = [[sg.Level(0.0, 1.0, 30, 16)], [sg.Level(1.0, 1.0, 30)], [sg.Level(0.0, 1.0, 30, 8)]]
    shared = sg.Context(0)
    pose = sg.pose_identity()
    try:
        for lv in schedules:
            pose.copy_(sg.pose_identity())
            got, _ = shared.register_pyramid(tm, rf, prm, lv, pose=pose)
            fresh = sg.Context(0)
            try:
                want, _ = fresh.register_pyramid(tm, rf, prm, lv)
            finally:
                fresh.close()
            torch.cuda.synchronize()
            assert torch.equal(got, want), lv
    finally:
        shared.close()
