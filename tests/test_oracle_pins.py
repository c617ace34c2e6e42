"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics (not by the oracle itself): a hand-worked force, closed forms,
Newton's third law, the energy gradient, equivariance, descriptor
invariance and closed-form descriptors, Kabsch special cases and an
independent solver, scale idempotence, the G schedule, the fixed point and
exact recovery."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ref as O
from synth import config1, random_pair, rot_axis_angle
from synth.clouds import ellipsoid_patch

HERE = os.path.dirname(__file__)


def _setup(X, aX, aY, p=1.0, g_mode=0, sigma=0.2, eps=0.0, L=None, wX=None, mY=None):
    prm = O.Params(p=p, g_mode=g_mode, sigma=sigma, eps=eps)
    S = O.make_setup(X, np.zeros((len(aY), 3)), prm, aX=aX, aY=aY, wX=wX, mY=mY)
    if L is not None:
        S.L = L
    return S


# ------------------------------------------------------------ eqs. 3, 5, 10, 11
@pytest.mark.parametrize("mu", [0.0, 0.5, 0.9])
def test_velocity_state_closed_form(mu):
    """Eq. 5.5 with the template's previous velocity (and eq. 1's friction,
    mu = 1 - its share): with s = 1, p = 1 and unit masses the translation is
    d_t = -G_t dt2 (ybar_t - xbar) + mu d_(t-1) (d_(-1) = 0, the template
    starts at rest) and the centroid moves by d_t, whatever the rotation and
    scale do, so ybar - xbar follows a scalar recurrence per axis."""
    pr = random_pair(40, 60, seed=3)
    X, Y0 = pr.ref.astype(np.float64), pr.tmpl.astype(np.float64)
    rng = np.random.default_rng(0)
    prm = O.Params(p=1.0, sigma=1e30, E=20, momentum=mu)
    S = O.make_setup(X, Y0, prm, aX=rng.uniform(0, 0.3, 60), aY=rng.uniform(0, 0.3, 40))
    _, _, hist = O.register(Y0, S, keep=True)
    dt2 = 1.0 / prm.G1
    e, d_prev = Y0.mean(0) - X.mean(0), np.zeros(3)
    for t, so in enumerate(hist):
        d = -O.G_schedule(t, prm.E, prm.G1) * dt2 * e + mu * d_prev
        np.testing.assert_allclose(so.d, d, rtol=1e-9, atol=1e-12)
        e, d_prev = e + d, d
        np.testing.assert_allclose(so.Y.mean(0) - X.mean(0), e, rtol=1e-9, atol=1e-12)
    if mu > 0:   # the carried velocity changes the path, not only the last digits
        _, _, h0 = O.register(Y0, O.make_setup(X, Y0, O.Params(p=1.0, sigma=1e30, E=20), aX=S.aX, aY=S.aY), keep=True)
        assert np.abs(h0[5].d - hist[5].d).max() > 1e-6


def test_hand_worked_force():
    gold = json.load(open(os.path.join(HERE, "golden", "hand_force.json")))
    X = np.array(gold["reference"])
    Y = np.array(gold["template"])
    for case in gold["cases"]:
        S = _setup(X, np.array(gold["a_reference"]), np.array(gold["a_template"]), p=case["p"],
                   g_mode=case["g_mode"], sigma=gold["sigma"], L=gold["L"])
        for fn in (O.forces, O.forces_c):
            f, U = fn(Y, S, gold["G"])
            np.testing.assert_allclose(f[0], case["f"], rtol=1e-14, atol=1e-14)
            assert U == pytest.approx(case["U"], rel=1e-14)


def test_closed_form_uniform_similarity_p1():
    """p = 1, s = 1 (sigma -> inf), unit masses: f_i = -G (y_i - xbar),
    F = -G M (ybar - xbar), K = -G M Sigma_Y."""
    pr = random_pair(40, 60, seed=3)
    X, Y = pr.ref.astype(np.float64), pr.tmpl.astype(np.float64)
    rng = np.random.default_rng(0)
    S = _setup(X, rng.uniform(0, 0.3, 60), rng.uniform(0, 0.3, 40), p=1.0, sigma=1e30)
    G = 7.5
    f, _ = O.forces(Y, S, G)
    np.testing.assert_allclose(f, -G * (Y - X.mean(axis=0)), rtol=1e-12, atol=1e-12)
    so = O.step(Y, S, t=3)
    Gt = so.G
    M = len(Y)
    np.testing.assert_allclose(so.F, -Gt * M * (Y.mean(0) - X.mean(0)), rtol=1e-11)
    Yc = Y - Y.mean(0)
    np.testing.assert_allclose(so.K, -Gt * Yc.T @ Yc, rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("p", [1.0, 2.0, 3.0, 1.5])
@pytest.mark.parametrize("g_mode", [0, 1])
@pytest.mark.parametrize("eps", [0.0, 0.1])
def test_newton_third_law_self_registration(p, g_mode, eps):
    """Y = X with equal descriptors: the pair weights are symmetric and h r
    antisymmetric, so F = 0 and K = K^T exactly."""
    rng = np.random.default_rng(11)
    X = rng.normal(size=(50, 3))
    a = rng.uniform(0.0, 0.3, 50)
    S = _setup(X, a, a, p=p, g_mode=g_mode, sigma=0.07, eps=eps, L=0.8)
    f, _ = O.forces(X, S, 100.0)
    scale = np.abs(f).sum()
    F = f.sum(axis=0)
    K = f.T @ (X - X.mean(0))
    assert np.abs(F).max() <= 1e-13 * scale
    assert np.abs(K - K.T).max() <= 1e-13 * scale * np.abs(X).max()


def test_force_is_negative_energy_gradient():
    pr = random_pair(6, 30, seed=5)
    X = pr.ref.astype(np.float64)
    Y = pr.tmpl.astype(np.float64)
    rng = np.random.default_rng(1)
    for p, g_mode in ((2.0, 0), (1.0, 1), (3.0, 0)):
        S = _setup(X, rng.uniform(0.01, 0.3, 30), rng.uniform(0.01, 0.3, 6), p=p, g_mode=g_mode,
                   sigma=0.1, eps=0.05, L=0.9)
        f, _ = O.forces(Y, S, 3.0)
        h = 1e-6
        for i in range(6):
            for c in range(3):
                Yp, Ym = Y.copy(), Y.copy()
                Yp[i, c] += h
                Ym[i, c] -= h
                dU = (O.forces(Yp, S, 3.0)[1] - O.forces(Ym, S, 3.0)[1]) / (2 * h)
                assert -dU == pytest.approx(f[i, c], rel=1e-6, abs=1e-8)


def test_gravitational_mode_is_eq1_written_out():
    """g = 1, p = -2, eps > 0 is the softened inverse-square attraction of
    eq. (1): per unit template mass f_i = -G' sum_j m_j r_ij / (|r_ij|^2 +
    eps^2)^(3/2) with G' = G L^3 / Z, and U = -G' sum_ij m_j / sqrt(|r_ij|^2 +
    eps^2) (the Newtonian potential).  Written here with plain loops over
    pairs, without the oracle's normalised form."""
    pr = random_pair(9, 13, seed=21)
    X, Y = pr.ref.astype(np.float64), pr.tmpl.astype(np.float64)
    rng = np.random.default_rng(4)
    m = rng.uniform(0.5, 2.0, 13)
    eps, L, G = 0.07, 0.6, 2.5
    S = _setup(X, rng.uniform(0, 0.3, 13), rng.uniform(0, 0.3, 9), p=-2.0, g_mode=2, sigma=0.05, eps=eps, L=L,
               wX=m)
    Gp = G * L ** 3 / m.sum()
    f_ref = np.zeros((9, 3))
    U_ref = 0.0
    for i in range(9):
        for j in range(13):
            r = Y[i] - X[j]
            d2 = r @ r + eps * eps
            f_ref[i] -= Gp * m[j] * r / d2 ** 1.5
            U_ref -= Gp * m[j] / math.sqrt(d2)
    for fn in (O.forces, O.forces_c):
        f, U = fn(Y, S, G)
        np.testing.assert_allclose(f, f_ref, rtol=1e-12, atol=1e-14)
        assert U == pytest.approx(U_ref, rel=1e-12)
    # the shape term is gone: the descriptors do not enter
    S2 = _setup(X, rng.uniform(0, 0.3, 13), rng.uniform(0, 0.3, 9), p=-2.0, g_mode=2, sigma=0.05, eps=eps, L=L,
                wX=m)
    np.testing.assert_array_equal(O.forces(Y, S2, G)[0], O.forces(Y, S, G)[0])


def test_gravitational_mode_third_law_and_energy_gradient():
    rng = np.random.default_rng(12)
    X = rng.normal(size=(40, 3))
    a = rng.uniform(0.0, 0.3, 40)
    S = _setup(X, a, a, p=-2.0, g_mode=2, sigma=0.07, eps=0.1, L=0.8)
    f, _ = O.forces(X, S, 100.0)
    scale = np.abs(f).sum()
    assert np.abs(f.sum(axis=0)).max() <= 1e-13 * scale
    K = f.T @ (X - X.mean(0))
    assert np.abs(K - K.T).max() <= 1e-13 * scale * np.abs(X).max()
    Y = rng.normal(size=(5, 3))
    S = _setup(X, a, rng.uniform(0.0, 0.3, 5), p=-2.0, g_mode=2, sigma=0.07, eps=0.05, L=0.8)
    f, _ = O.forces(Y, S, 3.0)
    h = 1e-6
    for i in range(5):
        for c in range(3):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            dU = (O.forces(Yp, S, 3.0)[1] - O.forces(Ym, S, 3.0)[1]) / (2 * h)
            assert -dU == pytest.approx(f[i, c], rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("p,g_mode,eps", [(1.0, 0, 0.0), (2.0, 0, 0.05), (2.0, 1, 0.02), (1.5, 0, 0.1),
                                        (-2.0, 2, 0.05)])
def test_force_vjp_matches_central_differences(p, g_mode, eps):
    """The analytic FP64 adjoint against central differences of the force
    itself, in every coordinate, mass, sigma and eps."""
    pr = random_pair(9, 14, seed=19)
    rng = np.random.default_rng(23)
    X, Y = pr.ref.astype(np.float64), pr.tmpl.astype(np.float64)
    aX, aY = rng.uniform(0.01, 0.3, 14), rng.uniform(0.01, 0.3, 9)
    wX, m = rng.uniform(0.5, 2.0, 14), rng.uniform(0.5, 2.0, 9)
    gf, gF, gK = rng.normal(size=(9, 3)), rng.normal(size=3), rng.normal(size=(3, 3))
    sigma, G = 0.09, 3.0

    def L(Yv=Y, mv=m, sv=sigma, ev=eps):
        S = _setup(X, aX, aY, p=p, g_mode=g_mode, sigma=sv, eps=ev, L=0.8, wX=wX, mY=mv)
        f, _ = O.forces(Yv, S, G)
        return float(np.sum(gf * f) + gF @ (mv[:, None] * f).sum(0) + np.sum(gK * (f.T @ (Yv - Yv.mean(0)))))

    S = _setup(X, aX, aY, p=p, g_mode=g_mode, sigma=sigma, eps=eps, L=0.8, wX=wX, mY=m)
    gY, gm, gs, ge = O.force_vjp(Y, S, G, gf, gF, gK)
    h = 1e-6
    for i in range(9):
        for c in range(3):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            assert gY[i, c] == pytest.approx((L(Yv=Yp) - L(Yv=Ym)) / (2 * h), rel=1e-6, abs=1e-8)
        e = np.zeros(9)
        e[i] = h
        assert gm[i] == pytest.approx((L(mv=m + e) - L(mv=m - e)) / (2 * h), rel=1e-6, abs=1e-8)
    assert gs == pytest.approx((L(sv=sigma + h) - L(sv=sigma - h)) / (2 * h), rel=1e-6, abs=1e-8)
    if eps > 0:
        assert ge == pytest.approx((L(ev=eps + h) - L(ev=eps - h)) / (2 * h), rel=1e-6, abs=1e-8)
    if g_mode == 2:
        assert gs == 0.0


def test_force_equivariance():
    pr = random_pair(20, 35, seed=8)
    X = pr.ref.astype(np.float64)
    Y = pr.tmpl.astype(np.float64)
    rng = np.random.default_rng(2)
    aX, aY = rng.uniform(0, 0.3, 35), rng.uniform(0, 0.3, 20)
    S = _setup(X, aX, aY, p=2.0, sigma=0.1, eps=0.02, L=1.0)
    f, U = O.forces(Y, S, 5.0)
    t = np.array([3.0, -1.0, 2.5])
    Q = rot_axis_angle([0.2, -0.5, 1.0], 73.0)
    St = _setup(X + t, aX, aY, p=2.0, sigma=0.1, eps=0.02, L=1.0)
    ft, Ut = O.forces(Y + t, St, 5.0)
    np.testing.assert_allclose(ft, f, rtol=1e-10, atol=1e-10)
    Sq = _setup(X @ Q.T, aX, aY, p=2.0, sigma=0.1, eps=0.02, L=1.0)
    fq, Uq = O.forces(Y @ Q.T, Sq, 5.0)
    np.testing.assert_allclose(fq, f @ Q.T, rtol=1e-10, atol=1e-10)
    assert Ut == pytest.approx(U, rel=1e-12) and Uq == pytest.approx(U, rel=1e-12)


# ------------------------------------------------------------ descriptors
def test_knn_matches_bruteforce_and_c():
    P = ellipsoid_patch(5000, 4).astype(np.float32)
    q = np.arange(0, 5000, 7)
    a = O.knn_bruteforce(P, 16, q)
    b = O.knn(P, 16, q)
    c = O.knn_c(P, 16, q)
    assert (a == b).all() and (a == c).all()
    assert (a[:, 0] == q).all()                      # self first (distance 0)


def test_knn_tie_break_by_index():
    # a square lattice: many exactly equal float32 distances
    g = np.stack(np.meshgrid(np.arange(6), np.arange(6), [0.0]), -1).reshape(-1, 3).astype(np.float32)
    nb = O.knn_bruteforce(g, 5)
    # the centre-ish point 14 = (2,2): neighbours at distance 1 are 8, 13, 15, 20
    i = 2 * 6 + 2
    assert list(nb[i]) == [i, i - 6, i - 1, i + 1, i + 6]
    assert (O.knn_c(g, 5) == nb).all()


def test_descriptor_closed_form_box_corners():
    """k = n = 8 box corners with half-sides (1, 2, 3): every neighbourhood
    is the whole cloud, covariance diag(1, 4, 9), so a = 1/14."""
    c = np.array([[x, y, z] for x in (-1, 1) for y in (-2, 2) for z in (-3, 3)], dtype=np.float32)
    a = O.descriptors(c, 8)
    np.testing.assert_allclose(a, 1.0 / 14.0, rtol=1e-14)


def test_descriptor_plane_is_zero():
    rng = np.random.default_rng(3)
    P = np.stack([rng.uniform(-1, 1, 300), rng.uniform(-1, 1, 300), np.full(300, -0.4)], 1).astype(np.float32)
    assert np.abs(O.descriptors(P, 16)).max() == 0.0


def test_descriptor_invariance():
    """a is invariant under rotation, translation and uniform scale; checked
    where the float32 neighbour sets agree (they may differ at near-ties)."""
    P = ellipsoid_patch(1500, 9).astype(np.float32)
    Q = rot_axis_angle([1.0, 2.0, -0.5], 37.0)
    P2 = (1.7 * P.astype(np.float64) @ Q.T + np.array([0.3, -2.0, 5.0])).astype(np.float32)
    n1, n2 = O.knn(P, 16), O.knn(P2, 16)
    same = np.array([set(a) == set(b) for a, b in zip(n1, n2)])
    assert same.mean() > 0.95
    a1 = O.surface_variation(P, n1)
    a2 = O.surface_variation(P2, n2)
    np.testing.assert_allclose(a1[same], a2[same], rtol=0, atol=2e-6)


# ------------------------------------------------------------ Kabsch, scale
def _horn_rotation(A, B):
    """Rotation R (row convention) minimising |A R - B| by Horn's unit
    quaternion method (an independent closed-form solver)."""
    S = A.T @ B
    Sxx, Sxy, Sxz = S[0]
    Syx, Syy, Syz = S[1]
    Szx, Szy, Szz = S[2]
    N = np.array([
        [Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx],
        [Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz],
        [Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy],
        [Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz]])
    w, v = np.linalg.eigh(N)
    q = v[:, -1]
    from synth.clouds import quat_to_R
    return quat_to_R(q).T        # column rotation of B ~ R_col A -> row form R_col^T


# ------------------------------------------------------------ radius neighbourhoods
def test_radius_descriptor_box_corners_closed_form():
    """The 8 corners of a box with half-sides (3, 2, 1), radius covering all:
    covariance diag(9, 4, 1), so every a = 1/14."""
    P = np.array([[sx * 3.0, sy * 2.0, sz * 1.0] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                 np.float32) + np.float32([5, -7, 2])
    a, cnt = O.radius_descriptors(P, 100.0)
    assert (cnt == 8).all()
    np.testing.assert_allclose(a, 1.0 / 14.0, rtol=1e-14)


def test_radius_membership_is_inclusive_and_counts_self():
    P = np.zeros((10, 3), np.float32)
    P[:, 0] = np.arange(10)
    a, cnt = O.radius_descriptors(P, 1.0)           # key 1.0 <= 1.0: both lattice neighbours
    assert list(cnt) == [2] + [3] * 8 + [2]
    assert (a == 0.0).all()                          # collinear: lambda_0 = lambda_1 = 0
    a, cnt = O.radius_descriptors(P, np.nextafter(np.float32(1.0), np.float32(0)))
    assert (cnt == 1).all() and (a == 0.0).all()     # self only: trace 0
    Q = np.concatenate([P, P[3:4], [[np.nan, 0, 0]]]).astype(np.float32)
    a, cnt = O.radius_descriptors(Q, 0.0)
    assert cnt[3] == 2 and cnt[10] == 2 and cnt[0] == 1
    assert cnt[11] == 0 and np.isnan(a[11])          # a non-finite query has no neighbourhood
    assert not np.isnan(a[:11]).any()


def test_radius_equals_knn_when_the_radius_isolates_k_points():
    """With r2 set to the float32 key of a point's k-th neighbour (no tie),
    the radius neighbourhood is the kNN neighbourhood, whose curvature is
    pinned separately."""
    P = ellipsoid_patch(3000, 7).astype(np.float32)
    q = np.arange(0, 3000, 37)
    nb = O.knn_bruteforce(P, 16, q)
    for r, i in enumerate(q):
        d = O.sqdist32(P[nb[r]], P[i])
        a, cnt = O.radius_descriptors(P, d.max(), [i])
        assert cnt[0] == 16
        assert a[0] == pytest.approx(O.surface_variation(P, nb[r:r + 1])[0], rel=1e-11, abs=1e-15)


def test_radius_tree_path_matches_brute_force():
    """Clouds above 4096 points take k-d tree candidates; membership and
    curvature equal a brute-force scan of every point."""
    P = ellipsoid_patch(6000, 9).astype(np.float32)
    P[17] = np.nan
    lam = O.moments(P[np.isfinite(P).all(axis=1)])[2]
    q = np.arange(0, 6000, 151)
    for scale in (0.05, 0.4):
        r2 = np.float32(scale * scale * lam)
        a, cnt = O.radius_descriptors(P, r2, q)
        for r, i in enumerate(q):
            mem = np.flatnonzero(O.sqdist32(P, P[i]) <= r2)
            assert cnt[r] == len(mem)
            Q = P[mem].astype(np.float64)
            lam3 = np.linalg.eigvalsh(np.cov(Q.T, bias=True).reshape(3, 3))
            want = lam3[0] / lam3.sum() if lam3.sum() > 0 else 0.0
            assert a[r] == pytest.approx(want, rel=1e-10, abs=1e-14)
        assert (cnt > 1).mean() > 0.5


def test_pyramid_split_level_equals_one_level_and_checks_E():
    """t runs on across levels: two identical levels of 7 + 5 iterations are
    one level of 12 (up to the rounding of re-posing the template from the
    pose at the level boundary; restarting t would move G and the pose by
    far more)."""
    pr = config1(n=500)
    prm = O.Params(p=1.0, k=16, E=12)
    one = O.register_pyramid(pr.ref, pr.tmpl, prm, [O.Level(0.3, 0.7, 12)])
    two = O.register_pyramid(pr.ref, pr.tmpl, prm, [O.Level(0.3, 0.7, 7), O.Level(0.3, 0.7, 5)])
    np.testing.assert_allclose(two.as_array(), one.as_array(), rtol=0, atol=1e-13)
    lev = O.Level(0.3, 0.7, 7)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=O.level_descriptors(pr.ref, lev), aY=O.level_descriptors(pr.tmpl, lev))
    S.sigma *= lev.sigma_scale
    mid, _, _ = O.register(pr.tmpl, S, E=7)
    restart, _, _ = O.register(pr.tmpl, S, E=5, pose0=mid, t0=0)
    assert np.abs(restart.as_array() - two.as_array()).max() > 1e-6
    knn = O.register_pyramid(pr.ref, pr.tmpl, prm, [O.Level(0.0, 1.0, 12, k=16)])
    S = O.make_setup(pr.ref, pr.tmpl, prm)
    ref_pose, _, _ = O.register(pr.tmpl, S)
    np.testing.assert_array_equal(knn.as_array(), ref_pose.as_array())
    with pytest.raises(ValueError):
        O.register_pyramid(pr.ref, pr.tmpl, prm, [O.Level(0.3, 1.0, 11)])


# ------------------------------------------------------------ vector descriptors
def test_tent_weights_by_hand_and_partition_of_unity():
    w = O.tent_weights(np.array([0.0, 0.25, 0.5, 0.8, 1.0]), 3)      # centres 0, 0.5, 1
    np.testing.assert_allclose(w, [[1, 0, 0], [0.5, 0.5, 0], [0, 1, 0], [0, 0.4, 0.6], [0, 0, 1]], atol=1e-15)
    u = np.random.default_rng(2).random(1000)
    for D in (2, 5, 16, 30):
        np.testing.assert_allclose(O.tent_weights(u, D).sum(axis=1), 1.0, rtol=1e-14)


def test_normal_histograms_planes_and_crease():
    """On a plane every normal is the same, so every h is the last unit
    vector; on two perpendicular half-planes, points whose neighbourhoods do
    not reach the crease have the same, and points at the crease, whose
    normals tilt towards the bisector, spread their weight below the last
    bin."""
    g = np.stack(np.meshgrid(np.arange(20), np.arange(20)), -1).reshape(-1, 2).astype(np.float64) * 0.1
    plane = np.concatenate([g, np.zeros((len(g), 1))], axis=1)
    rng = np.random.default_rng(3)
    plane = plane @ O.Pose(1.0, rot_axis_angle([1, 2, 3], 40.0), np.zeros(3)).R.T + 2.0
    h, _ = O.normal_histograms(plane.astype(np.float32), 8, 16)
    np.testing.assert_allclose(h[:, -1], 1.0, atol=1e-6)
    np.testing.assert_allclose(h[:, :-1], 0.0, atol=1e-6)
    a = np.concatenate([g[:, :1] * 0 + g[:, :1], g[:, 1:], np.zeros((len(g), 1))], axis=1)    # z = 0, x >= 0
    b = np.concatenate([-np.ones((len(g), 1)) * 0.05 - g[:, :1] * 0, g[:, 1:], g[:, :1] + 0.05], axis=1)  # x = -0.05
    P = np.concatenate([a, b]).astype(np.float32)
    h, lam = O.normal_histograms(P, 8, 16)
    far = (P[:, 0] > 0.45) | (P[:, 2] > 0.45)
    np.testing.assert_allclose(h[far, -1], 1.0, atol=1e-6)
    near = (P[:, 0] < 0.05) & (P[:, 2] < 0.01)
    assert near.sum() == 20 and (h[near, -1] < 0.9).all()
    np.testing.assert_allclose(h.sum(axis=1), 1.0, rtol=1e-12)


def test_normal_histograms_invariance():
    P = ellipsoid_patch(3000, 11).astype(np.float64)
    q = np.arange(0, 3000, 29)
    h, lam = O.normal_histograms(P.astype(np.float32), 16, 16, q)
    T = (2.5 * P @ rot_axis_angle([0.3, -1, 0.5], 77.0).T + np.array([4.0, -2.0, 1.0])).astype(np.float32)
    h2, lam2 = O.normal_histograms(T, 16, 16, q)
    ok = (lam[:, 1] - lam[:, 0]) > 1e-3 * lam.sum(axis=1)     # normal determined
    assert ok.mean() > 0.9
    np.testing.assert_allclose(h2[ok], h[ok], atol=2e-4)      # float32 inputs: neighbours may move slightly


def test_vector_similarity_reduces_to_scalar_and_is_permutation_invariant():
    """D = 1 vector descriptors give the scalar force (eq. 3), and the force
    does not depend on the order of the descriptor dimensions."""
    pr = random_pair(30, 45, seed=14)
    rng = np.random.default_rng(8)
    aX, aY = rng.uniform(0, 0.3, 45), rng.uniform(0, 0.3, 30)
    S1 = _setup(pr.ref.astype(np.float64), aX, aY, p=1.0, sigma=0.0, L=0.8)
    Sv = _setup(pr.ref.astype(np.float64), aX[:, None], aY[:, None], p=1.0, sigma=0.0, L=0.8)
    assert Sv.sigma == pytest.approx(S1.sigma, rel=1e-14)
    f1, U1 = O.forces(pr.tmpl, S1, 3.0)
    fv, Uv = O.forces(pr.tmpl, Sv, 3.0)
    np.testing.assert_allclose(fv, f1, rtol=1e-13, atol=1e-15)
    AX, AY = rng.random((45, 16)), rng.random((30, 16))
    perm = rng.permutation(16)
    Sa = _setup(pr.ref.astype(np.float64), AX, AY, p=2.0, sigma=0.0, eps=0.01, L=0.8)
    Sb = _setup(pr.ref.astype(np.float64), AX[:, perm], AY[:, perm], p=2.0, sigma=0.0, eps=0.01, L=0.8)
    np.testing.assert_allclose(O.forces(pr.tmpl, Sb, 3.0)[0], O.forces(pr.tmpl, Sa, 3.0)[0], rtol=1e-12)
    with pytest.raises(ValueError):
        _setup(pr.ref.astype(np.float64), AX, AY, g_mode=1)


def test_kabsch_pure_rotation_and_spd():
    rng = np.random.default_rng(4)
    Y = rng.normal(size=(30, 3)) * [1.0, 0.5, 0.2]
    Y -= Y.mean(0)
    Q = rot_axis_angle([0.3, -1.0, 0.4], 63.0)       # column rotation
    R, _ = O.kabsch(Y, Y @ Q.T)                      # Y_D = Y Q^T, rows rotated by Q
    np.testing.assert_allclose(R, Q.T, atol=1e-12)  # Y R = Y_D
    R2, _ = O.kabsch(Y, 0.5 * Y)                      # C symmetric positive definite
    np.testing.assert_allclose(R2, np.eye(3), atol=1e-12)


def test_kabsch_matches_horn():
    rng = np.random.default_rng(6)
    for _ in range(5):
        A = rng.normal(size=(40, 3))
        A -= A.mean(0)
        B = A @ rot_axis_angle(rng.normal(size=3), rng.uniform(0, 170)) + 0.1 * rng.normal(size=(40, 3))
        B -= B.mean(0)
        R, _ = O.kabsch(A, B)
        np.testing.assert_allclose(R, _horn_rotation(A, B), atol=1e-10)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)


def test_scale_is_idempotent():
    pr = config1(n=400)
    S = O.make_setup(pr.ref, pr.tmpl, O.Params(k=16, E=10))
    so = O.step(pr.tmpl.astype(np.float64), S, 0)
    assert so.c == pytest.approx(1 / 1.2, rel=2e-3)
    assert O.moments(so.Y)[2] == pytest.approx(S.lamX, rel=1e-12)
    so2 = O.step(so.Y, S, 1)
    assert so2.c == pytest.approx(1.0, abs=1e-12)


# ------------------------------------------------------------ eq. 12
def test_G_schedule_closed_form():
    G1, E = 10000.0, 100
    assert O.G_schedule(0, E, G1) == pytest.approx(1000.0 + 9000.0 / (1 + math.exp(51)), rel=1e-15)
    assert O.G_schedule(51, E, G1) == 5500.0
    assert O.G_schedule(100, E, G1) == pytest.approx(10000.0, rel=1e-10)
    g = [O.G_schedule(t, E, G1) for t in range(E)]
    assert all(b >= a for a, b in zip(g, g[1:])) and g[60] > g[40]


# ------------------------------------------------------------ whole iteration
def test_true_alignment_is_fixed_point():
    pr = config1(n=600, noise=0.0)
    X = pr.ref
    for p in (1.0, 2.0):
        S = O.make_setup(X, X, O.Params(p=p, k=16, E=20))
        so = O.step(X.astype(np.float64), S, 5)
        np.testing.assert_allclose(so.Y, X.astype(np.float64), atol=1e-12)
        np.testing.assert_allclose(so.R, np.eye(3), atol=1e-13)
        assert so.c == pytest.approx(1.0, abs=1e-13)


def test_exact_recovery_translation_scale_symmetric_cloud():
    """Noise-free, centrally symmetric cloud, template = 1.3 x + t: the
    torque vanishes by symmetry and the translation/scale are recovered."""
    P = ellipsoid_patch(256, 77)
    X = np.concatenate([P, -P]).astype(np.float32)
    s, t = 1.3, np.array([0.4, -0.3, 0.2])
    Y0 = (s * X.astype(np.float64) + t).astype(np.float32)
    S = O.make_setup(X, Y0, O.Params(p=1.0, k=16, E=100))
    S.aY = S.aX.copy()                              # pose-invariant descriptors
    pose, Y, _ = O.register(Y0, S)
    assert O.pose_rmse(pose, Y0, s, np.eye(3), t) <= 1e-9 * O.diameter(X)


def test_pose_composition_matches_point_update():
    pr = config1(n=300)
    S = O.make_setup(pr.ref, pr.tmpl, O.Params(k=16, E=15))
    pose, Y, _ = O.register(pr.tmpl, S)
    np.testing.assert_allclose(pose.apply(pr.tmpl), Y, atol=1e-11)
    assert np.allclose(pose.R @ pose.R.T, np.eye(3), atol=1e-12)


def test_c_oracle_matches_numpy():
    pr = random_pair(70, 90, seed=12)
    rng = np.random.default_rng(9)
    for p, g_mode, eps in ((1.0, 0, 0.0), (2.0, 1, 0.03), (3.0, 0, 0.0), (2.5, 0, 0.1), (-2.0, 2, 0.05)):
        S = _setup(pr.ref.astype(np.float64), rng.uniform(0.01, 0.3, 90), rng.uniform(0.01, 0.3, 70),
                   p=p, g_mode=g_mode, sigma=0.08, eps=eps, L=0.7, wX=rng.uniform(0.5, 2, 90))
        f1, U1 = O.forces(pr.tmpl, S, 42.0)
        f2, U2 = O.forces_c(pr.tmpl, S, 42.0)
        np.testing.assert_allclose(f2, f1, rtol=1e-12, atol=1e-12 * np.abs(f1).max())
        assert U2 == pytest.approx(U1, rel=1e-12)


def test_residual_closed_forms():
    """RMSE with correspondences of a cloud shifted by a known vector is the
    shift length; the one-sided NN RMSE of a cloud against itself is 0 and
    against a copy shifted by a tenth of the smallest point spacing is that
    shift; pose_rmse of the generating transform's inverse is 0."""
    rng = np.random.default_rng(13)
    X = rng.normal(size=(200, 3))
    d = np.array([0.3, -0.4, 1.2])
    ident = O.Pose.identity()
    assert O.residual_corr(ident, X + d, X, np.arange(200)) == pytest.approx(np.linalg.norm(d), rel=1e-14)
    corr = np.arange(200)
    corr[::2] = -1                                   # half without counterpart
    assert O.residual_corr(ident, X + d, X, corr) == pytest.approx(np.linalg.norm(d), rel=1e-14)
    assert O.residual_nn(ident, X, X) == 0.0
    from scipy.spatial.distance import pdist
    h = 0.1 * pdist(X).min()
    e = np.array([1.0, 2.0, 2.0]) / 3.0
    assert O.residual_nn(ident, X + h * e, X) == pytest.approx(h, rel=1e-12)
    R = rot_axis_angle([1, 1, 0], 33.0)
    s, t = 1.3, np.array([0.5, 0.1, -2.0])
    Y = s * X @ R.T + t
    inv = O.Pose(1 / s, R.T, -(R.T @ t) / s)
    assert O.pose_rmse(inv, Y, s, R, t) <= 1e-14 * np.abs(X).max()


# ------------------------------------------------------ change detection
def test_nearest_matches_brute_force_with_ties_and_far_queries():
    """The k-d tree path of the nearest-point search returns what a brute
    force over all points returns (float32 key, ties by lowest index): with
    exactly duplicated reference points, lattice queries equidistant from
    several points, and queries far outside the cloud."""
    rng = np.random.default_rng(21)
    X = rng.normal(size=(3000, 3)).astype(np.float32)
    X[100:110] = X[50]                                 # exact duplicates of point 50
    L = np.array([[i, j, k] for i in range(4) for j in range(4) for k in range(4)], np.float32)
    X = np.concatenate([X, L])                          # a unit lattice: midpoint queries tie
    Q = np.concatenate([rng.normal(size=(500, 3)), X[[50, 7, 3001]], L[:20] + 0.5,
                        rng.normal(size=(20, 3)) * 50.0]).astype(np.float32)
    nn, key = O.nearest(Q, X)
    idx = np.arange(len(X))
    for i in range(len(Q)):
        d = O.sqdist32(X, Q[i])
        j = int(np.lexsort((idx, d))[0])
        assert nn[i] == j and key[i] == d[j]
    assert nn[500] == 50                               # duplicate: lowest index wins
    bad = np.array([[np.nan, 0, 0]], np.float32)
    nb, kb = O.nearest(bad, X)
    assert nb[0] == -1 and np.isinf(kb[0])


def test_posed32_closed_form():
    """A quarter turn about z with scale 2 and an integer shift maps integer
    points to exactly known float32 values."""
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    pose = O.Pose(2.0, R, np.array([1.0, -3.0, 0.5]))
    Y = np.array([[1, 2, 3], [-4, 0, 7]], np.float32)
    want = np.array([[2 * -2 + 1, 2 * 1 - 3, 2 * 3 + 0.5], [2 * 0 + 1, 2 * -4 - 3, 2 * 7 + 0.5]], np.float32)
    np.testing.assert_array_equal(O.posed32(Y, pose), want)


def test_change_flags_self_pair_added_object_and_shape_change():
    """Against itself at the identity pose nothing is flagged; a cluster
    placed far from the reference is flagged by distance only; shifting
    some curvatures by more (less) than sigma sqrt(-ln s_min) sets (does not
    set) the shape bit."""
    rng = np.random.default_rng(22)
    X = rng.normal(size=(2000, 3)).astype(np.float32)
    aX = rng.uniform(0.0, 0.2, 2000).astype(np.float32)
    ident = O.Pose.identity()
    sigma, s_min, tau = 0.05, 0.5, 0.05
    f, nn, key = O.change_flags(X, aX, X, aX, ident, tau, sigma, s_min)
    assert not f.any() and (key == 0).all()
    blob = (rng.normal(size=(100, 3)) * 0.1 + np.array([10.0, 0.0, 0.0])).astype(np.float32)
    Y = np.concatenate([X, blob])
    aY = np.concatenate([aX, np.full(100, 0.1, np.float32)])
    f, nn, key = O.change_flags(Y, aY, X, aX, ident, tau, sigma, s_min)
    assert not f[:2000].any() and (f[2000:] & 1).all()
    thr = sigma * np.sqrt(-np.log(s_min))
    aY2 = aX.copy()
    aY2[:50] += np.float32(1.5 * thr)
    aY2[50:100] += np.float32(0.5 * thr)
    f, nn, key = O.change_flags(X, aY2, X, aX, ident, tau, sigma, s_min)
    assert (f[:50] == 2).all() and not f[50:].any()
    f, _, _ = O.change_flags(X, aY2, X, aX, ident, tau, sigma, 0.0)   # shape test off
    assert not f.any()


# ------------------------------------------------- local polynomial descriptor
def _quadric_grid(a, b, c, n=7):
    g = np.array([[x, y] for x in np.linspace(-1, 1, n) for y in np.linspace(-1, 1, n)])
    return np.column_stack([g[:, 0], g[:, 1], a * g[:, 0] ** 2 + b * g[:, 0] * g[:, 1] + c * g[:, 1] ** 2])


def _rho(Q):
    qc = Q - Q.mean(axis=0)
    return np.sqrt(np.mean(np.sum(qc * qc, axis=1)))


@pytest.mark.parametrize("a,b,c", [(0.05, 0.0, -0.02), (0.03, 0.0, 0.03), (-0.04, 0.0, -0.01), (0.02, 0.0, -0.05)])
def test_poly_fit_exact_quadric(a, b, c):
    """Points exactly on h = a u^2 + c v^2 over a grid symmetric in u and v:
    the covariance frame is the (u, v, h) frame, the fit is exact, and the
    descriptor is the Hessian's eigenvalues 2 a rho and 2 c rho, sorted, with
    both negated and swapped when their sum is negative; residual 0."""
    Q = _quadric_grid(a, b, c)
    rho = _rho(Q)
    mu = np.sort([2 * a * rho, 2 * c * rho])[::-1]
    if mu.sum() < 0:
        mu = -mu[::-1]
    d = O.poly_fit(Q)
    np.testing.assert_allclose(d[:2], mu, rtol=1e-12, atol=1e-14)
    assert d[2] < 1e-14


def test_poly_fit_plane_and_degenerate():
    g = _quadric_grid(0.0, 0.0, 0.0)
    np.testing.assert_allclose(O.poly_fit(g), 0.0, atol=1e-14)
    assert np.isnan(O.poly_fit(np.ones((8, 3)))).all()


def test_poly_fit_sphere_cap_is_umbilic_and_convex():
    """A cap of a sphere sampled symmetrically under a quarter turn about its
    axis: mu1 = mu2 (an umbilic), positive by the sign convention, close to
    rho / R."""
    R = 3.0
    g = _quadric_grid(0.0, 0.0, 0.0, n=9)[:, :2] * 0.4
    Q = np.column_stack([g, np.sqrt(R * R - np.sum(g * g, axis=1))])
    d = O.poly_fit(Q)
    assert d[0] == pytest.approx(d[1], rel=1e-9)
    assert d[0] > 0
    assert d[0] == pytest.approx(_rho(Q) / R, rel=2e-2)


def test_poly_fit_residual_of_a_cubic():
    """h = u^3 is not in the fitted space: the residual is the RMS of the
    part of u^3 orthogonal to {1, u, v, u^2, u v, v^2} over the samples."""
    g = _quadric_grid(0.0, 0.0, 0.0, n=9)[:, :2]
    Q = np.column_stack([g, 0.05 * g[:, 0] ** 3])
    d = O.poly_fit(Q)
    qc = Q - Q.mean(axis=0)
    lam, vec = np.linalg.eigh(qc.T @ qc / len(Q))
    rho = np.sqrt(lam.sum())
    u, v, h = qc @ vec[:, 2] / rho, qc @ vec[:, 1] / rho, qc @ vec[:, 0] / rho
    A = np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], axis=1)
    resid = h - A @ np.linalg.pinv(A) @ h             # projection residual, another route
    assert d[2] == pytest.approx(np.sqrt(np.mean(resid ** 2)), rel=1e-9)
    assert d[2] > 1e-4


def test_poly_fit_invariances():
    rng = np.random.default_rng(4)
    base = _quadric_grid(0.08, 0.03, -0.05, n=5) + rng.normal(0, 0.01, (25, 3))
    d0 = O.poly_fit(base)
    Rm = rot_axis_angle([1.0, -2.0, 0.5], 73.0)
    t = np.array([3.0, -1.0, 2.0])
    for Q in (base @ Rm.T + t,                        # rotation + translation
              2.7 * base,                             # uniform scale
              base * np.array([1.0, 1.0, -1.0]),      # reflection of the normal axis
              base * np.array([-1.0, 1.0, 1.0]),      # reflection of a tangent axis
              base[rng.permutation(len(base))],       # order of the neighbours
              base @ rot_axis_angle([0.0, 0.0, 1.0], 30.0).T):   # rotation of the tangent frame
        np.testing.assert_allclose(O.poly_fit(Q), d0, rtol=1e-9, atol=1e-12)


# ------------------------------------------- Sec. III-B moments, set-up defaults
def _box_corners(hx, hy, hz):
    return np.array([[sx * hx, sy * hy, sz * hz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)


def test_moments_box_corners():
    """The 8 corners (+-1, +-2, +-3): centroid 0 and, with the 1/n
    normalisation, covariance diag(1, 4, 9) exactly, whose LARGEST eigenvalue
    (eX of Sec. III-B) is 9.  Fails for eigvalsh()[0] (gives 1), for a
    1/(n-1) covariance (9 * 8/7) and for a centroid that is not subtracted."""
    X = _box_corners(1.0, 2.0, 3.0) + 0.0
    c, S, lam = O.moments(X)
    np.testing.assert_array_equal(c, np.zeros(3))
    np.testing.assert_array_equal(S, np.diag([1.0, 4.0, 9.0]))
    assert lam == 9.0
    c2, S2, lam2 = O.moments(X + np.array([5.0, -1.0, 0.5]))
    np.testing.assert_allclose(c2, [5.0, -1.0, 0.5], atol=1e-15)
    assert lam2 == pytest.approx(9.0, rel=1e-14)


def test_step_scale_is_sqrt_of_largest_eigenvalue_ratio():
    """Eq. 8 as read: c = sqrt(lambda_max(Sigma_X) / lambda_max(Sigma_Y)),
    both covariances 1/count.  Reference: the 8 corners (+-1, +-2, +-3)
    (lambda_max 9, lambda_min 1); template: the corners stretched 5x along x,
    each taken twice (16 points; lambda_max 25, lambda_min 4).  c = 0.6
    exactly.  The smallest eigenvalues would give 0.5; 1/(n-1) covariances,
    with n = 8 and 16, would give sqrt((72/7) / (400/15)) = 0.621."""
    X = _box_corners(1.0, 2.0, 3.0)
    Y = np.concatenate([_box_corners(5.0, 2.0, 3.0)] * 2)
    rng = np.random.default_rng(2)
    S = O.make_setup(X, Y, O.Params(p=1.0, E=10), aX=np.array([0.1, 0.3] * 4), aY=rng.uniform(0.1, 0.3, 16))
    so = O.step(Y, S, 0)
    assert so.c == pytest.approx(0.6, rel=1e-13)
    assert abs(so.c - 0.5) > 0.05 and abs(so.c - math.sqrt((72 / 7) / (400 / 15))) > 0.01


def test_setup_defaults_and_p2_force_by_hand():
    """Defaults of make_setup written out by hand.  Reference x1 = (-2, 0, 0),
    x2 = (2, 0, 0) with curvatures 0.1, 0.3: abar = 0.2, sigma = population
    std = 0.1 (the sample std would be 0.1414), lambda_max = 4 and L =
    sqrt(lambda_max) = 2 (L = lambda_max would be 4; a 1/(n-1) covariance
    2 sqrt(2); lambda_min = 0 would make the p = 2 law infinite).  Template
    point y = (0, 1, 0) with a = 0.2: s_1 = s_2 = exp(-(0.1/0.1)^2) = 1/e,
    r_1 = (2, 1, 0), r_2 = (-2, 1, 0), |r| = sqrt(5), and for p = 2, eps = 0
    the distance factor (|r|^2 / L^2)^(1/2) = sqrt(5)/2.  With G = 1, Z = 2:
      g = s:      f = -(1/2)(sqrt(5)/2)(1/e)(r_1 + r_2) = (0, -sqrt(5)/(2e), 0)
      g = a a s:  weights (a_j/abar) = 1/2, 3/2:
                  f = -(1/2)(sqrt(5)/2)(1/e)(r_1/2 + 3 r_2/2) = (sqrt(5)/(2e), -sqrt(5)/(2e), 0)
    Neither sigma nor L is overridden."""
    X = np.array([[-2.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    aX = np.array([0.1, 0.3])
    Y = np.array([[0.0, 1.0, 0.0]])
    v = math.sqrt(5.0) / (2.0 * math.e)
    for g_mode, want in ((0, [0.0, -v, 0.0]), (1, [v, -v, 0.0])):
        S = O.make_setup(X, Y, O.Params(p=2.0, g_mode=g_mode), aX=aX, aY=np.array([0.2]))
        assert S.sigma == pytest.approx(0.1, rel=1e-14)
        assert S.abar == pytest.approx(0.2, rel=1e-15)
        assert S.lamX == 4.0 and S.L == 2.0
        for fn in (O.forces, O.forces_c):
            f, _ = fn(Y, S, 1.0)
            np.testing.assert_allclose(f[0], want, rtol=1e-14, atol=1e-15)


def _labelled_pair(n=40, seed=8):
    """A 3-D cloud whose points carry distinct labels (curvatures 0.01 i),
    with a similarity spread that couples every template point to its own
    counterpart only (other pairs: exp(-100) or less)."""
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 3)) * np.array([1.0, 0.6, 0.3])
    X -= X.mean(0)
    a = 0.01 * np.arange(n)
    return X, a, 0.001


def _angle_about_z(A, B):
    """Mean signed angle (about z, through the centroids) that carries the
    rows of A to the rows of B, weighted by squared radius in the xy plane."""
    A = A - A.mean(0)
    B = B - B.mean(0)
    cr = A[:, 0] * B[:, 1] - A[:, 1] * B[:, 0]
    dt = A[:, 0] * B[:, 0] + A[:, 1] * B[:, 1]
    return math.atan2(cr.sum(), dt.sum())


def test_step_rotates_toward_the_reference():
    """Direction of eq. 6 as eq. 9 applies it.  The template is the
    reference turned by +10 degrees about z (through the centroid), every
    point coupled only to its counterpart, p = 1, so f_i = -(G/N)(y_i - x_i);
    dt2 is chosen so that G dt2 / N = 1/2, i.e. "after" is the midpoint
    cloud.  The Kabsch rotation from the template to the midpoints turns by
    about -5 degrees, so one step must leave about +5 degrees (between 4 and
    6).  Passing the Kabsch arguments in the wrong order (kabsch(YD, Yc), a
    transposed R) or applying R^T in eq. 9 would leave about +15 degrees."""
    X, a, sig = _labelled_pair()
    th = math.radians(10.0)
    Q = rot_axis_angle([0.0, 0.0, 1.0], 10.0)
    Y = X @ Q.T
    assert _angle_about_z(X, Y) == pytest.approx(th, rel=1e-12)
    t, E = 3, 50
    G = O.G_schedule(t, E)
    prm = O.Params(p=1.0, sigma=sig, E=E, dt2=0.5 * len(X) / G)
    S = O.make_setup(X, Y, prm, aX=a, aY=a)
    so = O.step(Y, S, t)
    assert so.c == pytest.approx(1.0, rel=1e-12)                      # same eigenvalues
    left = _angle_about_z(X, so.Y)
    assert 0.4 * th < left < 0.6 * th, math.degrees(left)


def test_exact_recovery_of_a_similarity_transform():
    """Noise-free template y = s Q x + t (40 degrees about an oblique axis,
    s = 1.3) whose points are coupled only to their counterparts, p = 1,
    dt2 = N/G1 so that the displacement G_t dt2 / N = G_t/G1 reaches 1 at
    the end of eq. 12's schedule (the midpoint becomes the reference point
    itself).  Registration must recover rotation, scale and translation to
    rounding: pose-RMSE <= 1e-9 of the diameter."""
    X, a, sig = _labelled_pair(n=60, seed=9)
    Q = rot_axis_angle([0.3, -0.8, 0.5], 40.0)
    s, t = 1.3, np.array([0.5, -0.2, 0.3])
    Y0 = s * X @ Q.T + t
    prm = O.Params(p=1.0, sigma=sig, E=60, dt2=len(X) / O.G1_DEFAULT)
    S = O.make_setup(X, Y0, prm, aX=a, aY=a)
    pose, Y, _ = O.register(Y0, S)
    assert O.pose_rmse(pose, Y0, s, Q, t) <= 1e-9 * O.diameter(X)
    np.testing.assert_allclose(pose.R, Q.T, atol=1e-10)
    assert pose.s == pytest.approx(1.0 / s, rel=1e-10)


def test_force_scale_bounds_and_equality():
    """S_i = (G/Z) sum_j |c_ij| |r_ij| bounds |f_i| (triangle inequality),
    with equality for a single reference point and for reference points that
    all lie on one side of y_i along one line; rows subset equals full."""
    pr = random_pair(30, 50, seed=4)
    rng = np.random.default_rng(3)
    S = _setup(pr.ref.astype(np.float64), rng.uniform(0, 0.3, 50), rng.uniform(0, 0.3, 30), p=2.0, sigma=0.1,
               eps=0.02, L=0.9)
    f, _ = O.forces(pr.tmpl, S, 5.0)
    sc = O.force_scale(pr.tmpl, S, 5.0)
    assert np.all(np.linalg.norm(f, axis=1) <= sc * (1 + 1e-14))
    assert np.all(np.linalg.norm(f, axis=1) < 0.999 * sc)            # generic rows cancel
    np.testing.assert_array_equal(O.force_scale(pr.tmpl, S, 5.0, rows=[3, 7]), sc[[3, 7]])
    X1 = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [4.0, 8.0, 12.0]])    # one ray from the origin
    S1 = _setup(X1, np.array([0.1, 0.2, 0.15]), np.array([0.12]), p=1.5, sigma=0.1, L=1.3)
    Y1 = np.zeros((1, 3))
    f1, _ = O.forces(Y1, S1, 2.0)
    assert np.linalg.norm(f1[0]) == pytest.approx(O.force_scale(Y1, S1, 2.0)[0], rel=1e-14)


def test_force_scale_c_matches_numpy():
    pr = random_pair(40, 70, seed=13)
    rng = np.random.default_rng(14)
    for p, g_mode, eps in ((1.0, 0, 0.0), (2.0, 1, 0.03), (-2.0, 2, 0.05)):
        S = _setup(pr.ref.astype(np.float64), rng.uniform(0.01, 0.3, 70), rng.uniform(0.01, 0.3, 40), p=p,
                   g_mode=g_mode, sigma=0.08, eps=eps, L=0.7, wX=rng.uniform(0.5, 2, 70))
        rows = [0, 5, 39]
        f, U, sc = O.forces_c(pr.tmpl, S, 3.0, rows=rows, want_scale=True)
        np.testing.assert_allclose(sc, O.force_scale(pr.tmpl, S, 3.0, rows=rows), rtol=1e-12)
        np.testing.assert_allclose(f, O.forces(pr.tmpl, S, 3.0)[0][rows], rtol=1e-12, atol=1e-14)


# ------------------------------------------- p = 1: sums over the reference first
@pytest.mark.parametrize("g_mode,masses,eps", [(0, False, 0.0), (1, True, 0.05)])
def test_forces_from_pair_sums_equal_eq5(g_mode, masses, eps):
    """At p = 1, f_i = -(G/Z) sum_j c_ij (y_i - x_j) = -(G/Z)(y_i S0_i - Sx_i)
    with c_ij independent of the pose: forces_from_sums must equal forces()
    (eq. 5 summed pair by pair) at arbitrary poses, energy included."""
    pr = random_pair(70, 110, seed=31)
    rng = np.random.default_rng(32)
    wX = rng.uniform(0.5, 2.0, 110) if masses else None
    S = _setup(pr.ref.astype(np.float64), rng.uniform(0.01, 0.3, 110), rng.uniform(0.01, 0.3, 70), p=1.0,
               g_mode=g_mode, sigma=0.08, eps=eps, wX=wX)
    sums = O.pair_sums_c(S)
    for pose in (O.Pose.identity(), O.Pose(0.8, rot_axis_angle([1, 1, 0], 70.0), np.array([0.3, -1.0, 2.0]))):
        Y = pose.apply(pr.tmpl)
        f1, U1 = O.forces(Y, S, 9.0)
        f2, U2 = O.forces_from_sums(Y, S, 9.0, sums)
        np.testing.assert_allclose(f2, f1, rtol=1e-11, atol=1e-12 * np.abs(f1).max())
        assert U2 == pytest.approx(U1, rel=1e-11)


def test_register_p1_equals_register():
    """The registration with the sums formed once follows register() (eq.
    5 summed pair by pair at every iterate) to rounding."""
    pr = config1(n=400)
    S = O.make_setup(pr.ref, pr.tmpl, O.Params(p=1.0, k=16, E=40))
    po, Y1, _ = O.register(pr.tmpl, S)
    pq, Y2, _, _ = O.register_p1(pr.tmpl, S)
    assert np.sqrt(np.mean(np.sum((Y1 - Y2) ** 2, axis=1))) <= 1e-12 * O.diameter(pr.ref)
    with pytest.raises(ValueError):
        O.pair_sums_c(O.make_setup(pr.ref, pr.tmpl, O.Params(p=2.0, k=16, E=5), aX=S.aX, aY=S.aY))
