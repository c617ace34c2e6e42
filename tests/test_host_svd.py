"""The 3x3 FP64 routines of the rigid update (one-sided Jacobi SVD, the
Kabsch rotation of eq. 6, eigenvalues of a PSD matrix), compiled for the
host from the same header the kernels include and checked against numpy's
SVD and eigensolver: singular values, orthonormal singular vectors, the
reconstruction, R = V diag(1, 1, sign det(V U^T)) U^T with C = U S V^T
(reflections included), the rank tests, and a warm start from a nearby
matrix's right singular vectors giving the same result as a cold start."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _build(tmp_path_factory, name, extra):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("svd") / name)
    subprocess.run([hipcc, "--offload-arch=gfx950", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops"] + extra + [os.path.join(HERE, "host", "svd_check.hip"), "-o", exe],
                   check=True, capture_output=True)

    def run(cases):
        """cases: list of (A 3x3, V0 3x3 or None)."""
        lines = []
        for A, V0 in cases:
            v0 = np.zeros(9) if V0 is None else np.asarray(V0, float).ravel()
            lines.append(" ".join([str(int(V0 is not None))] + [repr(float(x)) for x in np.asarray(A).ravel()]
                                  + [repr(float(x)) for x in v0]))
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True)
        assert out.returncode == 0 and "runtime error" not in out.stderr and "Sanitizer" not in out.stderr, \
            out.stderr[-2000:]
        res = []
        for ln in out.stdout.strip().split("\n"):
            x = np.array([float(t) for t in ln.split()])
            res.append(dict(sv=x[0:3], u=x[3:12].reshape(3, 3), v=x[12:21].reshape(3, 3), R=x[21:30].reshape(3, 3),
                            ok=int(x[30]), lam=x[31:34]))
        return res
    return run


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return _build(tmp_path_factory, "svd_check", ["-O2"])


def _kabsch(C):
    U, S, Vt = np.linalg.svd(C)
    V = Vt.T
    d = np.sign(np.linalg.det(V @ U.T))
    return V @ np.diag([1.0, 1.0, d]) @ U.T


def _random_rot(rng):
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return Q * np.sign(np.linalg.det(Q))


def _cases(rng, n):
    out = []
    for _ in range(n):
        # well separated singular values, random signs of the determinant
        s = np.sort(rng.uniform(0.5, 10.0, 3))[::-1] * np.array([1.0, 0.7, 0.4])
        A = _random_rot(rng) @ np.diag(s) @ _random_rot(rng).T
        if rng.random() < 0.5:
            A = A @ np.diag([1.0, 1.0, -1.0])
        out.append(A * 10.0 ** rng.uniform(-3, 3))
    return out


def test_svd_and_kabsch_match_numpy(harness):
    rng = np.random.default_rng(7)
    mats = _cases(rng, 40)
    res = harness([(A, None) for A in mats])
    for A, r in zip(mats, res):
        nrm = np.linalg.norm(A)
        sv_np = np.linalg.svd(A, compute_uv=False)
        assert np.all(np.diff(r["sv"]) <= 0)
        np.testing.assert_allclose(r["sv"], sv_np, rtol=0, atol=1e-13 * sv_np[0])
        U, V = r["u"].T, r["v"].T                        # columns: singular vectors
        np.testing.assert_allclose(U.T @ U, np.eye(3), atol=1e-13)
        np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-13)
        np.testing.assert_allclose(U @ np.diag(r["sv"]) @ V.T, A, atol=1e-13 * nrm)
        assert r["ok"] == 1
        R = r["R"]
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-13)
        assert abs(np.linalg.det(R) - 1.0) < 1e-13
        np.testing.assert_allclose(R, _kabsch(A), atol=1e-11)


def test_warm_start_gives_the_cold_result(harness):
    """V0 from a matrix 1e-3 away (as the previous iteration's C is), made a
    proper rotation as the update keeps it."""
    rng = np.random.default_rng(8)
    mats = _cases(rng, 30)
    cases = []
    for A in mats:
        B = A + 1e-3 * np.linalg.norm(A) * rng.normal(size=(3, 3))
        _, _, Vt = np.linalg.svd(B)
        V0 = Vt.T * np.sign(np.linalg.det(Vt))
        cases += [(A, None), (A, V0)]
    res = harness(cases)
    for A, cold, warm in zip(mats, res[0::2], res[1::2]):
        np.testing.assert_allclose(warm["sv"], cold["sv"], rtol=0, atol=1e-13 * cold["sv"][0])
        np.testing.assert_allclose(warm["R"], cold["R"], atol=1e-12)
        np.testing.assert_allclose(warm["R"], _kabsch(A), atol=1e-11)


def test_rank_cases_and_psd_eigenvalues(harness):
    rng = np.random.default_rng(9)
    P, Q = _random_rot(rng), _random_rot(rng)
    rank2 = P @ np.diag([3.0, 1.0, 0.0]) @ Q.T
    rank1 = P @ np.diag([3.0, 0.0, 0.0]) @ Q.T
    B = rng.normal(size=(3, 3))
    psd = B @ B.T
    res = harness([(rank2, None), (rank1, None), (np.zeros((3, 3)), None), (np.eye(3), None), (psd, None)])
    r2, r1, z, eye, ps = res
    # rank 2: the rotation is still determined (third axis from the cross products)
    assert r2["ok"] == 1
    np.testing.assert_allclose(r2["R"], _kabsch(rank2), atol=1e-12)
    assert r1["ok"] == 0 and z["ok"] == 0
    np.testing.assert_array_equal(z["sv"], np.zeros(3))
    assert eye["ok"] == 1
    np.testing.assert_allclose(eye["R"], np.eye(3), atol=1e-15)
    lam_np = np.sort(np.linalg.eigvalsh(psd))[::-1]
    np.testing.assert_allclose(ps["lam"], lam_np, rtol=0, atol=1e-13 * lam_np[0])


def test_extreme_scales(harness):
    """Entries near 1e-100 or 1e100 (and subnormal or near-overflow ones):
    products of squared column norms would under- or overflow in the
    rotation tests, so the routine works on an exactly rescaled copy.
    Singular values scale with A, vectors and the rotation do not."""
    rng = np.random.default_rng(10)
    base = _cases(rng, 6)
    scales = [1e-100, 1e100, 1e-300, 1e300, 2.0 ** -1060, 1e-160]
    cases = [(A / np.abs(A).max() * sc, None) for A in base for sc in scales]
    res = harness(cases)
    for (A, _), r in zip(cases, res):
        sv_np = np.linalg.svd(A, compute_uv=False)
        # subnormal inputs carry fewer significant bits
        tol = 1e-13 if sv_np[0] > 1e-290 else 1e-3
        np.testing.assert_allclose(r["sv"], sv_np, rtol=tol)
        assert r["ok"] == 1
        np.testing.assert_allclose(r["R"], _kabsch(A), atol=1e-11 if tol < 1e-6 else 1e-2)
        assert abs(np.linalg.det(r["R"]) - 1.0) < 1e-12


def test_routines_under_host_sanitizers(harness, tmp_path_factory):
    """The same routines built for the host with AddressSanitizer and
    UndefinedBehaviorSanitizer (no recovery: any report ends the run with an
    error), over every case above: warm and cold starts, rank 2, 1 and 0,
    the identity, PSD eigenvalues and entries from 2^-1060 to 1e300.  No
    report, and the same results as the optimised build."""
    san = _build(tmp_path_factory, "svd_check_san",
                 ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all"])
    rng = np.random.default_rng(11)
    mats = _cases(rng, 20)
    cases = [(A, None) for A in mats]
    for A in mats[:10]:
        _, _, Vt = np.linalg.svd(A + 1e-3 * np.linalg.norm(A) * rng.normal(size=(3, 3)))
        cases.append((A, Vt.T * np.sign(np.linalg.det(Vt))))
    P, Q = _random_rot(rng), _random_rot(rng)
    cases += [(P @ np.diag([3.0, 1.0, 0.0]) @ Q.T, None), (P @ np.diag([3.0, 0.0, 0.0]) @ Q.T, None),
              (np.zeros((3, 3)), None), (np.eye(3), None)]
    cases += [(A / np.abs(A).max() * sc, None) for A in mats[:3] for sc in (1e-300, 1e300, 2.0 ** -1060)]
    a, b = san(cases), harness(cases)
    assert len(a) == len(b) == len(cases)
    for x, y in zip(a, b):
        assert x["ok"] == y["ok"]
        for key in ("sv", "R", "lam"):
            np.testing.assert_allclose(x[key], y[key], rtol=1e-12, atol=1e-12 * max(1.0, float(np.abs(y[key]).max())))
