"""The C oracle kernels (force and energy of eq. 5, the per-point scale, the
p = 1 pair sums, the float32 kNN) built for the host under AddressSanitizer
and UndefinedBehaviorSanitizer (no recovery, OpenMP on) and driven by
`tests/host/oracle_check.c`: no report on ragged sizes and every force law,
and the same values as the NumPy oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ref as O
from synth import random_pair

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("ora") / "oracle_check")
    r = subprocess.run([gcc, "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "oracle_c.c"),
                        os.path.join(HERE, "host", "oracle_check.c"), "-o", exe, "-lm"], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    return exe


def _run(exe, Y, S, G, k):
    prm = S.prm
    head = [len(Y), len(S.X), k, prm.p, prm.g_mode, S.sigma, prm.eps, S.L, S.abar, G, S.Z]
    body = np.concatenate([np.ravel(Y), S.aY, np.ravel(S.X), S.aX, S.wX])
    txt = " ".join(repr(float(v)) if isinstance(v, float) else str(v) for v in head) + "\n" + \
        " ".join(repr(float(v)) for v in body) + "\n"
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([exe], input=txt, capture_output=True, text=True, env=env)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-2000:]
    v = r.stdout.split()
    M, N = len(Y), len(S.X)
    f = np.array(v[:3 * M], float).reshape(M, 3)
    U = float(v[3 * M])
    sc = np.array(v[3 * M + 1:4 * M + 1], float)
    ps = np.array(v[4 * M + 1:9 * M + 1], float).reshape(M, 5)
    nn = np.array(v[9 * M + 1:9 * M + 1 + N * k], int).reshape(N, k)
    return f, U, sc, ps, nn


@pytest.mark.parametrize("p,g_mode,eps,masses", [(1.0, 0, 0.0, False), (2.0, 1, 0.02, True), (-2.0, 2, 0.1, True),
                                                 (1.5, 0, 0.05, False)])
def test_c_oracle_under_sanitizers_matches_numpy(driver, p, g_mode, eps, masses):
    pr = random_pair(37, 53, seed=21)
    rng = np.random.default_rng(22)
    aX, aY = rng.uniform(0.05, 0.3, 53), rng.uniform(0.05, 0.3, 37)
    wX = rng.uniform(0.5, 2.0, 53) if masses else None
    prm = O.Params(p=p, g_mode=g_mode, eps=eps, k=5)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX, aY=aY, wX=wX)
    Y = pr.tmpl.astype(np.float64)
    G = 1234.5
    f, U, sc, ps, nn = _run(driver, Y, S, G, 5)
    f_o, U_o = O.forces(Y, S, G)
    scale = np.abs(f_o).sum()
    np.testing.assert_allclose(f, f_o, rtol=0, atol=1e-12 * scale)
    assert U == pytest.approx(U_o, rel=1e-12)
    np.testing.assert_allclose(sc, O.force_scale(Y, S, G), rtol=1e-12)
    if p == 1.0:
        f_s, _ = O.forces_from_sums(Y, S, G, ps)
        np.testing.assert_allclose(f_s, f_o, rtol=0, atol=1e-12 * scale)
    np.testing.assert_array_equal(nn, O.knn_bruteforce(pr.ref, 5))
