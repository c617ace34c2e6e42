"""Mixed-precision force (p = 1): pair weights in FP32 rounded to bf16, the
similarity-weighted sums on the matrix cores, FP64 wrench.  Compared with
the FP64 oracle one step at a time.  Tolerance derived from the arithmetic:
each weight carries a relative rounding error of at most 2^-9 (round to
nearest even, unbiased), coordinates 2^-17 (bf16 head + tail); over the
N_eff reference points that carry weight the random errors average to about
2^-9 / sqrt(N_eff) relative, and forming f = y S0 - S_x can amplify it by
|y| / |y - xbar_c| (about 10 here), so the gate is 2e-3 for clouds of a few
thousand points; the measured errors are printed."""
import numpy as np
import pytest
import torch

from oracle import ref as O
from synth import config1, random_pair, rot_axis_angle

pytestmark = pytest.mark.gpu

MIXED = 2   # params flag bit


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


@pytest.mark.parametrize("g_mode,masses", [(0, False), (1, False), (0, True)])
def test_mixed_step_matches_oracle(sg, ctx, g_mode, masses):
    pr = random_pair(1300, 2900, seed=41)
    rng = np.random.default_rng(7)
    aX32 = rng.uniform(0.01, 0.3, pr.N).astype(np.float32)
    aY32 = rng.uniform(0.01, 0.3, pr.M).astype(np.float32)
    wX = rng.uniform(0.5, 2.0, pr.N).astype(np.float32) if masses else None
    mY = rng.uniform(0.5, 2.0, pr.M).astype(np.float32) if masses else None
    prm = O.Params(p=1.0, g_mode=g_mode, k=16, E=40)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX32.astype(np.float64), aY=aY32.astype(np.float64),
                     wX=None if wX is None else wX.astype(np.float64), mY=None if mY is None else mY.astype(np.float64))
    pose = O.Pose(1.1, rot_axis_angle([1, 2, 3], 20.0), np.array([0.1, -0.2, 0.05]))
    Y = pose.apply(pr.tmpl)
    so = O.step(Y, S, 21)
    gp = sg.Params(p=1.0, g_mode=g_mode, k=16, E=40, flags=MIXED)
    _, wr, f = ctx.step(sg.Cloud(pr.tmpl, masses=mY), _dt(aY32), sg.Cloud(pr.ref, masses=wX), _dt(aX32),
                        _dt(_mom(pr.tmpl), torch.float64), _dt(_mom(pr.ref), torch.float64), gp, 21,
                        sg.pose_from_srt(pose.s, pose.R, pose.t), want_wrench=True, want_f=True)
    f = f.cpu().numpy().astype(np.float64)
    wr = wr.cpu().numpy()
    m = np.ones(pr.M) if mY is None else mY.astype(np.float64)
    e_f = np.linalg.norm(f - so.f) / np.linalg.norm(so.f)
    e_F = np.linalg.norm(wr[0:3] - so.F) / np.sum(m * np.linalg.norm(so.f, axis=1))
    Yc = Y - Y.mean(0)
    e_K = np.linalg.norm(wr[3:12].reshape(3, 3) - so.K) / np.sum(np.linalg.norm(so.f, axis=1) * np.linalg.norm(Yc, axis=1))
    print(f"mixed one-step errors: e_f={e_f:.2e} e_F={e_F:.2e} e_K={e_K:.2e}")
    assert e_f <= 2e-3 and e_F <= 2e-3 and e_K <= 2e-3


def test_mixed_register_close_to_oracle(sg, ctx):
    pr = config1(n=4000)
    S = O.make_setup(pr.ref, pr.tmpl, O.Params(p=1.0, k=16, E=40))
    po, _, _ = O.register(pr.tmpl, S)
    pg, _ = ctx.register(sg.Cloud(pr.tmpl), sg.Cloud(pr.ref), sg.Params(p=1.0, k=16, E=40, flags=MIXED))
    s, R, t = sg.pose_to_srt(pg)
    d = O.Pose(s, R, t).apply(pr.tmpl) - po.apply(pr.tmpl)
    err = np.sqrt(np.mean(np.sum(d * d, axis=1))) / O.diameter(pr.ref)
    print(f"mixed registration pose parity RMSE / diameter = {err:.2e}")
    assert err <= 1e-3


def test_mixed_rejects_p_other_than_one(sg, ctx):
    pr = random_pair(50, 60, seed=2)
    with pytest.raises(sg.SgrError):
        ctx.register(sg.Cloud(pr.tmpl), sg.Cloud(pr.ref), sg.Params(p=2.0, k=8, E=3, flags=MIXED))
