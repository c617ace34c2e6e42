"""sgr_step_static, the allocation-free form of sgr_step, through the C ABI:
bit-identical pose, wrench and per-point forces to sgr_step on the same
inputs, for two calls in a row (the second with a smaller pair, so that the
static scratch holds the first call's contents), for the p = 1 and p = 2
laws, with and without per-point output; a pair beyond the scratch's size
is rejected on the host before anything is launched."""
import numpy as np
import pytest
import torch

from synth import random_pair, rot_axis_angle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_01061_amd as sg
    return sg


def _mom(P):
    Q = P.astype(np.float64)
    c = Q.mean(0)
    Qc = Q - c
    S = Qc.T @ Qc / len(Q)
    return torch.tensor([c[0], c[1], c[2], S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2],
                         np.linalg.eigvalsh(S)[-1]], dtype=torch.float64, device="cuda")


def test_static_step_equals_step(sg):
    ctx = sg.Context(0)
    try:
        for M, N, seed in ((5000, 6100, 1), (700, 900, 2)):
            pr = random_pair(M, N, seed=seed)
            tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
            a_t, _ = ctx.descriptors(tm, 16)
            a_r, _ = ctx.descriptors(rf, 16)
            mt, mr = _mom(pr.tmpl), _mom(pr.ref)
            pin = sg.pose_from_srt(1.05, rot_axis_angle([1, -2, 1], 15.0), np.array([0.1, 0.0, -0.2]))
            for p, eps in ((1.0, 0.0), (2.0, 0.02)):
                prm = sg.Params(p=p, k=16, eps=eps, E=30)
                for want_f in (True, False):
                    print(f"M={M} N={N} p={p} want_f={want_f}", flush=True)
                    a = ctx.step(tm, a_t, rf, a_r, mt, mr, prm, 7, pin, want_wrench=True, want_f=want_f)
                    b = ctx.step(tm, a_t, rf, a_r, mt, mr, prm, 7, pin, want_wrench=True, want_f=want_f,
                                 static_scratch=True)
                    torch.cuda.synchronize()
                    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
                    if want_f:
                        assert torch.equal(a[2], b[2])
                    assert torch.isfinite(b[0]).all()
    finally:
        ctx.close()


def test_static_step_rejects_a_pair_beyond_the_scratch(sg):
    ctx = sg.Context(0)
    try:
        n = 1_200_000                   # about 96 MB of buffers, beyond the 64 MiB array
        P = torch.rand((n, 3), dtype=torch.float32, device="cuda")
        cl = sg.Cloud(P)
        a = torch.rand(n, dtype=torch.float32, device="cuda")
        mom = torch.tensor([0.5, 0.5, 0.5, 1 / 12, 1 / 12, 1 / 12, 0, 0, 0, 1 / 12], dtype=torch.float64,
                           device="cuda")
        with pytest.raises(sg.SgrError) as e:
            ctx.step(cl, a, cl, a, mom, mom, sg.Params(p=1.0, k=16, E=10), 0, sg.pose_identity(),
                     static_scratch=True)
        assert e.value.code == -1 and "static scratch" in str(e.value)
    finally:
        ctx.close()
