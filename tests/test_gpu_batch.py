"""Batched registrations and multi-start: one persistent launch per
iteration over many uneven registrations, against single registrations
(same method, one call each) and the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import ref as O
from synth import config1, config4, rot_axis_angle, super_fibonacci_rotations

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


def _pose(sg, v):
    s, R, t = sg.pose_to_srt(v)
    return O.Pose(s, R, t)


def _prmse(pa, pb, Y):
    d = pa.apply(Y) - pb.apply(Y)
    return float(np.sqrt(np.mean(np.sum(d * d, axis=1))))


def test_batch_matches_single_registrations(sg, ctx):
    pairs = config4(B=7, nmin=300, nmax=6000, iters=25)
    prm = sg.Params(p=1.0, k=16, E=25)
    tms = [sg.Cloud(p.tmpl) for p in pairs]
    rfs = [sg.Cloud(p.ref) for p in pairs]
    poses, energy, _ = ctx.register_batch(tms, rfs, prm)
    poses = poses.cpu().numpy()
    for r, pr in enumerate(pairs):
        single, _ = ctx.register(tms[r], rfs[r], prm)
        pb, ps = _pose(sg, torch.as_tensor(poses[r])), _pose(sg, single)
        assert _prmse(pb, ps, pr.tmpl) <= 1e-5 * O.diameter(pr.ref), r
    # one of them against the oracle
    pr = pairs[0]
    S = O.make_setup(pr.ref, pr.tmpl, O.Params(p=1.0, k=16, E=25))
    po, Y, hist = O.register(pr.tmpl, S, keep=True)
    assert _prmse(_pose(sg, torch.as_tensor(poses[0])), po, pr.tmpl) <= 1e-4 * O.diameter(pr.ref)
    assert energy[0].item() == pytest.approx(hist[-1].U, rel=1e-4)


def test_batch_is_deterministic_and_graph_equals_eager(sg, ctx):
    pairs = config4(B=5, nmin=500, nmax=3000, iters=12)
    tms = [sg.Cloud(p.tmpl) for p in pairs]
    rfs = [sg.Cloud(p.ref) for p in pairs]
    outs = []
    for flags in (0, 0, 1):
        poses, energy, st = ctx.register_batch(tms, rfs, sg.Params(p=1.0, k=16, E=12, flags=flags), stats=True)
        outs.append((poses.cpu().numpy(), energy.cpu().numpy(), st.cpu().numpy()))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_multistart_matches_single_starts_and_picks_lowest_energy(sg, ctx):
    pr = config1(n=1500)
    R0 = super_fibonacci_rotations(6)
    prm = sg.Params(p=1.0, k=16, E=20)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    poses, energy, best = ctx.multistart(tm, rf, prm, R0)
    poses, energy = poses.cpu().numpy(), energy.cpu().numpy()
    ybar = pr.tmpl.astype(np.float64).mean(axis=0)
    for s in range(len(R0)):
        p0 = sg.pose_from_srt(1.0, R0[s], ybar - R0[s] @ ybar)
        single, _ = ctx.register(tm, rf, prm, pose=p0)
        assert _prmse(_pose(sg, torch.as_tensor(poses[s])), _pose(sg, single), pr.tmpl) <= 1e-5 * O.diameter(pr.ref)
    assert best == int(np.argmin(energy))
    assert np.isfinite(energy).all()
