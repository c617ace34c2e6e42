"""Change detection after registration (the application of Sec. I and
Sec. IV) against the oracle: flags, nearest reference indices and float32
keys are integer or exactly specified float32 decisions, compared bit for
bit, on small pairs with edge cases and on the full depth-frame scene in
both directions (template parts missing from the reference, and reference
parts missing from the template under the inverse pose)."""
import math

import numpy as np
import pytest
import torch

from oracle import ref as O
from synth import config1, config5, random_pair, rot_axis_angle

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


def _dt(x, dtype=torch.float32):
    return torch.as_tensor(np.asarray(x)).to(device="cuda", dtype=dtype).contiguous()


def _check(sg, ctx, Y, aY, X, aX, pose, tau, sigma, s_min):
    f_o, nn_o, key_o = O.change_flags(Y, aY, X, aX, pose, tau, sigma, s_min)
    f, nn, key = ctx.change_detect(sg.Cloud(np.asarray(Y, np.float32)), _dt(aY), sg.Cloud(np.asarray(X, np.float32)),
                                   _dt(aX), _dt(pose.as_array(), torch.float64), tau, sigma, s_min)
    f, nn, key = f.cpu().numpy(), nn.cpu().numpy(), key.cpu().numpy()
    assert np.array_equal(nn, nn_o.astype(np.int32)), "nearest indices differ"
    assert np.array_equal(key.view(np.uint32), key_o.view(np.uint32)), "keys differ"
    assert np.array_equal(f, f_o), "flags differ"
    return f


@pytest.mark.parametrize("case", ["config1", "random", "edges"])
def test_change_detect_matches_oracle(sg, ctx, case):
    rng = np.random.default_rng(31)
    if case == "config1":
        pr = config1(n=3000)
        Y, X = pr.tmpl, pr.ref
        pose = O.Pose(1 / pr.gt_s, pr.gt_R.T, -(pr.gt_R.T @ pr.gt_t) / pr.gt_s)   # template onto reference
        tau = 0.02
    elif case == "random":
        pr = random_pair(2500, 4100, seed=32)
        Y, X = pr.tmpl, pr.ref
        pose = O.Pose(0.9, rot_axis_angle([1, -1, 2], 25.0), np.array([0.1, 0.2, -0.1]))
        tau = 0.1
    else:
        # duplicates, a template far outside the reference box, a NaN point
        X = rng.normal(size=(700, 3)).astype(np.float32)
        X[10:20] = X[3]
        Y = np.concatenate([X[:300], rng.normal(size=(50, 3)) * 30.0, [[np.nan, 0.0, 0.0]]]).astype(np.float32)
        pose = O.Pose.identity()
        tau = 0.5
    aX = rng.uniform(0.0, 0.2, len(X)).astype(np.float32)
    aY = rng.uniform(0.0, 0.2, len(Y)).astype(np.float32)
    sigma = float(np.std(aX.astype(np.float64)))
    f = _check(sg, ctx, Y, aY, X, aX, pose, tau, sigma, 0.5)
    assert 0 < np.count_nonzero(f) < len(f)
    _check(sg, ctx, Y, aY, X, aX, pose, math.inf, sigma, 0.5)      # shape test only
    _check(sg, ctx, Y, aY, X, aX, pose, tau, sigma, 0.0)           # distance test only


def test_change_detect_scene_full_size(sg, ctx):
    """The depth-frame scene at the generating transform: both directions
    bit for bit against the oracle; the flags' agreement with the scene's
    own change labels is printed."""
    pr = config5()
    aX, _ = ctx.descriptors(sg.Cloud(pr.ref), 16)
    aY, _ = ctx.descriptors(sg.Cloud(pr.tmpl), 16)
    aX, aY = aX.cpu().numpy(), aY.cpu().numpy()
    sigma = float(np.std(aX.astype(np.float64)))
    fwd = O.Pose(1 / pr.gt_s, pr.gt_R.T, -(pr.gt_R.T @ pr.gt_t) / pr.gt_s)
    inv = O.Pose(pr.gt_s, pr.gt_R, pr.gt_t)
    tau = 0.05
    f = _check(sg, ctx, pr.tmpl, aY, pr.ref, aX, fwd, tau, sigma, 0.0)
    g = _check(sg, ctx, pr.ref, aX, pr.tmpl, aY, inv, tau, sigma, 0.0)
    hit = (f & 1) > 0
    print(f"scene change detection (tau = {tau}): template recall {np.mean(hit[pr.changed]):.3f} on the added boxes, "
          f"flag rate {np.mean(hit[~pr.changed]):.3f} elsewhere; reference recall "
          f"{np.mean((g & 1)[pr.ref_changed] > 0):.3f} on the removed box")


def test_change_detect_rejects_bad_arguments(sg, ctx):
    X = np.random.default_rng(1).normal(size=(64, 3)).astype(np.float32)
    a = _dt(np.zeros(64, np.float32))
    c = sg.Cloud(X)
    p = sg.pose_identity()
    with pytest.raises(sg.SgrError):
        ctx.change_detect(c, a, c, a, p, 0.0)           # tau must be > 0
    with pytest.raises(sg.SgrError):
        ctx.change_detect(c, a, c, a, p, 0.1, 0.0, 0.5)  # shape test without sigma
    with pytest.raises(sg.SgrError):
        ctx.change_detect(c, a, c, a, p, 0.1, 0.1, 1.5)  # s_min > 1
