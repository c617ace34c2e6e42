"""Launch shapes of the pair-force kernel (sgr_set_tiles, sgr_autotune,
sgr_tiles_save / sgr_tiles_load).  A shape changes how the template is cut
into blocks and the reference into chunks, hence the order of the FP32 and
FP64 sums, never the result beyond rounding: registrations under every shape
match the default shape (whose registrations are checked against the oracle
elsewhere) to 1e-6 of the diameter.  The shape R = 1 with 64 blocks per CU
writes over 6 000 wrench rows per launch, so the update's partial-row
reduction takes several rounds of loads."""
import json

import numpy as np
import pytest
import torch

from oracle import ref as O
from synth import config1

pytestmark = pytest.mark.gpu

SHAPES = [(1, 64, 0), (8, 1, 1), (4, 16, 1), (2, 3, 0), (1, 2, 1)]


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1902_01061_amd as sg
    return sg


def _pose(sg, p):
    s, R, t = sg.pose_to_srt(p)
    return O.Pose(s, R, t)


def _rmse(pa, pb, P):
    d = pa.apply(P) - pb.apply(P)
    return float(np.sqrt(np.mean(np.sum(d * d, axis=1))))


@pytest.mark.parametrize("p,g_mode,eps", [(1.0, 0, 0.0), (-2.0, 2, 0.05)])
def test_launch_shapes_agree(sg, p, g_mode, eps):
    """The p = 1 law (moment form of the pair loop) and eq. 1's law (general
    distance law); 30 iterations."""
    pr = config1(n=20000)
    ctx = sg.Context(0)
    try:
        tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
        prm = sg.Params(p=p, g_mode=g_mode, eps=eps, k=16, E=30)
        base, _ = ctx.register(tm, rf, prm)
        pb = _pose(sg, base)
        D = O.diameter(pr.ref)
        for R, bpc, var in SHAPES:
            ctx.set_tiles(pr.M, pr.N, p, R, bpc, var)
            pose, st = ctx.register(tm, rf, prm, stats=True)
            e = _rmse(_pose(sg, pose), pb, pr.tmpl) / D
            print(f"p = {p}, R = {R}, blocks/CU = {bpc}, variant = {var}: {e:.1e} D from the default shape")
            assert np.all(st.cpu().numpy()[:, 28] == 0), (R, bpc, var)
            assert e <= 1e-6, (R, bpc, var)
        ctx.set_tiles(pr.M, pr.N, p, 0, 1, 0)               # entry removed: the default again
        again, _ = ctx.register(tm, rf, prm)
        assert torch.equal(again, base)
    finally:
        ctx.close()


def test_autotune_and_tile_table_round_trip(sg, tmp_path):
    pr = config1(n=3000)
    ctx = sg.Context(0)
    try:
        tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
        a_t, mom_t = ctx.descriptors(tm, 16)
        a_r, mom_r = ctx.descriptors(rf, 16)
        prm = sg.Params(p=1.0, k=16, E=20)
        base, _ = ctx.register(tm, rf, prm)
        (R, bpc, var), ms = ctx.autotune(tm, a_t, rf, a_r, mom_t, mom_r, prm, reps=2)
        assert R in (1, 2, 4, 8) and 1 <= bpc <= 64 and var in (0, 1)
        assert np.isfinite(ms) and ms > 0
        tuned, _ = ctx.register(tm, rf, prm)
        assert _rmse(_pose(sg, tuned), _pose(sg, base), pr.tmpl) <= 1e-6 * O.diameter(pr.ref)
        path = tmp_path / "tiles.json"
        ctx.save_tiles(str(path))
        saved = json.loads(path.read_text())
        ctx2 = sg.Context(0)
        try:
            ctx2.load_tiles(str(path))
            path2 = tmp_path / "tiles2.json"
            ctx2.save_tiles(str(path2))
            assert json.loads(path2.read_text()) == saved
            again, _ = ctx2.register(tm, rf, prm)
            assert torch.equal(again, tuned)
        finally:
            ctx2.close()
    finally:
        ctx.close()
