"""Write the tile table (launch shapes of the all-pairs force kernel) for
the workloads this library is measured on, with sgr_autotune on one MI355X:

  tiny pair 1 024 x 1 024 (p = 1), scan pair 32 400 x 36 000 (p = 1 and
  p = 2, whose entry the other laws of the r-form share),
  differentiation pair 8 192 x 8 192 (p = 2, eps = 0.05 L), the median
  registration of the 256-registration batch (p = 1), the multi-start pair
  22 000 x 20 000 (p = 1), and the depth-frame scene 250 000 x 307 200
  (p = 1 and p = 2, g = a a s).

Entries are keyed by (log2 M, log2 N, distance-law mode); a call whose sizes
fall in a bucket uses the entry.  Usage (on the GPU):

    python paper_1902_01061_amd/tune_tiles.py [out.json]
"""
from __future__ import annotations

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> int:
    import numpy as np

    import paper_1902_01061_amd as sg
    from synth import config1, config2, config3, config4, config4_multistart, config5

    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "tiles_gfx950.json")
    ctx = sg.Context(0)
    pairs4 = config4()
    med = sorted(pairs4, key=lambda p: p.N)[len(pairs4) // 2]
    ms_pair, _ = config4_multistart()
    jobs = [("tiny 1024 x 1024, p = 1", config1(), dict(p=1.0), 16),
            ("scan 32400 x 36000, p = 1", config2(), dict(p=1.0), 24),
            ("scan 32400 x 36000, p = 2", config2(), dict(p=2.0), 24),
            ("differentiation 8192 x 8192, p = 2", config3(), dict(p=2.0, eps_rel=0.05), 16),
            (f"batch median {med.M} x {med.N}, p = 1", med, dict(p=1.0), 16),
            (f"multi-start {ms_pair.M} x {ms_pair.N}, p = 1", ms_pair, dict(p=1.0), 16)]
    scene = config5()
    jobs += [("scene 250000 x 307200, p = 1, g = a a s", scene, dict(p=1.0, g_mode=1), 16),
             ("scene 250000 x 307200, p = 2, g = a a s", scene, dict(p=2.0, g_mode=1), 16)]
    for name, pr, kw, k in jobs:
        tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
        a_t, mom_t = ctx.descriptors(tm, k)
        a_r, mom_r = ctx.descriptors(rf, k)
        eps = kw.pop("eps_rel", 0.0) * float(np.sqrt(mom_r[9].item()))
        prm = sg.Params(k=k, E=100, eps=eps, **kw)
        best, ms = ctx.autotune(tm, a_t, rf, a_r, mom_t, mom_r, prm, reps=5)
        print(f"{name}: R={best[0]} blocks/CU={best[1]} variant={best[2]}: {ms * 1e3:.1f} us per launch",
              flush=True)
    ctx.save_tiles(out)
    ctx.close()
    print(f"tile table written to {out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
