"""Per-point force bar of the GPU parity tests (imported by them; not a test
module).

The force on template point i (eq. 5) is a sum of terms c_ij r_ij; any
evaluation that rounds the terms or adds them in another order errs by an
amount bounded relative to the absolute-sum scale S_i = (G/Z) sum_j |c_ij|
|r_ij| (oracle: force_scale, forces_c(want_scale=True)), not relative to
|f_i|, which cancels.  The bar is therefore, for every compared row,

    |f_i(GPU) - f_i(oracle)| <= F_TOL (S_i + FLOOR max_k S_k).

FLOOR covers rows whose every term lies below float32's smallest normal
number (2^-126 of the largest possible weight): the GPU flushes such terms
to zero, so a row's lost share is at most N 2^-126 max|r| G/Z, while
max_k S_k is of order G max|r| whenever any row has a weight near 1.
1e-20 is far above that share and far below any row that matters to F or K.
"""
import numpy as np

F_TOL = 1e-4
FLOOR = 1e-20


def row_error(f_gpu, f_ora, scale) -> float:
    """max_i |f_gpu_i - f_ora_i| / (S_i + FLOOR max S)."""
    f_gpu = np.asarray(f_gpu, np.float64)
    f_ora = np.asarray(f_ora, np.float64)
    scale = np.asarray(scale, np.float64)
    den = scale + FLOOR * float(scale.max())
    if not float(scale.max()) > 0:
        return float(np.abs(f_gpu - f_ora).max())
    return float(np.max(np.linalg.norm(f_gpu - f_ora, axis=1) / den))


def nonzero_rows(f_ora, scale) -> int:
    """Rows whose force is not negligible: |f_i| > 1e-6 max |f|."""
    n = np.linalg.norm(np.asarray(f_ora, np.float64), axis=1)
    return int(np.count_nonzero(n > 1e-6 * n.max())) if n.max() > 0 else 0
