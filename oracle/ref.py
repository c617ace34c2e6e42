"""FP64 CPU oracle of shape-constrained gravitational registration.

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import or call this
module: only the tests, the smoke check and the bench's CPU-baseline leg do.
It shares no code with the HIP path.

It follows the paper (Agarwal & Bhowmick, "3D Point Cloud Registration with
Shape Constraint", arXiv 1902.01061) step by step, in float64, literally
updating the template point array as eq. (9) does, with these readings of
passages the paper leaves open (each is repeated where it is used):

* X is the reference (N points), Y the template (M points); the mass and
  velocity "of X" in eq. (5.5) are the template's (Sec. III-B calls the
  template X there).
* n_ij = (y_i - x_j)/|y_i - x_j|, so -G n_ij pulls the template point toward
  the reference point (eq. 5; attraction, Sec. II/III).
* Distance law (eqs. 4, 11): h(d) n = d^(p-1) r with r = y_i - x_j, i.e.
  |f| grows like d^p; p = 1 by default (larger p overshoots, as Sec. IV
  warns: with p = 2 the update flips the template by 180 degrees once
  G dt^2 nears 1).  Softening eps and the length scale L = sqrt(lambda_max
  of the reference covariance) are added for dimensional consistency:
  h = ((d^2 + eps^2)/L^2)^((p-1)/2); eps = 0 reproduces the paper exactly.
* g(s) = s (Sec. IV, equal weightage) or g = (a_i/abar)(a_j/abar) s (eq. 10),
  with abar the mean reference descriptor; g = 1 (g_mode 2) drops the shape
  term and leaves the masses, so p = -2 with eps > 0 is eq. (1): the text
  states |f| ~ 1/d^2, so the numerator of eq. (1) is read as the vector
  r = y_i - x_j (standard softened gravity r/(d^2 + eps^2)^(3/2)), not a
  unit vector, whose force would fall as 1/d^3.  Eq. (1)'s friction term is
  not part of this force.
* The similarity spread sigma defaults to the population std of the
  reference descriptors (the paper gives no value, eq. 3).
* Radius neighbourhoods (Sec. IV: radius sqrt(eX), sqrt(eY), eX and eY the
  largest covariance eigenvalues of Sec. III-B): the members are decided by
  the same float32 key as the k nearest neighbours, against the float32
  threshold float32(scale^2 * lambda_max); the query is a member of its own
  neighbourhood.  The pyramidal schedule (Sec. IV, its figure is in a
  supplement that is not available) is read as a list of levels, each with a
  radius scale, a sigma scale and an iteration count; t and the G schedule
  run on across levels.
* Curvature (Sec. III-A): PCA surface variation lambda_0/(lambda_0 +
  lambda_1 + lambda_2) of the k nearest neighbours, self included, ties in
  float32 squared distance broken by index, covariance normalised by 1/k.
* The force is normalised by Z = sum_j w_j and only G dt^2 is identifiable;
  dt2 = 1/G1 by default, so G_t dt2 runs over [0.1, 1].
* Per-point displacement delta_i = dt2 f_i (Newton, v = 0); the translation
  is d = dt2 F / sum_i m_i with F = sum_i m_i f_i (eq. 5.5).
* Kabsch (eq. 6): "after" is Y + delta; C = Y_D^T Y with both centred.
* Scale (eq. 8): c = sqrt(lambda_max(Sigma_X) / lambda_max(Sigma_Y(t))),
  covariances normalised by point count, V diag(c) V^T = c I.
* Update (eq. 9): Y(t+1) = c (Y - ybar) R + ybar + d (row vectors).
* G schedule (eq. 12): iteration t (0-based) uses
  G_t = 0.1 G1 + 0.9 G1 / (1 + exp(-(t - 1 - E/2))).
* Local polynomial coefficients (Sec. III-A names them among the features
  evaluated, without a definition): a quadratic height function fitted by
  least squares in the neighbourhood's covariance frame, coordinates divided
  by the neighbourhood's RMS spread, reduced to quantities that no rotation,
  scale or frame sign changes: the fitted Hessian's eigenvalues (sign fixed
  by their sum) and the RMS residual (poly_fit).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

G1_DEFAULT = 10000.0


# ------------------------------------------------------------------ params
@dataclasses.dataclass
class Params:
    p: float = 1.0           # distance exponent, p >= 1 (eq. 11); 1 is the stable choice
    g_mode: int = 0          # 0: g = s ; 1: g = (a_i/abar)(a_j/abar) s (eq. 10) ; 2: g = 1 (eq. 1)
    k: int = 16
    sigma: float = 0.0       # <= 0: population std of the reference descriptors
    eps: float = 0.0         # softening (0 = the paper's law)
    G1: float = G1_DEFAULT   # eq. 12
    E: int = 100             # number of iterations
    dt2: float = 0.0         # <= 0: 1 / G1
    momentum: float = 0.0    # mu in [0, 1): share of the previous translation carried (0: v = 0)


# -------------------------------------------------------------- kNN (fp32)
def sqdist32(P: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Squared distances from float32 point q to rows of float32 P, each
    operation rounded to float32 in the order ((dx*dx + dy*dy) + dz*dz).
    The neighbour choice is an integer decision taken in float32; this
    fixes the exact float32 arithmetic that decides it."""
    P = P.astype(np.float32, copy=False)
    q = np.asarray(q, dtype=np.float32)
    d = P - q                                  # float32, exactly rounded
    return (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]


def knn_bruteforce(P: np.ndarray, k: int, queries=None) -> np.ndarray:
    """Exact k nearest neighbours (self included) of each query row of P,
    ordered by (float32 squared distance, index).  Returns int64 (nq, k)."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    n = P.shape[0]
    if queries is None:
        queries = np.arange(n)
    out = np.empty((len(queries), k), dtype=np.int64)
    idx = np.arange(n)
    for r, i in enumerate(queries):
        d = sqdist32(P, P[i])
        order = np.lexsort((idx, d))          # primary d, ties by index
        out[r] = order[:k]
    return out


def knn(P: np.ndarray, k: int, queries=None) -> np.ndarray:
    """Same result as knn_bruteforce.  For large clouds a k-d tree (float64)
    proposes k + 8 candidates which are then ranked by the float32 key; a
    query whose float32 k-th distance is not clearly inside the candidate
    radius is redone by brute force, so the result is always exact."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    n = P.shape[0]
    if queries is None:
        queries = np.arange(n)
    queries = np.asarray(queries)
    if n <= 4096 or k + 8 >= n:
        return knn_bruteforce(P, k, queries)
    from scipy.spatial import cKDTree

    tree = cKDTree(P.astype(np.float64))
    kk = k + 8
    dd, cand = tree.query(P[queries].astype(np.float64), k=kk)
    out = np.empty((len(queries), k), dtype=np.int64)
    for r, i in enumerate(queries):
        c = cand[r]
        d32 = sqdist32(P[c], P[i])
        order = np.lexsort((c, d32))
        kth = float(d32[order[k - 1]])
        # every point outside the candidate set lies at float64 distance
        # >= dd[r, -1]; float32 rounding moves squared distances by far less
        # than this margin unless the radii nearly coincide.
        if kth * (1 + 1e-5) + 1e-30 < dd[r, -1] ** 2:
            out[r] = c[order[:k]]
        else:
            out[r] = knn_bruteforce(P, k, [i])[0]
    return out


# -------------------------------------------------------------- descriptors
def surface_variation(P: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    """Curvature a_i = lambda_0 / (lambda_0 + lambda_1 + lambda_2) of the
    neighbourhood covariance (1/k, centred at the neighbourhood mean); 0
    when the trace is 0.  Sec. III-A (curvature as the local shape)."""
    Q = P.astype(np.float64)[nbr]                     # (n, k, 3)
    Qc = Q - Q.mean(axis=1, keepdims=True)
    C = np.einsum("nki,nkj->nij", Qc, Qc) / nbr.shape[1]
    lam = np.linalg.eigvalsh(C)                       # ascending
    tr = lam.sum(axis=1)
    a = np.zeros(len(nbr))
    nz = tr > 0
    a[nz] = lam[nz, 0] / tr[nz]
    return a


def descriptors(P: np.ndarray, k: int, queries=None) -> np.ndarray:
    """Curvature of every point (or of the ``queries`` rows) of cloud P."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    return surface_variation(P, knn(P, k, queries))


def tent_weights(u: np.ndarray, D: int) -> np.ndarray:
    """Soft binning of values u in [0, 1] into D bins centred at b/(D-1):
    bin b receives max(0, 1 - (D-1)|u - b/(D-1)|), so every u spreads a unit
    weight over its two nearest centres (linear interpolation).  (n, D)."""
    u = np.asarray(u, np.float64)
    c = np.arange(D) / (D - 1)
    return np.maximum(0.0, 1.0 - (D - 1) * np.abs(u[:, None] - c[None, :]))


def normals(P: np.ndarray, nbr: np.ndarray):
    """Unit normal of each point: the eigenvector of the smallest eigenvalue
    of its neighbourhood covariance (1/k, centred at the neighbourhood mean);
    its sign is arbitrary.  Also returns the eigenvalues (ascending), from
    which a caller can tell whether the normal is determined (lambda_0 <
    lambda_1)."""
    Q = P.astype(np.float64)[nbr]
    Qc = Q - Q.mean(axis=1, keepdims=True)
    C = np.einsum("nki,nkj->nij", Qc, Qc) / nbr.shape[1]
    lam, vec = np.linalg.eigh(C)
    return vec[:, :, 0], lam


def normal_histograms(P: np.ndarray, k: int, D: int, queries=None):
    """Vector shape descriptor (Sec. III-A names histograms of normals among
    the features evaluated): for point i with k nearest neighbours N_i (self
    included), h_i = (1/k) sum_{j in N_i} tent_weights(|n_i . n_j|), D bins
    over [0, 1].  |.| removes the arbitrary sign of the normals; the soft
    bins make h continuous in the normals.  Returns (h (nq, D), eigenvalues
    of each query's covariance)."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    n_all, lam_all = normals(P, knn(P, k))
    q = np.arange(len(P)) if queries is None else np.asarray(queries)
    nbr = knn(P, k, q)
    u = np.abs(np.einsum("qc,qkc->qk", n_all[q], n_all[nbr]))
    h = tent_weights(np.minimum(u, 1.0).reshape(-1), D).reshape(len(q), k, D).mean(axis=1)
    return h, lam_all[q]


def poly_fit(Q: np.ndarray) -> np.ndarray:
    """Local polynomial descriptor of one neighbourhood (Sec. III-A names local
    polynomial coefficients among the features evaluated), as read here: the
    points Q (k x 3, k >= 6) in the frame of their covariance (1/k, centred at
    their mean; tangent axes t1, t2 of the two largest eigenvalues, normal n of
    the smallest), every coordinate divided by rho = sqrt(trace), so that
    u = (q - qbar).t1 / rho, v = (q - qbar).t2 / rho, h = (q - qbar).n / rho;
    the least-squares fit h ~ c0 + c1 u + c2 v + c3 u^2 + c4 u v + c5 v^2; and
    the descriptor [mu1, mu2, r]: mu1 >= mu2 the eigenvalues of the fitted
    Hessian [[2 c3, c4], [c4, 2 c5]], negated and swapped when their sum is
    negative (the sign of n is arbitrary), and r the RMS residual of the fit.
    It does not change under rotation, translation, uniform scale, a change of
    sign of any axis or a rotation of the tangent axes.  rho = 0 (all points
    equal) gives NaN."""
    Q = np.asarray(Q, dtype=np.float64)
    qc = Q - Q.mean(axis=0)
    C = qc.T @ qc / len(Q)
    lam, vec = np.linalg.eigh(C)                    # ascending: n = vec[:, 0]
    rho = np.sqrt(lam.sum())
    if not rho > 0:
        return np.full(3, np.nan)
    u, v, h = qc @ vec[:, 2] / rho, qc @ vec[:, 1] / rho, qc @ vec[:, 0] / rho
    A = np.stack([np.ones_like(u), u, v, u * u, u * v, v * v], axis=1)
    c = np.linalg.lstsq(A, h, rcond=None)[0]
    mu = np.linalg.eigvalsh(np.array([[2 * c[3], c[4]], [c[4], 2 * c[5]]]))[::-1]
    if mu.sum() < 0:
        mu = -mu[::-1]
    r = np.sqrt(np.mean((h - A @ c) ** 2))
    return np.array([mu[0], mu[1], r])


def poly_descriptors(P: np.ndarray, k: int, queries=None):
    """poly_fit over every point's k nearest neighbours (self included, the
    neighbour lists of the curvature).  Returns (descriptors (nq, 3),
    covariance eigenvalues (nq, 3) ascending): the normal, and so the
    descriptor, is determined only where lambda_0 < lambda_1."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    q = np.arange(len(P)) if queries is None else np.asarray(queries)
    nbr = knn(P, k, q)
    _, lam = normals(P, nbr)
    out = np.stack([poly_fit(P[nb]) for nb in nbr]) if len(q) else np.zeros((0, 3))
    return out, lam


def radius_descriptors(P: np.ndarray, r2, queries=None):
    """Curvature of radius neighbourhoods (Sec. IV: neighbourhood radius
    sqrt(eX) for the reference, sqrt(eY) for the template).  The members of
    query i are the points j whose float32 key sqdist32 (the kNN key) is
    <= the float32 threshold r2, the query itself included; a_i is the
    surface variation of their covariance (1/n, centred at their mean).
    Returns (a float64, member count int64); a = NaN where there is no member
    (a non-finite query), 0 where the covariance trace is 0."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    r2 = np.float32(r2)
    n = P.shape[0]
    queries = np.arange(n) if queries is None else np.asarray(queries)
    fin = np.isfinite(P).all(axis=1)
    a = np.full(len(queries), np.nan)
    cnt = np.zeros(len(queries), dtype=np.int64)
    tree = None
    if n > 4096:
        from scipy.spatial import cKDTree

        fidx = np.flatnonzero(fin)
        tree = cKDTree(P[fidx].astype(np.float64))
        # the float32 key is within a few 1e-7 of the true squared distance,
        # so this ball holds every member
        rad = float(np.sqrt(float(r2) * (1 + 1e-5))) + 1e-30
    P64 = P.astype(np.float64)
    for r, i in enumerate(queries):
        if not fin[i]:
            continue
        if tree is None:
            cand = np.arange(n)
        else:
            cand = fidx[np.asarray(tree.query_ball_point(P64[i], rad), dtype=np.int64)]
        mem = cand[sqdist32(P[cand], P[i]) <= r2]
        cnt[r] = len(mem)
        Q = P64[mem]
        Qc = Q - Q.mean(axis=0)
        lam = np.linalg.eigvalsh(Qc.T @ Qc / len(mem))
        tr = lam.sum()
        a[r] = lam[0] / tr if tr > 0 else 0.0
    return a, cnt


def moments(P: np.ndarray):
    """Centroid, 1/n covariance and its largest eigenvalue (Sec. III-B,
    scale model)."""
    Q = P.astype(np.float64)
    c = Q.mean(axis=0)
    Qc = Q - c
    S = Qc.T @ Qc / len(Q)
    return c, S, float(np.linalg.eigvalsh(S)[-1])


# ------------------------------------------------------------ G schedule
def G_schedule(t: int, E: int, G1: float = G1_DEFAULT) -> float:
    """eq. 12, with iteration t (0-based) using G(t) = formula at t - 1."""
    return 0.1 * G1 + 0.9 * G1 / (1.0 + math.exp(-((t - 1) - E / 2.0)))


# ---------------------------------------------------------------- setup
@dataclasses.dataclass
class Setup:
    X: np.ndarray          # (N,3) float64 reference
    aX: np.ndarray         # (N,)
    aY: np.ndarray         # (M,)
    wX: np.ndarray         # (N,) reference masses
    mY: np.ndarray         # (M,) template masses
    lamX: float
    L: float
    abar: float
    sigma: float
    Z: float
    prm: Params


def make_setup(X, Y0, prm: Params, aX=None, aY=None, wX=None, mY=None) -> Setup:
    X = np.asarray(X, dtype=np.float64)
    if aX is None:
        aX = descriptors(np.asarray(X, dtype=np.float32), prm.k)
    if aY is None:
        aY = descriptors(np.asarray(Y0, dtype=np.float32), prm.k)
    N, M = len(X), len(Y0)
    wX = np.ones(N) if wX is None else np.asarray(wX, dtype=np.float64)
    mY = np.ones(M) if mY is None else np.asarray(mY, dtype=np.float64)
    _, _, lamX = moments(X)
    aX64 = np.asarray(aX, dtype=np.float64)
    if aX64.ndim == 2:
        # vector descriptors: sigma^2 = mean_j |a_j - abar|^2, the population
        # spread (the std of the scalar case when D = 1); g_mode 1 needs a
        # scalar curvature
        if prm.g_mode == 1:
            raise ValueError("g_mode 1 needs scalar descriptors")
        spread = float(np.sqrt(np.mean(np.sum((aX64 - aX64.mean(axis=0)) ** 2, axis=1))))
    else:
        spread = float(np.std(aX64))
    sigma = prm.sigma if prm.sigma > 0 else spread
    return Setup(X=X, aX=np.asarray(aX, np.float64), aY=np.asarray(aY, np.float64), wX=wX, mY=mY,
                 lamX=lamX, L=math.sqrt(lamX), abar=float(np.mean(aX)) if aX64.ndim == 1 else float("nan"),
                 sigma=sigma,
                 Z=float(wX.sum()), prm=prm)


# ---------------------------------------------------------------- forces
def pair_weights(Yi, aYi, S: Setup):
    """Per-pair factors for a block of template points: r (b,N,3),
    q = |r|^2 + eps^2 (b,N), and w_j g_ij h_ij (b,N).  eqs. 3, 5, 10, 11."""
    prm = S.prm
    r = Yi[:, None, :] - S.X[None, :, :]
    q = np.einsum("bnk,bnk->bn", r, r) + prm.eps ** 2
    if S.aX.ndim == 2:                                                        # vector descriptors
        d2 = np.zeros((len(aYi), len(S.aX)))
        for c in range(S.aX.shape[1]):
            d2 += (aYi[:, None, c] - S.aX[None, :, c]) ** 2
    else:
        d2 = (aYi[:, None] - S.aX[None, :]) ** 2
    s = np.exp(-d2 / S.sigma ** 2)                                            # eq. 3
    if prm.g_mode == 1:                                                       # eq. 10
        g = (aYi[:, None] / S.abar) * (S.aX[None, :] / S.abar) * s
    elif prm.g_mode == 2:                                                     # eq. 1: masses only
        g = np.ones_like(s)
    else:
        g = s
    h = (q / S.L ** 2) ** ((prm.p - 1) / 2.0)                                 # eqs. 4, 11
    return r, q, S.wX[None, :] * g * h


def forces(Y: np.ndarray, S: Setup, G: float, rows=None, block: int = 256):
    """f_i = -(G/Z) sum_j w_j g_ij h_ij (y_i - x_j)  (eq. 5) and the energy
    U = (G/Z) sum_ij w_j g_ij L^(1-p) q^((p+1)/2)/(p+1), whose negative
    gradient is f.  Returns (f (b,3), U)."""
    Y = np.asarray(Y, dtype=np.float64)
    rows = np.arange(len(Y)) if rows is None else np.asarray(rows)
    f = np.empty((len(rows), 3))
    U = 0.0
    p = S.prm.p
    for b0 in range(0, len(rows), block):
        rr = rows[b0:b0 + block]
        r, q, c = pair_weights(Y[rr], S.aY[rr], S)
        f[b0:b0 + block] = -(G / S.Z) * np.einsum("bn,bnk->bk", c, r)
        U += (G / S.Z) * float(np.sum(c * q)) / (p + 1)
    return f, U


def force_scale(Y: np.ndarray, S: Setup, G: float, rows=None, block: int = 256) -> np.ndarray:
    """Absolute-sum scale of each force of eq. 5: S_i = (G/Z) sum_j
    |w_j g_ij h_ij| |y_i - x_j|, the sum of the norms of the terms whose
    vector sum is f_i, so |f_i| <= S_i, with equality when all r_ij point the
    same way.  Rounding in any evaluation of f_i that adds the terms in
    another order is bounded relative to S_i, not to |f_i| (which cancels)."""
    Y = np.asarray(Y, dtype=np.float64)
    rows = np.arange(len(Y)) if rows is None else np.asarray(rows)
    out = np.empty(len(rows))
    for b0 in range(0, len(rows), block):
        rr = rows[b0:b0 + block]
        r, _, c = pair_weights(Y[rr], S.aY[rr], S)
        out[b0:b0 + block] = (G / S.Z) * np.sum(np.abs(c) * np.sqrt(np.einsum("bnk,bnk->bn", r, r)), axis=1)
    return out


def force_vjp(Y: np.ndarray, S: Setup, G: float, gf: np.ndarray, gF: np.ndarray, gK: np.ndarray, block: int = 256):
    """Gradient of L = sum_i gf_i . f_i + gF . F + sum_ab gK_ab K_ab, with
    F = sum_i m_i f_i and K = sum_i f_i (y_i - ybar)^T (ybar the unweighted
    mean), with respect to the template points, the template masses, sigma
    and eps; the curvatures are held fixed.  Written from eqs. 3, 5, 11:
    with lambda_i = dL/df_i = gf_i + m_i gF + gK (y_i - ybar) and
    c_ij = w_j g_ij h_ij,
      dL/dy_i = -(G/Z) sum_j c_ij [lambda_i + (p-1) (r_ij . lambda_i) r_ij / q_ij]
                + gK^T (f_i - fbar)                   (K's lever arm),
      dL/dm_i = gF . f_i,
      dL/dsigma = -(G/Z) sum_ij c_ij (dln g/dsigma) (r_ij . lambda_i),
                  dln g/dsigma = 2 (a_i - a_j)^2 / sigma^3 (0 when g = 1),
      dL/deps = -(G/Z) sum_ij c_ij (p-1) eps / q_ij (r_ij . lambda_i).
    FP64, blocks of template rows.  Returns (gY (M,3), gm (M,), gsigma, geps)."""
    Y = np.asarray(Y, dtype=np.float64)
    prm = S.prm
    p, eps = prm.p, prm.eps
    f, _ = forces(Y, S, G, block=block)
    ybar = Y.mean(axis=0)
    lam = np.asarray(gf, np.float64) + S.mY[:, None] * np.asarray(gF, np.float64)[None, :] + \
        (Y - ybar) @ np.asarray(gK, np.float64).T
    gY = np.empty_like(Y)
    gs = ge = 0.0
    k = -(G / S.Z)
    for b0 in range(0, len(Y), block):
        rr = slice(b0, b0 + block)
        r, q, c = pair_weights(Y[rr], S.aY[rr], S)
        lr = np.einsum("bnk,bk->bn", r, lam[rr])                          # r_ij . lambda_i
        gY[rr] = k * (c.sum(axis=1)[:, None] * lam[rr] + (p - 1) * np.einsum("bn,bnk->bk", c * lr / q, r))
        if prm.g_mode != 2:
            if S.aX.ndim == 2:
                d2 = ((S.aY[rr][:, None, :] - S.aX[None, :, :]) ** 2).sum(axis=2)
            else:
                d2 = (S.aY[rr][:, None] - S.aX[None, :]) ** 2
            gs += k * float(np.sum(c * lr * 2.0 * d2 / S.sigma ** 3))
        ge += k * float(np.sum(c * lr * (p - 1) * eps / q))
    gY += (f - f.mean(axis=0)) @ np.asarray(gK, np.float64)
    gm = f @ np.asarray(gF, np.float64)
    return gY, gm, gs, ge


# ------------------------------------------------------------ rigid update
def kabsch(Yc: np.ndarray, YD: np.ndarray):
    """eq. 6: C = Y_D^T Y = U S V^T, d = sign det(V U^T), R = V diag(1,1,d) U^T.
    A zero determinant counts as positive."""
    C = YD.T @ Yc
    U, _, Vt = np.linalg.svd(C)
    V = Vt.T
    d = 1.0 if np.linalg.det(V @ U.T) >= 0 else -1.0
    return V @ np.diag([1.0, 1.0, d]) @ U.T, C


@dataclasses.dataclass
class StepOut:
    Y: np.ndarray       # Y(t+1)
    f: np.ndarray       # per-point force at Y(t)
    F: np.ndarray       # sum_i m_i f_i
    K: np.ndarray       # sum_i f_i (y_i - ybar)^T
    U: float
    G: float
    R: np.ndarray       # Kabsch rotation (row convention)
    c: float            # scale factor
    d: np.ndarray       # translation
    C: np.ndarray       # cross-covariance


def step(Y: np.ndarray, S: Setup, t: int, d_prev=None, force_fn=None) -> StepOut:
    """One iteration of Sec. III: forces (eq. 5), Newtonian translation
    (eq. 5.5), Kabsch rotation (eq. 6), eigenvalue scale (eq. 8), update
    (eq. 9), with G from eq. 12.  Velocity (eq. 5.5's v^X, eq. 1's friction
    -eta v): the template's velocity in the previous iteration is its
    translation then, d_prev, of which the share mu = prm.momentum is carried
    (mu = 1 - the friction's share); every point moves by it, so it shifts Y_D
    as a whole and leaves the rotation unchanged.  mu = 0 or d_prev None is
    the paper's v = 0.  force_fn(Y, S, G) -> (f, U) replaces forces() (the
    same quantities evaluated another way, e.g. forces_from_sums)."""
    prm = S.prm
    G = G_schedule(t, prm.E, prm.G1)
    dt2 = prm.dt2 if prm.dt2 > 0 else 1.0 / prm.G1
    f, U = forces(Y, S, G) if force_fn is None else force_fn(Y, S, G)
    carry = prm.momentum * np.asarray(d_prev, np.float64) if d_prev is not None else np.zeros(3)
    delta = dt2 * f + carry                           # per-point displacement
    F = (S.mY[:, None] * f).sum(axis=0)
    d = dt2 * F / S.mY.sum() + carry                  # eq. 5.5
    ybar = Y.mean(axis=0)
    Yc = Y - ybar
    YD = (Y + delta) - (Y + delta).mean(axis=0)
    R, C = kabsch(Yc, YD)                             # eq. 6
    lamY = float(np.linalg.eigvalsh(Yc.T @ Yc / len(Y))[-1])
    c = math.sqrt(S.lamX / lamY)                      # eq. 8
    Ynew = c * Yc @ R + ybar + d                      # eq. 9
    K = f.T @ Yc                                      # sum_i f_i (y_i - ybar)^T
    return StepOut(Y=Ynew, f=f, F=F, K=K, U=U, G=G, R=R, c=c, d=d, C=C)


@dataclasses.dataclass
class Pose:
    """T(y) = s R y + t (column vectors)."""
    s: float
    R: np.ndarray
    t: np.ndarray

    @staticmethod
    def identity():
        return Pose(1.0, np.eye(3), np.zeros(3))

    def apply(self, P):
        return self.s * np.asarray(P, np.float64) @ self.R.T + self.t

    def as_array(self):
        return np.concatenate([[self.s], self.R.reshape(-1), self.t])


def compose(pose: Pose, so: StepOut, ybar: np.ndarray) -> Pose:
    """Fold one update y' = c R^T (y - ybar) + ybar + d into the pose."""
    Rt = so.R.T
    return Pose(so.c * pose.s, Rt @ pose.R, so.c * Rt @ (pose.t - ybar) + ybar + so.d)


def register(Y0, S: Setup, E=None, pose0: Pose | None = None, t0: int = 0, keep=False, force_fn=None):
    """E iterations from Y0 (optionally pre-posed).  Returns the final pose
    (mapping the input template onto the registered one), the final points,
    and (if keep) the per-iteration StepOut list.  force_fn: as in step()."""
    E = S.prm.E if E is None else E
    pose = Pose.identity() if pose0 is None else pose0
    Y = pose.apply(Y0)
    hist = []
    d_prev = None                                     # the template starts at rest
    for t in range(t0, t0 + E):
        ybar = Y.mean(axis=0)
        so = step(Y, S, t, d_prev, force_fn=force_fn)
        pose = compose(pose, so, ybar)
        Y = so.Y
        d_prev = so.d
        if keep:
            hist.append(so)
    return pose, Y, hist


def register_p1(Y0, S: Setup, E=None, pose0: Pose | None = None, keep=False, sums=None):
    """register() for p = 1 with the forces from the pose-independent pair
    sums (pair_sums_c, formed once): the same iteration, O(M) per step
    after an O(MN) start.  Returns (pose, Y, hist, sums)."""
    sums = pair_sums_c(S) if sums is None else sums
    pose, Y, hist = register(Y0, S, E=E, pose0=pose0, keep=keep,
                             force_fn=lambda Yt, S_, G: forces_from_sums(Yt, S_, G, sums))
    return pose, Y, hist, sums


# ------------------------------------------------------- pyramidal schedule
@dataclasses.dataclass
class Level:
    """One level of the pyramidal schedule (Sec. IV, for noisy data: the
    neighbourhood and sigma shrink with the iterations).  radius_scale > 0:
    radius neighbourhoods of radius radius_scale * sqrt(lambda_max) of each
    cloud's own covariance; 0: the k nearest neighbours.  sigma_scale
    multiplies the level's sigma (the explicit one, else the std of the
    level's reference curvatures)."""
    radius_scale: float
    sigma_scale: float
    iters: int
    k: int = 16


def level_descriptors(P: np.ndarray, lev: Level) -> np.ndarray:
    """Curvatures of cloud P for one level; the float32 radius threshold is
    float32((radius_scale * radius_scale) * lambda_max)."""
    if lev.radius_scale > 0:
        lam = moments(P)[2]
        return radius_descriptors(P, np.float32((lev.radius_scale * lev.radius_scale) * lam))[0]
    return descriptors(P, lev.k)


def register_pyramid(X, Y0, prm: Params, levels, pose0: Pose | None = None, wX=None, mY=None):
    """Registration through the levels in order: each level recomputes both
    clouds' curvatures and sigma, then runs its iterations from the pose the
    previous level reached.  The iteration count t runs on over the levels, so
    the G schedule of eq. 12 spans E = the sum of the levels' iterations."""
    if sum(lev.iters for lev in levels) != prm.E:
        raise ValueError("the levels' iterations must add up to E")
    pose = Pose.identity() if pose0 is None else pose0
    t0 = 0
    for lev in levels:
        S = make_setup(X, Y0, prm, aX=level_descriptors(X, lev), aY=level_descriptors(Y0, lev), wX=wX, mY=mY)
        S.sigma *= lev.sigma_scale
        pose, _, _ = register(Y0, S, E=lev.iters, pose0=pose, t0=t0)
        t0 += lev.iters
    return pose


# ---------------------------------------------------------------- metrics
def pose_rmse(pose: Pose, Y0, gt_s, gt_R, gt_t, corr=None) -> float:
    """sqrt(mean |T_est(y) - T_gt^{-1}(y)|^2) over inlier template points."""
    Y0 = np.asarray(Y0, np.float64)
    if corr is not None:
        Y0 = Y0[np.asarray(corr) >= 0]
    inv = (Y0 - gt_t) @ gt_R / gt_s
    return float(np.sqrt(np.mean(np.sum((pose.apply(Y0) - inv) ** 2, axis=1))))


def residual_corr(pose: Pose, Y0, X, corr) -> float:
    """sqrt(mean |T(y_i) - x_corr(i)|^2) over i with corr >= 0."""
    corr = np.asarray(corr)
    sel = corr >= 0
    D = pose.apply(np.asarray(Y0, np.float64)[sel]) - np.asarray(X, np.float64)[corr[sel]]
    return float(np.sqrt(np.mean(np.sum(D * D, axis=1))))


def residual_nn(pose: Pose, Y0, X) -> float:
    """One-sided nearest-neighbour RMSE, template -> reference, in float64."""
    from scipy.spatial import cKDTree

    d, _ = cKDTree(np.asarray(X, np.float64)).query(pose.apply(Y0))
    return float(np.sqrt(np.mean(d * d)))


def diameter(X) -> float:
    """Bounding-box diagonal of a cloud."""
    X = np.asarray(X, np.float64)
    return float(np.linalg.norm(X.max(axis=0) - X.min(axis=0)))


# ----------------------------------------------------- C loops (same maths)
_LIB = None


def _clib():
    global _LIB
    if _LIB is None:
        import ctypes

        from .build import build

        _LIB = ctypes.CDLL(build(force=False))
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        _LIB.ora_forces.argtypes = [I64, I64, P, P, P, P, P, D, ctypes.c_int, D, D, D, D, D, D, P, P, P]
        _LIB.ora_knn.argtypes = [I64, P, ctypes.c_int, I64, P, P]
        _LIB.ora_pair_sums.argtypes = [I64, I64, P, P, P, P, ctypes.c_int, D, D, P]
        _LIB.ora_threads.restype = ctypes.c_int
        _LIB.ora_set_threads.argtypes = [ctypes.c_int]
    return _LIB


def c_threads(n=None) -> int:
    """Thread count of the C loops; sets it first when n is given."""
    if n is not None:
        _clib().ora_set_threads(int(n))
    return int(_clib().ora_threads())


def _ptr(a):
    import ctypes

    return a.ctypes.data_as(ctypes.c_void_p)


def forces_c(Y: np.ndarray, S: Setup, G: float, rows=None, want_scale: bool = False):
    """forces() evaluated by the plain C loops (OpenMP); same definition.
    With want_scale, also force_scale() of the same rows: (f, U, scale)."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    aY = np.ascontiguousarray(S.aY)
    if rows is not None:
        rows = np.asarray(rows)
        Y = np.ascontiguousarray(Y[rows])
        aY = np.ascontiguousarray(aY[rows])
    X = np.ascontiguousarray(S.X)
    f = np.empty((len(Y), 3))
    U = np.zeros(1)
    sc = np.empty(len(Y)) if want_scale else None
    prm = S.prm
    _clib().ora_forces(len(Y), len(X), _ptr(Y), _ptr(aY), _ptr(X), _ptr(np.ascontiguousarray(S.aX)),
                       _ptr(np.ascontiguousarray(S.wX)), float(prm.p), int(prm.g_mode), S.sigma,
                       float(prm.eps), S.L, S.abar, float(G), S.Z, _ptr(f), _ptr(U),
                       _ptr(sc) if want_scale else None)
    if want_scale:
        return f, float(U[0]), sc
    return f, float(U[0])


def pair_sums_c(S: Setup) -> np.ndarray:
    """For p = 1 (h = 1) the pair weights c_ij = w_j g_ij of eq. 5 do not
    depend on the pose, so per template row the sums S0 = sum_j c_ij,
    Sx = sum_j c_ij x_j (3) and Sxx = sum_j c_ij |x_j|^2 hold for every
    iterate (C loops).  Returns (M, 5)."""
    if S.prm.p != 1.0:
        raise ValueError("pose-independent pair sums need p = 1")
    aY = np.ascontiguousarray(S.aY, dtype=np.float64)
    X = np.ascontiguousarray(S.X, dtype=np.float64)
    out = np.empty((len(aY), 5))
    _clib().ora_pair_sums(len(aY), len(X), _ptr(aY), _ptr(X), _ptr(np.ascontiguousarray(S.aX, dtype=np.float64)),
                          _ptr(np.ascontiguousarray(S.wX, dtype=np.float64)), int(S.prm.g_mode), float(S.sigma),
                          float(S.abar), _ptr(out))
    return out


def forces_from_sums(Y: np.ndarray, S: Setup, G: float, sums: np.ndarray):
    """forces() at p = 1 from pair_sums_c: f_i = -(G/Z) (y_i S0_i - Sx_i)
    and U = (G/Z) sum_i [(|y_i|^2 + eps^2) S0_i - 2 y_i . Sx_i + Sxx_i] / 2,
    i.e. eq. 5 and its energy with the sum over the reference taken first."""
    Y = np.asarray(Y, np.float64)
    f = -(G / S.Z) * (Y * sums[:, 0:1] - sums[:, 1:4])
    q = (np.sum(Y * Y, axis=1) + S.prm.eps ** 2) * sums[:, 0] - 2.0 * np.sum(Y * sums[:, 1:4], axis=1) + sums[:, 4]
    return f, (G / S.Z) * float(np.sum(q)) / 2.0


def knn_c(P: np.ndarray, k: int, queries=None) -> np.ndarray:
    """knn_bruteforce() evaluated by the plain C loops; same definition."""
    P = np.ascontiguousarray(P, dtype=np.float32)
    q = np.arange(len(P), dtype=np.int64) if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    out = np.empty((len(q), k), dtype=np.int64)
    _clib().ora_knn(len(P), _ptr(P), int(k), len(q), _ptr(q), _ptr(out))
    return out


# ------------------------------------------------------- change detection
def posed32(Y0, pose: "Pose") -> np.ndarray:
    """T(y) = s R y + t in FP64 with every operation rounded on its own, in
    the order s ((R_r0 y_0 + R_r1 y_1) + R_r2 y_2) + t_r, then rounded to
    float32: the posed template on which change detection decides."""
    Y = np.asarray(Y0, np.float32).astype(np.float64)
    out = np.empty_like(Y)
    for r in range(3):
        a = pose.R[r, 0] * Y[:, 0]
        b = pose.R[r, 1] * Y[:, 1]
        c = pose.R[r, 2] * Y[:, 2]
        out[:, r] = pose.s * ((a + b) + c) + pose.t[r]
    return out.astype(np.float32)


def nearest(Q: np.ndarray, X: np.ndarray):
    """Nearest row of X to each row of Q by (float32 key of sqdist32, index).
    Candidates from a float64 k-d tree are ranked by the key; a query whose
    best key is not clearly inside the candidate radius is redone by brute
    force, so the result is exact.  Non-finite queries: (-1, inf)."""
    Q = np.ascontiguousarray(Q, dtype=np.float32)
    X = np.ascontiguousarray(X, dtype=np.float32)
    nq = Q.shape[0]
    nn = np.full(nq, -1, dtype=np.int64)
    key = np.full(nq, np.inf, dtype=np.float32)
    ok = np.isfinite(Q).all(axis=1)
    idx_all = np.arange(X.shape[0])

    def brute(i):
        d = sqdist32(X, Q[i])
        j = int(np.lexsort((idx_all, d))[0])
        return j, d[j]

    if X.shape[0] <= 64:
        for i in np.nonzero(ok)[0]:
            nn[i], key[i] = brute(i)
        return nn, key
    from scipy.spatial import cKDTree

    tree = cKDTree(X.astype(np.float64))
    kk = min(8, X.shape[0])
    qi = np.nonzero(ok)[0]
    dd, cand = tree.query(Q[qi].astype(np.float64), k=kk)
    # float32 keys of all candidates, in the same operation order as sqdist32
    d = X[cand] - Q[qi][:, None, :]
    k32 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    o = np.lexsort((cand, k32), axis=-1)[:, 0]      # primary key, ties by index
    rows = np.arange(len(qi))
    best, bidx = k32[rows, o], cand[rows, o]
    # every point outside the candidate set lies at float64 distance
    # >= dd[:, -1]; float32 rounding moves keys by far less unless the radii
    # nearly coincide, in which case the query is redone by brute force
    clear = best.astype(np.float64) * (1 + 1e-5) + 1e-30 < dd[:, -1] ** 2
    nn[qi[clear]], key[qi[clear]] = bidx[clear], best[clear]
    for i in qi[~clear]:
        nn[i], key[i] = brute(i)
    return nn, key


def change_flags(Y0, aY, X, aX, pose: "Pose", tau: float, sigma: float, s_min: float):
    """Change detection after registration (Sec. I and IV: registered
    template parts without a similar reference part nearby).  Per template
    point, with j its nearest reference point to the posed point among
    those with float32 key <= float32(tau^2): bit 0: there is none (nn -1,
    key +inf); bit 1 (s_min > 0): (a_i - a_j)^2 in FP64 > sigma^2 (-ln
    s_min), i.e. the shape similarity of eq. 3 is below s_min.  Returns
    (flags uint8, nn int64, key float32)."""
    Q = posed32(Y0, pose)
    nn, key = nearest(Q, X)
    tau2 = np.float32(tau * tau)
    far = ~(key <= tau2)
    nn[far] = -1
    key[far] = np.inf
    thr = sigma * sigma * (-math.log(s_min)) if s_min > 0 else math.inf
    flags = np.zeros(len(Q), dtype=np.uint8)
    valid = nn >= 0
    flags[~valid] = 1
    da = np.asarray(aY, np.float32).astype(np.float64) - np.asarray(aX, np.float32).astype(np.float64)[np.maximum(nn, 0)]
    flags[valid & (da * da > thr)] |= 2
    return flags, nn, key
