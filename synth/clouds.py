"""Seeded synthetic point clouds for the five registration workloads.

This module only draws inputs: surfaces, rigid/similarity transforms applied
to make templates, noise and outliers.  It holds none of the registration
method's arithmetic, so both the FP64 oracle and the HIP path may use it.

Seeds follow one rule: ``seed = 1000 * workload + role`` with roles
0 surface, 1 template transform, 2 noise, 3 outliers, 4 crop / multi-start.

Every generator returns a ``Pair`` of float32 arrays: ``ref`` (N x 3),
``tmpl`` (M x 3), the ground-truth similarity ``gt = (s, R, t)`` that maps
the reference frame to the template frame (``y = s R x + t``), and ``corr``
(int32, M): the reference index each template point was made from, or -1
for an outlier / a point with no counterpart.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Pair:
    name: str
    ref: np.ndarray          # (N, 3) float32
    tmpl: np.ndarray         # (M, 3) float32
    gt_s: float
    gt_R: np.ndarray         # (3, 3) float64
    gt_t: np.ndarray         # (3,) float64
    corr: np.ndarray         # (M,) int32
    k: int                   # neighbourhood size for the local descriptor
    iters: int               # iteration count E
    g_mode: int = 0          # 0: g = s, 1: g = a a s
    p: int = 2
    eps_rel: float = 0.0     # softening as a fraction of the cloud length scale
    changed: np.ndarray | None = None      # (M,) bool: template point on an object absent from the reference
    ref_changed: np.ndarray | None = None  # (N,) bool: reference point on an object absent from the template

    @property
    def N(self) -> int:
        return int(self.ref.shape[0])

    @property
    def M(self) -> int:
        return int(self.tmpl.shape[0])


# ---------------------------------------------------------------- rotations
def rot_axis_angle(axis, deg: float) -> np.ndarray:
    """Rodrigues rotation matrix (column convention) about ``axis``."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    th = math.radians(deg)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * (K @ K)


def random_unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def quat_to_R(q) -> np.ndarray:
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def super_fibonacci_rotations(n: int) -> np.ndarray:
    """n near-uniform rotations of SO(3): the super-Fibonacci spiral of
    Alexa (CVPR 2022).  Returns (n, 3, 3) float64."""
    phi = math.sqrt(2.0)
    psi = 1.533751168755204288118041  # real root of psi^4 = psi + 4
    out = np.empty((n, 3, 3))
    for i in range(n):
        s = i + 0.5
        r = math.sqrt(s / n)
        R = math.sqrt(1.0 - s / n)
        alpha = 2 * math.pi * s / phi
        beta = 2 * math.pi * s / psi
        q = (r * math.sin(alpha), r * math.cos(alpha), R * math.sin(beta), R * math.cos(beta))
        out[i] = quat_to_R(q)
    return out


# ---------------------------------------------------------------- surfaces
def ellipsoid_patch(n: int, seed: int, axes=(1.0, 0.6, 0.4), patch=(1.0, 0.8)) -> np.ndarray:
    """Ellipsoid (semi-axes ``axes``) fused with a planar patch tangent at its
    bottom (z = -c), sampled uniformly by area.  Points are split between the
    two parts in proportion to area (ellipsoid area by Thomsen's formula)."""
    rng = np.random.default_rng(seed)
    a, b, c = axes
    pp = 1.6075
    area_e = 4 * math.pi * (((a * b) ** pp + (a * c) ** pp + (b * c) ** pp) / 3) ** (1 / pp)
    area_p = patch[0] * patch[1]
    n_e = int(round(n * area_e / (area_e + area_p)))
    n_p = n - n_e
    pts = []
    gmax = max(b * c, a * c, a * b)
    got = 0
    while got < n_e:
        u = rng.normal(size=(2 * (n_e - got) + 64, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        g = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
        keep = rng.uniform(size=len(u)) * gmax < g
        sel = u[keep][: n_e - got] * np.array([a, b, c])
        pts.append(sel)
        got += len(sel)
    px = rng.uniform(-patch[0] / 2, patch[0] / 2, size=n_p)
    py = rng.uniform(-patch[1] / 2, patch[1] / 2, size=n_p)
    pts.append(np.stack([px, py, np.full(n_p, -c)], axis=1))
    return np.concatenate(pts, axis=0)


def _real_sph_harm(l: int, m: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    from scipy.special import lpmv

    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    P = lpmv(am, l, np.cos(theta))
    if m == 0:
        return norm * P
    if m > 0:
        return math.sqrt(2) * norm * P * np.cos(am * phi)
    return math.sqrt(2) * norm * P * np.sin(am * phi)


def sh_surface(n: int, seed: int, lmax: int = 6, amp: float = 0.15) -> np.ndarray:
    """Closed radial surface r(theta, phi) = 1 + sum_{l<=lmax} c_lm Y_lm with
    c_lm ~ N(0, (amp/l)^2), r clipped at 0.5; directions uniform on S^2."""
    rng = np.random.default_rng(seed)
    coef = {(l, m): rng.normal(0.0, amp / l) for l in range(1, lmax + 1) for m in range(-l, l + 1)}
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    theta = np.arccos(np.clip(u[:, 2], -1, 1))
    phi = np.arctan2(u[:, 1], u[:, 0])
    r = np.ones(n)
    for (l, m), cl in coef.items():
        r += cl * _real_sph_harm(l, m, theta, phi)
    r = np.maximum(r, 0.5)
    return u * r[:, None]


# ------------------------------------------------------------- templates
def _apply(s, R, t, p):
    return s * p @ R.T + t


def _pair(name, ref, tmpl, s, R, t, corr, **kw) -> Pair:
    return Pair(name=name, ref=np.ascontiguousarray(ref, dtype=np.float32),
                tmpl=np.ascontiguousarray(tmpl, dtype=np.float32), gt_s=float(s),
                gt_R=np.asarray(R, dtype=np.float64), gt_t=np.asarray(t, dtype=np.float64),
                corr=np.asarray(corr, dtype=np.int32), **kw)


def config1(n: int = 1024, noise: float = 0.005, wl: int = 1, iters: int = 100, k: int = 16) -> Pair:
    """Tiny plain-method pair: ellipsoid + patch, template = 1.2 R_x(50deg) x
    + (0.3, -0.2, 0.1) + N(0, noise^2)."""
    ref = ellipsoid_patch(n, 1000 * wl + 0)
    R = rot_axis_angle([1, 0, 0], 50.0)
    s, t = 1.2, np.array([0.3, -0.2, 0.1])
    rng = np.random.default_rng(1000 * wl + 2)
    tmpl = _apply(s, R, t, ref) + rng.normal(0.0, noise, size=ref.shape) if noise > 0 else _apply(s, R, t, ref)
    return _pair(f"ellipsoid+patch {n}x{n}", ref, tmpl, s, R, t, np.arange(n), k=k, iters=iters)


def config2(n: int = 36000, wl: int = 2, iters: int = 300, k: int = 24) -> Pair:
    """Scan-sized pair: spherical-harmonic surface; template drops a 25% cap,
    adds a 15% Gaussian blob (sd 0.1 at 0.8 v) and 5% uniform bbox outliers,
    then 0.8 R(60deg, random axis) and noise sd 0.003."""
    ref = sh_surface(n, 1000 * wl + 0)
    rng_c = np.random.default_rng(1000 * wl + 4)
    u = random_unit(rng_c)
    dirs = ref / np.linalg.norm(ref, axis=1, keepdims=True)
    order = np.argsort(dirs @ u, kind="stable")
    keep = np.sort(order[: n - n // 4])
    rng_o = np.random.default_rng(1000 * wl + 3)
    v = random_unit(rng_o)
    n_blob = int(round(0.15 * len(keep)))   # outlier shares are of the kept part
    n_uni = int(round(0.05 * len(keep)))
    blob = 0.8 * v + rng_o.normal(0.0, 0.1, size=(n_blob, 3))
    lo, hi = ref.min(axis=0), ref.max(axis=0)
    uni = rng_o.uniform(lo, hi, size=(n_uni, 3))
    pts = np.concatenate([ref[keep], blob, uni], axis=0)
    corr = np.concatenate([keep, np.full(n_blob + n_uni, -1)])
    rng_t = np.random.default_rng(1000 * wl + 1)
    R = rot_axis_angle(random_unit(rng_t), 60.0)
    s, t = 0.8, np.zeros(3)
    rng_n = np.random.default_rng(1000 * wl + 2)
    tmpl = _apply(s, R, t, pts) + rng_n.normal(0.0, 0.003, size=pts.shape)
    return _pair(f"sh-surface {len(tmpl)}x{n}", ref, tmpl, s, R, t, corr, k=k, iters=iters)


def config3(n: int = 8192) -> Pair:
    """Differentiation pair: built like the tiny pair at n = 8192, with
    softening eps = 0.05 L so its gradient is non-trivial."""
    pr = config1(n=n, wl=3, iters=50, k=16)
    pr.name = f"ellipsoid+patch {n}x{n} (adjoint)"
    pr.eps_rel = 0.05
    return pr


def _c4_one(seed_base: int, n: int, rng_t: np.random.Generator, outlier_frac=0.1, noise=0.005):
    ref = ellipsoid_patch(n, seed_base + 0)
    ang = rng_t.uniform(0.0, 90.0)
    R = rot_axis_angle(random_unit(rng_t), ang)
    t = rng_t.uniform(-0.5, 0.5, size=3)
    s = rng_t.uniform(0.7, 1.4)
    rng_o = np.random.default_rng(seed_base + 3)
    n_out = int(round(outlier_frac * n))
    lo, hi = ref.min(axis=0), ref.max(axis=0)
    pts = np.concatenate([ref, rng_o.uniform(lo, hi, size=(n_out, 3))], axis=0)
    rng_n = np.random.default_rng(seed_base + 2)
    tmpl = _apply(s, R, t, pts) + rng_n.normal(0.0, noise, size=pts.shape)
    corr = np.concatenate([np.arange(n), np.full(n_out, -1)])
    return ref, tmpl, s, R, t, corr


def config4(B: int = 256, nmin: int = 2000, nmax: int = 40000, wl: int = 4, iters: int = 100):
    """Batch of B uneven registrations, N_r log-uniform in [nmin, nmax],
    M_r = 1.1 N_r (10% uniform outliers), random rotation 0-90 deg,
    translation U(-0.5, 0.5)^3, scale U(0.7, 1.4), noise sd 0.005."""
    rng = np.random.default_rng(1000 * wl + 4)
    sizes = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=B))).astype(int)
    out = []
    for r, n in enumerate(sizes):
        rng_t = np.random.default_rng(1000 * wl + 1 + 10 * (r + 1))
        ref, tmpl, s, R, t, corr = _c4_one(100000 * wl + 10 * (r + 1), int(n), rng_t)
        out.append(_pair(f"batch[{r}] {len(tmpl)}x{n}", ref, tmpl, s, R, t, corr, k=16, iters=iters))
    return out


def config4_multistart(n: int = 20000, S: int = 32, wl: int = 4, iters: int = 100):
    """One 20k cloud (template 22k with 10% outliers) under a large seeded
    rotation, plus S super-Fibonacci initial rotations."""
    rng_t = np.random.default_rng(1000 * wl + 7)
    ref = ellipsoid_patch(n, 1000 * wl + 5)
    R = rot_axis_angle(random_unit(rng_t), 150.0)
    t = rng_t.uniform(-0.5, 0.5, size=3)
    s = 1.1
    rng_o = np.random.default_rng(1000 * wl + 3)
    n_out = int(round(0.1 * n))
    lo, hi = ref.min(axis=0), ref.max(axis=0)
    pts = np.concatenate([ref, rng_o.uniform(lo, hi, size=(n_out, 3))], axis=0)
    rng_n = np.random.default_rng(1000 * wl + 2)
    tmpl = _apply(s, R, t, pts) + rng_n.normal(0.0, 0.005, size=pts.shape)
    corr = np.concatenate([np.arange(n), np.full(n_out, -1)])
    pr = _pair(f"multistart {len(tmpl)}x{n}", ref, tmpl, s, R, t, corr, k=16, iters=iters)
    return pr, super_fibonacci_rotations(S)


# ------------------------------------------------------------- depth room
def _raycast_room(dirs: np.ndarray, boxes, room_lo, room_hi, want_id: bool = False):
    """Distance along each unit ray (from the origin) to the first surface
    of a closed axis-aligned room containing axis-aligned boxes (and, with
    want_id, the index of the box hit, -1 for the room)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dirs
        t1 = (room_lo - 0.0) * inv
        t2 = (room_hi - 0.0) * inv
        tfar = np.nanmin(np.maximum(t1, t2), axis=1)  # exit of the room box
        best = tfar.copy()
        hit_id = np.full(best.shape, -1, dtype=np.int64)
        for b_i, (lo, hi) in enumerate(boxes):
            a = lo * inv
            b = hi * inv
            tn = np.nanmax(np.minimum(a, b), axis=1)
            tf = np.nanmin(np.maximum(a, b), axis=1)
            hit = (tf >= tn) & (tn > 1e-6) & (tn < best)
            best = np.where(hit, tn, best)
            hit_id = np.where(hit, b_i, hit_id)
    return (best, hit_id) if want_id else best


ROOM = ((-2.5, -1.2, -0.5), (2.5, 1.8, 3.5))   # 5 x 3 x 4 m, camera 1.2 m above the floor


def _room_boxes(rng: np.random.Generator, count: int, floor_y: float):
    boxes = []
    for _ in range(count):
        sx, sy, sz = rng.uniform(0.2, 0.8, size=3)
        cx = rng.uniform(-2.0, 2.0)
        cz = rng.uniform(0.8, 3.0)
        lo = np.array([cx - sx / 2, floor_y, cz - sz / 2])
        hi = np.array([cx + sx / 2, floor_y + sy, cz + sz / 2])
        boxes.append((lo, hi))
    return boxes


def _render(boxes, cam_R, rng_noise, width=640, height=480, f=525.0, room=ROOM, want_id: bool = False):
    """Render a depth frame from a camera at the origin with orientation
    ``cam_R`` (camera-to-world), return points in the camera frame (and,
    with want_id, the box each pixel sees, -1 for the room)."""
    cx, cy = (width - 1) / 2, (height - 1) / 2
    u, v = np.meshgrid(np.arange(width), np.arange(height))
    d_cam = np.stack([(u - cx) / f, -(v - cy) / f, np.ones_like(u, dtype=np.float64)], axis=-1).reshape(-1, 3)
    z_per_len = 1.0 / np.linalg.norm(d_cam, axis=1)
    dirs_cam = d_cam * z_per_len[:, None]
    dirs_w = dirs_cam @ cam_R.T
    lo, hi = np.array(room[0]), np.array(room[1])
    dist, hit_id = _raycast_room(dirs_w, boxes, lo, hi, want_id=True)
    z = dist * z_per_len
    z = z + rng_noise.normal(0.0, 1.0, size=z.shape) * 0.001 * z * z
    pts = d_cam * z[:, None]
    return (pts, hit_id) if want_id else pts


def _visible_pixels(boxes, cam_R, idx, width=640, height=480, f=525.0, room=ROOM) -> int:
    """Number of pixels of a depth frame that see box ``idx``."""
    cx, cy = (width - 1) / 2, (height - 1) / 2
    u, v = np.meshgrid(np.arange(width), np.arange(height))
    d_cam = np.stack([(u - cx) / f, -(v - cy) / f, np.ones_like(u, dtype=np.float64)], axis=-1).reshape(-1, 3)
    dirs_w = (d_cam / np.linalg.norm(d_cam, axis=1)[:, None]) @ cam_R.T
    _, hit_id = _raycast_room(dirs_w, boxes, np.array(room[0]), np.array(room[1]), want_id=True)
    return int(np.count_nonzero(hit_id == idx))


def config5(wl: int = 5, iters: int = 100, m: int = 250000) -> Pair:
    """Depth-frame pair: a 5x4x3 m room with 20 floor boxes rendered at
    640x480 (fx = fy = 525) with depth noise sd 0.001 z^2; the template is
    the same room with one box removed and two added, seen from the camera
    turned 30 deg about the vertical axis, subsampled to ``m`` points."""
    rng = np.random.default_rng(1000 * wl + 0)
    floor_y = ROOM[0][1]
    boxes = _room_boxes(rng, 20, floor_y)
    pitch = rot_axis_angle([1, 0, 0], 20.0)  # both views look 20 deg down (+y is up, the floor at y = -1.2)
    ref, ref_id = _render(boxes, pitch, np.random.default_rng(1000 * wl + 2), want_id=True)
    rng_c = np.random.default_rng(1000 * wl + 3)
    boxes2 = list(boxes)
    removed = int(rng_c.integers(len(boxes2)))
    boxes2.pop(removed)
    Rc = rot_axis_angle([0, 1, 0], 30.0) @ pitch  # camera-to-world of the second view
    # two added boxes, each drawn until it overlaps no other box and at least
    # 2000 pixels of the second view see it (so the change is observable)
    for _ in range(2):
        while True:
            cand = _room_boxes(rng_c, 1, floor_y)[0]
            overlap = any(np.all(cand[0][[0, 2]] < hi[[0, 2]]) and np.all(lo[[0, 2]] < cand[1][[0, 2]])
                          for lo, hi in boxes2)
            if not overlap and _visible_pixels(boxes2 + [cand], Rc, len(boxes2)) >= 2000:
                boxes2.append(cand)
                break
    tm, tm_id = _render(boxes2, Rc, np.random.default_rng(1000 * wl + 12), want_id=True)
    rng_s = np.random.default_rng(1000 * wl + 4)
    sel = np.sort(rng_s.choice(tm.shape[0], size=m, replace=False))
    tmpl = tm[sel]
    # ground-truth change labels: template points on the two added boxes,
    # reference points on the removed one
    changed = tm_id[sel] >= len(boxes2) - 2
    ref_changed = ref_id == removed
    # reference camera -> world -> second camera: y = Rc^T pitch x
    return _pair(f"depth-room {m}x{ref.shape[0]}", ref, tmpl, 1.0, Rc.T @ pitch, np.zeros(3),
                 np.full(m, -1), k=16, iters=iters, g_mode=1, changed=changed, ref_changed=ref_changed)


def random_pair(M: int, N: int, seed: int, spread: float = 1.0) -> Pair:
    """Small unstructured pair for unit tests: Gaussian blobs."""
    rng = np.random.default_rng(seed)
    ref = rng.normal(size=(N, 3)) * np.array([1.0, 0.7, 0.4]) * spread
    tmpl = rng.normal(size=(M, 3)) * np.array([0.9, 0.6, 0.5]) * spread + 0.2
    return _pair(f"random {M}x{N}", ref, tmpl, 1.0, np.eye(3), np.zeros(3), np.full(M, -1), k=8, iters=10)


WORKLOADS = {1: config1, 2: config2, 3: config3, 5: config5}
