"""Shape-constrained gravitational point-cloud registration on MI355X.

Thin Python binding over the C ABI of ``include/sgreg.h``: it only moves
arguments (torch tensors for device memory, torch's current stream).  Every
step of the computation runs in the HIP kernels of ``libsgreg.so``; there is
no CPU fallback, and importing fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _ffi
from ._ffi import SgrCloud, SgrError, SgrParams, check, lib

__all__ = ["Params", "Cloud", "Context", "Plan", "ForceField", "UnrolledRegistration", "SgrError", "pose_identity",
           "pose_inverse", "pose_to_srt", "pose_from_srt"]

lib()  # fail at import when the native library is absent


@dataclasses.dataclass
class Params:
    """Method parameters (see include/sgreg.h for the reading of each)."""
    p: float = 1.0
    g_mode: int = 0
    k: int = 16
    sigma: float = 0.0
    eps: float = 0.0
    G1: float = 10000.0
    E: int = 100
    flags: int = 0
    dt2: float = 0.0
    momentum: float = 0.0

    def c(self) -> SgrParams:
        return SgrParams(float(self.p), int(self.g_mode), int(self.k), float(self.sigma), float(self.eps),
                         float(self.G1), int(self.E), int(self.flags), float(self.dt2), float(self.momentum))


@dataclasses.dataclass
class Level:
    """One level of the pyramidal schedule: radius_scale > 0 selects radius
    neighbourhoods of radius radius_scale * sqrt(lambda_max) of each cloud,
    0 the k nearest neighbours; sigma_scale multiplies the level's sigma."""
    radius_scale: float
    sigma_scale: float
    iters: int
    k: int = 16


def _dev(device) -> torch.device:
    d = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    if d.type != "cuda":
        raise ValueError("sgreg runs on a HIP device only")
    if d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Cloud:
    """A point cloud in device memory as structure-of-arrays float32
    (``soa`` has shape (3, n)), with optional per-point masses."""

    def __init__(self, points, masses=None, device=None):
        dev = _dev(device)
        p = torch.as_tensor(np.asarray(points) if not torch.is_tensor(points) else points)
        if p.ndim != 2 or p.shape[1] != 3:
            raise ValueError("points must have shape (n, 3)")
        self.soa = p.to(device=dev, dtype=torch.float32).t().contiguous()
        self.m = None
        if masses is not None:
            m = torch.as_tensor(masses).to(device=dev, dtype=torch.float32).contiguous()
            if m.shape != (p.shape[0],):
                raise ValueError("masses must have shape (n,)")
            self.m = m
        self.device = dev

    @property
    def n(self) -> int:
        return int(self.soa.shape[1])

    def c(self) -> SgrCloud:
        # rows of the contiguous (3, n) array by address arithmetic (indexing
        # the tensor three times per call costs more than the call itself
        # when a batch passes hundreds of clouds)
        base, n = self.soa.data_ptr(), self.n
        return SgrCloud(base, base + 4 * n, base + 8 * n, self.m.data_ptr() if self.m is not None else None, n)


def pose_inverse(pose: torch.Tensor) -> torch.Tensor:
    """The pose of T^-1(x) = (1/s) R^T (x - t) (13 float64, same layout)."""
    s, R, t = pose[0], pose[1:10].view(3, 3), pose[10:13]
    out = torch.empty_like(pose)
    out[0] = 1.0 / s
    out[1:10] = R.T.reshape(-1)
    out[10:13] = -(R.T @ t) / s
    return out


def pose_identity(device=None) -> torch.Tensor:
    p = torch.zeros(13, dtype=torch.float64, device=_dev(device))
    p[0] = 1.0
    p[1] = p[5] = p[9] = 1.0
    return p


def pose_from_srt(s, R, t, device=None) -> torch.Tensor:
    v = np.concatenate([[float(s)], np.asarray(R, np.float64).reshape(-1), np.asarray(t, np.float64).reshape(-1)])
    return torch.tensor(v, dtype=torch.float64, device=_dev(device))


def pose_to_srt(pose: torch.Tensor):
    v = pose.detach().double().cpu().numpy()
    return float(v[0]), v[1:10].reshape(3, 3), v[10:13].copy()


class Context:
    """A library context on one HIP device (owns workspace, graphs, tiles)."""

    def __init__(self, device=0):
        self.device = _dev(device)
        h = ctypes.c_void_p()
        check(lib().sgr_create(ctypes.byref(h), self.device.index))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            lib().sgr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tiles(self, M: int, N: int, p: float, R: int, blocks_per_cu: int, variant: int = 0):
        check(lib().sgr_set_tiles(self._h, int(M), int(N), float(p), int(R), int(blocks_per_cu), int(variant)))

    def autotune(self, tmpl: Cloud, a_t, ref: Cloud, a_r, mom_t, mom_r, params: Params, reps: int = 5):
        """Time every launch shape of the force kernel on this pair and keep
        the fastest for its size bucket; returns ((R, blocks_per_cu, variant), ms)."""
        best = (ctypes.c_int * 3)()
        ms = ctypes.c_double()
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_autotune(self._h, ctypes.byref(ct), _ptr(a_t), ctypes.byref(cr), _ptr(a_r), _ptr(mom_t),
                                 _ptr(mom_r), ctypes.byref(pr), int(reps), best, ctypes.byref(ms),
                                 _stream(self.device)))
        return (best[0], best[1], best[2]), ms.value

    def save_tiles(self, path: str):
        check(lib().sgr_tiles_save(self._h, str(path).encode()))

    def load_tiles(self, path: str):
        check(lib().sgr_tiles_load(self._h, str(path).encode()))

    # -------------------------------------------------------------- calls
    def descriptors(self, cloud: Cloud, k: int):
        a = torch.empty(cloud.n, dtype=torch.float32, device=self.device)
        mom = torch.empty(10, dtype=torch.float64, device=self.device)
        c = cloud.c()
        check(lib().sgr_descriptors(self._h, ctypes.byref(c), int(k), _ptr(a), _ptr(mom), _stream(self.device)))
        return a, mom

    def descriptors_batch(self, clouds, k: int, want_idx=False):
        """Curvatures (and neighbour lists) of many clouds in one call:
        ([a_c float32 [n_c]], [idx_c int32 [n_c, k]] or None)."""
        B = len(clouds)
        sizes = [c.n for c in clouds]
        # one allocation each, handed out as per-cloud views
        a = list(torch.empty(sum(sizes), dtype=torch.float32, device=self.device).split(sizes))
        idx = (list(torch.empty((sum(sizes), k), dtype=torch.int32, device=self.device).split(sizes))
               if want_idx else None)
        cc = (SgrCloud * B)(*[c.c() for c in clouds])
        pa = (ctypes.c_void_p * B)(*[t.data_ptr() for t in a])
        pi = (ctypes.c_void_p * B)(*[t.data_ptr() for t in idx]) if want_idx else None
        check(lib().sgr_descriptors_batch(self._h, B, cc, int(k), pa, pi, _stream(self.device)))
        return a, idx

    def knn(self, cloud: Cloud, k: int) -> torch.Tensor:
        idx = torch.empty((cloud.n, k), dtype=torch.int32, device=self.device)
        c = cloud.c()
        check(lib().sgr_knn(self._h, ctypes.byref(c), int(k), _ptr(idx), _stream(self.device)))
        return idx

    def step(self, tmpl: Cloud, a_t, ref: Cloud, a_r, mom_t, mom_r, params: Params, t: int, pose_in,
             pose_out=None, want_wrench=True, want_f=False, static_scratch=False, wrench=None, f=None):
        """One iteration.  static_scratch: through sgr_step_static (no device
        allocation; the caller may also pass the output buffers)."""
        pose_out = torch.empty(13, dtype=torch.float64, device=self.device) if pose_out is None else pose_out
        if wrench is None and want_wrench:
            wrench = torch.empty(13, dtype=torch.float64, device=self.device)
        if f is None and want_f:
            f = torch.empty((tmpl.n, 3), dtype=torch.float32, device=self.device)
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        fn = lib().sgr_step_static if static_scratch else lib().sgr_step
        check(fn(self._h, ctypes.byref(ct), _ptr(a_t), ctypes.byref(cr), _ptr(a_r), _ptr(mom_t), _ptr(mom_r),
                 ctypes.byref(pr), int(t), _ptr(pose_in), _ptr(pose_out), _ptr(wrench), _ptr(f),
                 _stream(self.device)))
        return pose_out, wrench, f

    def register(self, tmpl: Cloud, ref: Cloud, params: Params, pose=None, stats=False):
        pose = pose_identity(self.device) if pose is None else pose
        st = torch.empty((params.E, 32), dtype=torch.float64, device=self.device) if stats else None
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_register(self._h, ctypes.byref(ct), ctypes.byref(cr), ctypes.byref(pr), _ptr(pose),
                                 _ptr(st), _stream(self.device)))
        return pose, st

    def force_fwd(self, tmpl: Cloud, a_t, ref: Cloud, a_r, mom_r, params: Params, G: float):
        f = torch.empty((tmpl.n, 3), dtype=torch.float32, device=self.device)
        wrench = torch.empty(13, dtype=torch.float64, device=self.device)
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_force_fwd(self._h, ctypes.byref(ct), _ptr(a_t), ctypes.byref(cr), _ptr(a_r), _ptr(mom_r),
                                  ctypes.byref(pr), float(G), _ptr(f), _ptr(wrench), _stream(self.device)))
        return f, wrench

    def force_bwd(self, tmpl: Cloud, a_t, ref: Cloud, a_r, mom_r, params: Params, G: float, f, grad_f=None,
                  grad_wrench=None, want_m=True, want_se=True):
        gy = torch.empty((tmpl.n, 3), dtype=torch.float32, device=self.device)
        gm = torch.empty(tmpl.n, dtype=torch.float32, device=self.device) if want_m else None
        gse = torch.empty(2, dtype=torch.float64, device=self.device) if want_se else None
        gf = None if grad_f is None else grad_f.to(torch.float32).contiguous()
        gw = None if grad_wrench is None else grad_wrench.to(torch.float64).contiguous()
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_force_bwd(self._h, ctypes.byref(ct), _ptr(a_t), ctypes.byref(cr), _ptr(a_r), _ptr(mom_r),
                                  ctypes.byref(pr), float(G), _ptr(f.contiguous()), _ptr(gf), _ptr(gw), _ptr(gy),
                                  _ptr(gm), _ptr(gse), _stream(self.device)))
        return gy, gm, gse

    def unrolled_fwd(self, tmpl: Cloud, a_t, ref: Cloud, a_r, mom_t, mom_r, params: Params, ckpt_every: int = 10,
                     pose=None):
        """params.E iterations with the curvatures held constant; returns the
        final pose and the pose checkpoints [ceil(E / ckpt_every), 13]."""
        pose = pose_identity(self.device) if pose is None else pose.to(self.device, torch.float64).clone()
        pose = pose.contiguous()
        n = (params.E + ckpt_every - 1) // ckpt_every if ckpt_every >= 1 else 1  # the library rejects < 1
        ckpt = torch.empty((n, 13), dtype=torch.float64, device=self.device)
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_unrolled_fwd(self._h, ctypes.byref(ct), _ptr(a_t), ctypes.byref(cr), _ptr(a_r), _ptr(mom_t),
                                     _ptr(mom_r), ctypes.byref(pr), int(ckpt_every), _ptr(pose), _ptr(ckpt),
                                     _stream(self.device)))
        return pose, ckpt

    def unrolled_bwd(self, tmpl: Cloud, a_t, ref: Cloud, a_r, mom_t, mom_r, params: Params, ckpt_every: int, ckpt,
                     grad_final):
        """dL/d(initial pose) [13] and dL/d(sigma, eps) [2] from dL/d(final pose)."""
        g0 = torch.empty(13, dtype=torch.float64, device=self.device)
        gse = torch.empty(2, dtype=torch.float64, device=self.device)
        gf = grad_final.to(self.device, torch.float64).contiguous()
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_unrolled_bwd(self._h, ctypes.byref(ct), _ptr(a_t), ctypes.byref(cr), _ptr(a_r), _ptr(mom_t),
                                     _ptr(mom_r), ctypes.byref(pr), int(ckpt_every), _ptr(ckpt.contiguous()),
                                     _ptr(gf), _ptr(g0), _ptr(gse), _stream(self.device)))
        return g0, gse

    def change_detect(self, tmpl: Cloud, a_t, ref: Cloud, a_r, pose, tau: float, sigma: float = 0.0,
                      s_min: float = 0.0):
        """Per template point: flags (uint8; bit 0 nothing within tau, bit 1
        nearest point's shape similarity below s_min), nearest reference
        index (int32) and its float32 squared distance."""
        flags = torch.empty(tmpl.n, dtype=torch.uint8, device=self.device)
        nn = torch.empty(tmpl.n, dtype=torch.int32, device=self.device)
        d2 = torch.empty(tmpl.n, dtype=torch.float32, device=self.device)
        ct, cr = tmpl.c(), ref.c()
        check(lib().sgr_change_detect(self._h, ctypes.byref(ct), _ptr(a_t), ctypes.byref(cr), _ptr(a_r),
                                      _ptr(pose.to(self.device, torch.float64).contiguous()), float(tau), float(sigma),
                                      float(s_min), _ptr(flags), _ptr(nn), _ptr(d2), _stream(self.device)))
        return flags, nn, d2

    def descriptors_radius(self, cloud: Cloud, r2: float, want_count=True):
        """Curvature of the radius neighbourhood (float32 key <= r2) of every
        point, and the member counts."""
        a = torch.empty(cloud.n, dtype=torch.float32, device=self.device)
        cnt = torch.empty(cloud.n, dtype=torch.int32, device=self.device) if want_count else None
        cc = cloud.c()
        check(lib().sgr_descriptors_radius(self._h, ctypes.byref(cc), ctypes.c_float(r2), _ptr(a), _ptr(cnt),
                                           _stream(self.device)))
        return a, cnt

    def register_pyramid(self, tmpl: Cloud, ref: Cloud, params: Params, levels, pose=None, stats=False):
        """register() through the levels of a pyramidal schedule; params.E
        must equal the sum of the levels' iterations."""
        pose = pose_identity(self.device) if pose is None else pose
        st = torch.empty((params.E, 32), dtype=torch.float64, device=self.device) if stats else None
        lv = (_ffi.SgrLevel * len(levels))(*[_ffi.SgrLevel(float(v.radius_scale), float(v.sigma_scale), int(v.iters),
                                                          int(v.k)) for v in levels])
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_register_pyramid(self._h, ctypes.byref(ct), ctypes.byref(cr), ctypes.byref(pr), lv,
                                         len(levels), _ptr(pose), _ptr(st), _stream(self.device)))
        return pose, st

    def descriptors_hn(self, cloud: Cloud, k: int, D: int) -> torch.Tensor:
        """Soft histograms of normals, (n, D) float32."""
        h = torch.empty((cloud.n, D), dtype=torch.float32, device=self.device)
        c = cloud.c()
        check(lib().sgr_descriptors_hn(self._h, ctypes.byref(c), int(k), int(D), _ptr(h), _stream(self.device)))
        return h

    def descriptors_poly(self, cloud: Cloud, k: int) -> torch.Tensor:
        """Local polynomial descriptor (mu1, mu2, residual), (n, 3) float32."""
        out = torch.empty((cloud.n, 3), dtype=torch.float32, device=self.device)
        c = cloud.c()
        check(lib().sgr_descriptors_poly(self._h, ctypes.byref(c), int(k), _ptr(out), _stream(self.device)))
        return out

    def step_vec(self, tmpl: Cloud, a_t, ref: Cloud, a_r, mom_t, mom_r, params: Params, t: int, pose_in,
                 want_wrench=False, want_f=False):
        """step() with vector descriptors a_t (M, D), a_r (N, D)."""
        D = int(a_t.shape[1])
        if a_r.shape[1] != D:
            raise ValueError("descriptor widths differ")
        pout = torch.empty(13, dtype=torch.float64, device=self.device)
        wr = torch.empty(13, dtype=torch.float64, device=self.device) if want_wrench else None
        f = torch.empty((tmpl.n, 3), dtype=torch.float32, device=self.device) if want_f else None
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_step_vec(self._h, ctypes.byref(ct), _ptr(a_t.contiguous()), ctypes.byref(cr),
                                 _ptr(a_r.contiguous()), D, _ptr(mom_t), _ptr(mom_r), ctypes.byref(pr), int(t),
                                 _ptr(pose_in), _ptr(pout), _ptr(wr), _ptr(f), _stream(self.device)))
        return pout, wr, f

    def register_vec(self, tmpl: Cloud, a_t, ref: Cloud, a_r, params: Params, pose=None, stats=False):
        """register() with vector descriptors a_t (M, D), a_r (N, D)."""
        D = int(a_t.shape[1])
        if a_r.shape[1] != D:
            raise ValueError("descriptor widths differ")
        pose = pose_identity(self.device) if pose is None else pose
        st = torch.empty((params.E, 32), dtype=torch.float64, device=self.device) if stats else None
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_register_vec(self._h, ctypes.byref(ct), _ptr(a_t.contiguous()), ctypes.byref(cr),
                                     _ptr(a_r.contiguous()), D, ctypes.byref(pr), _ptr(pose), _ptr(st),
                                     _stream(self.device)))
        return pose, st

    def register_batch(self, tmpls, refs, params: Params, poses=None, want_energy=True, stats=False):
        """B registrations in one batched call; returns (poses [B, 13], energy [B] or None, stats)."""
        B = len(tmpls)
        if len(refs) != B:
            raise ValueError("tmpls and refs differ in length")
        if poses is None:
            poses = pose_identity(self.device).repeat(B, 1).contiguous()
        energy = torch.empty(B, dtype=torch.float64, device=self.device) if want_energy else None
        st = torch.empty((B, params.E, 32), dtype=torch.float64, device=self.device) if stats else None
        ct = (SgrCloud * B)(*[c.c() for c in tmpls])
        cr = (SgrCloud * B)(*[c.c() for c in refs])
        pr = params.c()
        check(lib().sgr_register_batch(self._h, B, ct, cr, ctypes.byref(pr), _ptr(poses), _ptr(energy), _ptr(st),
                                       _stream(self.device)))
        return poses, energy, st

    def multistart(self, tmpl: Cloud, ref: Cloud, params: Params, R0):
        """Multi-start registration; R0 (S, 3, 3) initial rotations about the
        template centroid.  Returns (poses [S, 13], energy [S], best index)."""
        R0 = torch.as_tensor(np.asarray(R0, np.float64)).reshape(-1, 9).to(self.device).contiguous()
        S = int(R0.shape[0])
        poses = torch.empty((S, 13), dtype=torch.float64, device=self.device)
        energy = torch.empty(S, dtype=torch.float64, device=self.device)
        best = torch.empty(1, dtype=torch.int32, device=self.device)
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_multistart(self._h, ctypes.byref(ct), ctypes.byref(cr), ctypes.byref(pr), S, _ptr(R0),
                                   _ptr(poses), _ptr(energy), _ptr(best), _stream(self.device)))
        return poses, energy, int(best.item())

    def residual(self, tmpl: Cloud, ref: Cloud, pose, corr=None) -> torch.Tensor:
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        if corr is not None:
            corr = torch.as_tensor(corr).to(device=self.device, dtype=torch.int32).contiguous()
        ct, cr = tmpl.c(), ref.c()
        check(lib().sgr_residual(self._h, ctypes.byref(ct), ctypes.byref(cr), _ptr(pose), _ptr(corr), _ptr(out),
                                 _stream(self.device)))
        return out


class Plan:
    """A prepared (template, reference) pair (sgr_plan_*): constants and the
    packed reference are built once; force evaluations and steps reuse them.
    Keeps references to every tensor the plan reads."""

    def __init__(self, ctx: Context, tmpl: Cloud, a_t, ref: Cloud, a_r, mom_t, mom_r, params: Params):
        self.ctx = ctx
        self._keep = (tmpl, a_t, ref, a_r, mom_t, mom_r)
        self.M, self.N = tmpl.n, ref.n
        h = ctypes.c_void_p()
        ct, cr, pr = tmpl.c(), ref.c(), params.c()
        check(lib().sgr_plan_create(ctx._h, ctypes.byref(ct), _ptr(a_t), ctypes.byref(cr), _ptr(a_r), _ptr(mom_t),
                                    _ptr(mom_r), ctypes.byref(pr), ctypes.byref(h), _stream(ctx.device)))
        self._h = h

    def force(self, pose, t=0, G=0.0, want_wrench=True, want_f=False):
        dev = self.ctx.device
        wrench = torch.empty(13, dtype=torch.float64, device=dev) if want_wrench else None
        f = torch.empty((self.M, 3), dtype=torch.float32, device=dev) if want_f else None
        check(lib().sgr_plan_force(self._h, int(t), float(G), _ptr(pose), _ptr(wrench), _ptr(f), _stream(dev)))
        return wrench, f

    def step(self, pose_in, t, pose_out=None, want_wrench=False):
        dev = self.ctx.device
        pose_out = torch.empty(13, dtype=torch.float64, device=dev) if pose_out is None else pose_out
        wrench = torch.empty(13, dtype=torch.float64, device=dev) if want_wrench else None
        check(lib().sgr_plan_step(self._h, int(t), _ptr(pose_in), _ptr(pose_out), _ptr(wrench), _stream(dev)))
        return pose_out, wrench

    def close(self):
        if getattr(self, "_h", None):
            lib().sgr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ForceField(torch.autograd.Function):
    """Differentiable shape-weighted force field (forward and adjoint are the
    library's kernels).  apply(ctx, Y, m, sigma, eps, a_t, ref, a_r, mom_r,
    params, G) -> (f [M, 3] float32, wrench [12] float64: F then K).
    Gradients flow to Y (template positions), m (template masses), sigma
    and eps (0-dim float64 tensors); the curvatures are constants."""

    @staticmethod
    def forward(fctx, sctx, Y, m, sigma, eps, a_t, ref, a_r, mom_r, params, G):
        prm = dataclasses.replace(params, sigma=float(sigma), eps=float(eps))
        tm = Cloud(Y.detach(), masses=None if m is None else m.detach(), device=sctx.device)
        f, wrench = sctx.force_fwd(tm, a_t, ref, a_r, mom_r, prm, G)
        fctx.save_for_backward(f)
        fctx.stuff = (sctx, tm, a_t, ref, a_r, mom_r, prm, G, m is not None)
        return f, wrench[:12]

    @staticmethod
    def backward(fctx, grad_f, grad_w):
        (f,) = fctx.saved_tensors
        sctx, tm, a_t, ref, a_r, mom_r, prm, G, has_m = fctx.stuff
        gy, gm, gse = sctx.force_bwd(tm, a_t, ref, a_r, mom_r, prm, G, f, grad_f, grad_w, want_m=has_m,
                                     want_se=True)
        return (None, gy, gm if has_m else None, gse[0], gse[1], None, None, None, None, None, None)


class UnrolledRegistration(torch.autograd.Function):
    """Final pose of params.E registration iterations as a differentiable
    function of the similarity spread sigma, the softening eps and the
    initial pose (forward and reverse passes are the library's kernels; the
    reverse pass recomputes each segment of ckpt_every iterations from the
    pose checkpoints of the forward pass).  apply(sigma, eps, pose0, ctx,
    tmpl, a_t, ref, a_r, mom_t, mom_r, params, ckpt_every) -> pose [13]."""

    @staticmethod
    def forward(fctx, sigma, eps, pose0, sctx, tmpl, a_t, ref, a_r, mom_t, mom_r, params, ckpt_every):
        prm = dataclasses.replace(params, sigma=float(sigma), eps=float(eps))
        pose, ckpt = sctx.unrolled_fwd(tmpl, a_t, ref, a_r, mom_t, mom_r, prm, ckpt_every, pose0.detach())
        fctx.save_for_backward(ckpt)
        fctx.args = (sctx, tmpl, a_t, ref, a_r, mom_t, mom_r, prm, ckpt_every)
        fctx.like = (sigma, eps, pose0)
        return pose

    @staticmethod
    def backward(fctx, grad_pose):
        (ckpt,) = fctx.saved_tensors
        sctx, tmpl, a_t, ref, a_r, mom_t, mom_r, prm, k = fctx.args
        g0, gse = sctx.unrolled_bwd(tmpl, a_t, ref, a_r, mom_t, mom_r, prm, k, ckpt, grad_pose)
        sigma, eps, pose0 = fctx.like
        as_like = lambda g, x: g.to(x.device, x.dtype) if torch.is_tensor(x) else g
        return (as_like(gse[0], sigma), as_like(gse[1], eps), as_like(g0, pose0)) + (None,) * 9
