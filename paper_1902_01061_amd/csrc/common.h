// Shared device helpers for the gfx950 kernels: FP64 3x3 linear algebra
// (one-sided Jacobi SVD), wave/block FP64 reductions, the per-registration
// constant block, and launch helpers.  Host-callable where marked so the
// 3x3 routines can be unit-checked on the CPU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SGR_HD __host__ __device__ inline
#define SGR_HDI __host__ __device__ inline __attribute__((always_inline))

namespace sgr {

// Per-registration constants, computed on the device once per call from the
// clouds, their descriptors and the parameters (kept in device memory so a
// captured graph can replay without host involvement).
struct Derived {
  double xbar[3];    // reference centroid
  double lamX;       // largest eigenvalue of the reference covariance (1/N)
  double L;          // sqrt(lamX): length scale of the distance law
  double ybar0[3];   // centroid of the input template (unweighted)
  double SigY0[6];   // template covariance (1/M): xx yy zz xy xz yz
  double lamY0;      // its largest eigenvalue
  double abar;       // mean reference curvature
  double sigma;      // similarity spread actually used
  double Z;          // sum of reference masses
  double Mtot;       // sum of template masses
  double Mcount;     // number of template points
  double bscale;     // sqrt(log2 e) / sigma: a -> b so that s = exp2(-(b_i - b_j)^2)
  double coefL;      // L^(1 - p)
  double hp;         // (p - 1) / 2
  double eps2;       // eps^2
  double dt2;        // G dt^2 / G
  double G1;
  double E;
  double p;
  double g_mode;
  double expand_ok;  // 1: the expanded similarity exponent 2 b_i b_j - b_j^2 + lw_j, b
                     //    centred at the mean curvature, stays below 64 for every pair
  double lw_max;     // largest log2 weight of the reference (0 if none is positive)
  double bref_lo;    // smallest and largest b of the reference (as rounded to FP32)
  double bref_hi;
  double Vw[9];      // right singular vectors of the last cross-covariance (warm start)
  int32_t cold_svd;  // 1: no warm start of the update's SVD
  int32_t pad2;
  int32_t status;    // 0 ok; bit flags set by the update kernel
  int32_t pad;
  double momentum;   // share of the previous translation carried (eq. 5.5's v^X); 0: v = 0
  double dprev[3];   // the previous iteration's translation (0 at the start)
};

// A pointer read from a table in device memory (a batch's job or
// registration descriptors) is a generic pointer to the compiler: its loads
// become flat loads, which wait on the LDS counter as well as the memory
// counter and are not moved past LDS stores, so loads meant to be in flight
// together are issued one at a time.  gptr(p) rebuilds p from its integer
// value as a global-memory pointer, so that its uses compile to global loads
// and stores.  Only for pointers to device (global) memory.
template <class T>
__device__ inline T* gptr(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

enum : int32_t {
  ST_NONFINITE = 1,   // non-finite wrench or cross-covariance
  ST_SINGULAR = 2,    // cross-covariance of rank < 2
  ST_SCALE = 4,       // pose scale outside [1e-6, 1e6]
  ST_DEGENERATE = 8,  // a cloud with zero variance
};

// Row slot layout of the per-block wrench partials.
constexpr int WR_F = 0;    // 3
constexpr int WR_K = 3;    // 9, row-major K[a][b] = sum_i f_ia (y_i - ybar)_b
constexpr int WR_U = 12;   // 1
constexpr int WR_STRIDE = 16;

// Per-iteration stats row written by the update kernel.
constexpr int ST_G = 0, ST_F = 1, ST_K = 4, ST_U = 13, ST_POSE = 14, ST_C = 27, ST_STATUS = 28;
constexpr int STATS_STRIDE = 32;

// ------------------------------------------------------------- 3x3 FP64
SGR_HD void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// One Jacobi rotation of the column pair (p, q) of a (and of v): makes the
// two columns orthogonal.  The relative non-orthogonality |ga| / sqrt(al be)
// is compared with its thresholds in squares (no square root or division):
// below 1e-17 the pair is left alone, at 1e-15 or above `more` is set (the
// sweeps have not converged).  Every index is a constant at its call sites,
// so the columns stay in registers.
SGR_HDI void jacobi_pair(double (&ap)[3], double (&aq)[3], double (&vp)[3], double (&vq)[3], bool& more) {
  double al = 0, be = 0, ga = 0;
  for (int r = 0; r < 3; ++r) {
    al += ap[r] * ap[r];
    be += aq[r] * aq[r];
    ga += ap[r] * aq[r];
  }
  const double g2 = ga * ga, ab = al * be;
  if (!(g2 > 1e-34 * ab)) return;
  if (g2 >= 1e-30 * ab) more = true;
  // tangent of the rotation angle, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2))
  // with zeta = (be - al) / (2 ga), multiplied through by |2 ga| (one
  // division fewer)
  const double d = be - al, g = 2.0 * ga;
  const double t = (d * g >= 0.0 ? fabs(g) : -fabs(g)) / (fabs(d) + sqrt(d * d + g * g));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = c * t;
  for (int r = 0; r < 3; ++r) {
    const double a0 = ap[r], a1 = aq[r];
    ap[r] = c * a0 - s * a1;
    aq[r] = s * a0 + c * a1;
    const double v0 = vp[r], v1 = vq[r];
    vp[r] = c * v0 - s * v1;
    vq[r] = s * v0 + c * v1;
  }
}

// Swap columns i and j (and their norms) when n[i] < n[j].
SGR_HDI void order_pair(double (&ni)[1], double (&nj)[1], double (&ai)[3], double (&aj)[3], double (&vi)[3],
                        double (&vj)[3]) {
  if (ni[0] < nj[0]) {
    const double t = ni[0];
    ni[0] = nj[0];
    nj[0] = t;
    for (int r = 0; r < 3; ++r) {
      const double x = ai[r];
      ai[r] = aj[r];
      aj[r] = x;
      const double y = vi[r];
      vi[r] = vj[r];
      vj[r] = y;
    }
  }
}

// One-sided (Hestenes) Jacobi SVD of a 3x3 matrix A (row-major):
// A = U diag(sv) V^T with sv sorted descending.  U and V are returned
// column-major in the sense u[k][*] = k-th left singular vector.  A column of
// A that collapses to zero leaves its u[k] undefined (set to 0); callers
// only use the vectors of non-zero singular values.
SGR_HDI void svd3(const double A_in[9], double sv[3], double u[3][3], double v[3][3], const double* V0 = nullptr) {
  double a[3][3];  // a[col][row]
  double vv[3][3]; // vv[col][row]
  // The rotation tests compare products of squared column norms, which
  // under- or overflow for entries far from 1 (below about 1e-77 or above
  // 1e77).  A is therefore scaled by an exact power of two that brings its
  // largest |entry| into [0.5, 1); the singular values are scaled back at
  // the end, and the singular vectors do not change.
  int ex = 0;
  {
    double amax = 0.0;
    for (int e = 0; e < 9; ++e) amax = fmax(amax, fabs(A_in[e]));
    if (amax > 0.0 && amax <= 1.7976931348623157e308) (void)frexp(amax, &ex);
  }
  double As[9];
  for (int e = 0; e < 9; ++e) As[e] = ldexp(A_in[e], -ex);
  // start from V0 (row-major, columns = right singular vectors of a nearby
  // matrix) when given: A V0 is then nearly column-orthogonal and the
  // rotations below converge in one or two sweeps
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) vv[c][r] = V0 ? V0[r * 3 + c] : ((r == c) ? 1.0 : 0.0);
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r)
      a[c][r] = As[r * 3 + 0] * vv[c][0] + As[r * 3 + 1] * vv[c][1] + As[r * 3 + 2] * vv[c][2];
  for (int sweep = 0; sweep < 30; ++sweep) {
    bool more = false;
    // cyclic order (0, 1), (0, 2), (1, 2)
    jacobi_pair(a[0], a[1], vv[0], vv[1], more);
    jacobi_pair(a[0], a[2], vv[0], vv[2], more);
    jacobi_pair(a[1], a[2], vv[1], vv[2], more);
    if (!more) break;
  }
  double n[3][1];
  for (int c = 0; c < 3; ++c) n[c][0] = sqrt(a[c][0] * a[c][0] + a[c][1] * a[c][1] + a[c][2] * a[c][2]);
  // sort descending (3 elements): the columns themselves are exchanged
  order_pair(n[0], n[1], a[0], a[1], vv[0], vv[1]);
  order_pair(n[1], n[2], a[1], a[2], vv[1], vv[2]);
  order_pair(n[0], n[1], a[0], a[1], vv[0], vv[1]);
  for (int k = 0; k < 3; ++k) {
    sv[k] = ldexp(n[k][0], ex);
    const double inv = n[k][0] > 0 ? 1.0 / n[k][0] : 0.0;
    for (int r = 0; r < 3; ++r) {
      u[k][r] = a[k][r] * inv;
      v[k][r] = vv[k][r];
    }
  }
}

// Eigenvalues of a symmetric positive semi-definite 3x3 matrix given as
// (xx, yy, zz, xy, xz, yz): for such matrices the singular values are the
// eigenvalues.  Returns them descending.
SGR_HDI void eig_psd3(const double S6[6], double lam[3]) {
  const double A[9] = {S6[0], S6[3], S6[4], S6[3], S6[1], S6[5], S6[4], S6[5], S6[2]};
  double u[3][3], v[3][3];
  svd3(A, lam, u, v);
}

// Kabsch rotation of eq. (6): with C = U S V^T (paper's hats), R =
// V diag(1, 1, sign det(V U^T)) U^T.  Written through the two leading
// singular pairs: R = v1 u1^T + v2 u2^T + (v1 x v2)(u1 x u2)^T, which is
// the same matrix and needs no sign bookkeeping.  Returns false if C has
// rank < 2 (the rotation is then not determined).
SGR_HDI bool kabsch_rot(const double C[9], double R[9], double* Vwarm = nullptr) {
  double sv[3], u[3][3], v[3][3];
  svd3(C, sv, u, v, Vwarm);
  if (Vwarm) {
    // keep the (sorted) right singular vectors, as a proper rotation, for the next call
    double v3[3];
    cross3(v[0], v[1], v3);
    for (int r = 0; r < 3; ++r) {
      Vwarm[r * 3 + 0] = v[0][r];
      Vwarm[r * 3 + 1] = v[1][r];
      Vwarm[r * 3 + 2] = v3[r];
    }
  }
  if (!(sv[1] > 0.0) || !(sv[1] > sv[0] * 1e-14)) return false;
  double u3[3], v3[3];
  cross3(u[0], u[1], u3);
  cross3(v[0], v[1], v3);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R[r * 3 + c] = v[0][r] * u[0][c] + v[1][r] * u[1][c] + v3[r] * u3[c];
  return true;
}

// ------------------------------------------------------------- reductions
__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ inline float wave_sum_f(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Sum NV doubles over a block of BT threads (BT a multiple of 64) in a fixed
// order; the result is valid in thread 0.  `lds` needs NV * BT/64 doubles.
template <int NV, int BT>
__device__ inline void block_sum(double (&v)[NV], double* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[w * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int ww = 0; ww < BT / 64; ++ww) s += lds[ww * NV + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Smallest and largest value over the threads of a block of BT threads
// (NaN is ignored; every thread receives both).  lds: 2 * BT / 64 doubles of
// scratch, free on entry (a barrier precedes its use).
template <int BT>
__device__ inline void block_range(float& lo, float& hi, double* lds) {
  for (int off = 32; off > 0; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off, 64));
    hi = fmaxf(hi, __shfl_xor(hi, off, 64));
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    lds[2 * w] = (double)lo;
    lds[2 * w + 1] = (double)hi;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < BT / 64; ++k) {
    lo = fminf(lo, (float)lds[2 * k]);
    hi = fmaxf(hi, (float)lds[2 * k + 1]);
  }
}

// Expanded similarity exponent for a block of template points whose b lies
// in [lo, hi] (eq. 3): with d = b - beta,
//   lw_j - (b_i - b_j)^2 = 2 d_i d_j + (lw_j - d_j^2) - d_i^2,
// so a pair costs one FMA and exp2(-d_i^2) is applied in FP64 at the end.
// The unscaled FP32 term exp2(2 d_i d_j + lw_j - d_j^2) must not overflow:
// since every b_j lies in [bref_lo, bref_hi], its exponent is at most
// lw_max + (b_i - beta)^2 - dist(b_i, [bref_lo, bref_hi])^2, which is
// linear or convex in b_i on each side of and inside the range, so its
// largest value over the block is taken at the block's ends or at a range
// end inside the block.  Returns whether that bound is <= 64, and sets beta:
// 0 when fixed (the scalar-load form reads the packed reference directly),
// else the centre of the part of the block inside the reference range, or
// the block end nearest to the range for a block entirely outside it (which
// makes the bound lw_max).  The template order sorted by curvature keeps
// block ranges narrow.
// `extra` bounds any further term of the FP32 exponent (the distance law of
// the r-form, hp log2(q), whose largest value for hp < 0 is hp log2(eps^2)).
__device__ inline bool expanded_centre(float lo, float hi, const Derived& D, bool fixed, float& beta,
                                       double extra = 0.0) {
  beta = 0.f;
  if (!(lo <= hi)) return false;
  const float rlo = (float)D.bref_lo, rhi = (float)D.bref_hi;
  if (!fixed) {
    const float ilo = fmaxf(lo, rlo), ihi = fminf(hi, rhi);
    if (ilo <= ihi)
      beta = 0.5f * ilo + 0.5f * ihi;
    else
      beta = lo > rhi ? lo : hi;
  }
  auto bound = [&](float b) {
    const double d = (double)b - (double)beta;
    const double g = b > rhi ? (double)b - rhi : (b < rlo ? (double)rlo - b : 0.0);
    return d * d - g * g;
  };
  double e = fmax(bound(lo), bound(hi));
  if (rlo > lo && rlo < hi) e = fmax(e, bound(rlo));
  if (rhi > lo && rhi < hi) e = fmax(e, bound(rhi));
  return e + D.lw_max + extra <= 64.0;
}

}  // namespace sgr
