// Shape-weighted all-pairs force (eqs. 3, 5, 10, 11) reduced to the net
// force F and moment matrix K that drive the rigid update.
//
//   f_i = -(G/Z) L^(1-p) g'_i sum_j exp2( hp log2(q_ij) + lw_j - (b_i - b_j)^2 ) r_ij
//   r_ij = y_i - x_j,  q_ij = |r_ij|^2 + eps^2,  hp = (p-1)/2,
//   b = a sqrt(log2 e)/sigma  (so exp2(-(b_i-b_j)^2) is the RBF similarity s_ij),
//   lw_j = log2(w_j) [+ log2(a_j/abar) for g = a a s],  g'_i = 1 [or a_i/abar].
//
// All similarity, mass and distance-law factors of one pair fold into a
// single exponent, so a pair costs 3 sub + 3 fma (q) + 2 fma + one log2 + one
// exp2 + 3 fma (accumulate) on the FP32 VALU for p != 1 (the similarity term
// in the block-centred expanded form below), and no log2 / q for p = 1.  Each lane holds R template points in registers (R
// independent dependency chains hide transcendental latency); the
// reference streams through LDS in tiles of 256 points that every lane reads
// by broadcast.  Per-tile FP32 partial sums (256 terms) are flushed into
// FP64 accumulators, and the per-point forces are reduced to the 13 wrench
// values with FP64 wave shuffles and a fixed-order block sum.  The
// reference is split into chunks across blocks (F and K are linear in the
// per-chunk partial forces), and a second kernel sums the block partials in
// a fixed order, so results are bitwise reproducible.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace sgr {

constexpr int F_BT = 256;  // threads per block
constexpr int F_TJ = 256;  // reference points per LDS tile
constexpr int F_GRAN = 16; // balanced reference chunks are cut at multiples of this

__device__ inline double G_at(const Derived& D, int t) {
  // eq. (12): G(t+1) = 0.1 G1 + 0.9 G1 / (1 + exp(-(t - E/2))); iteration t uses G(t).
  return 0.1 * D.G1 + 0.9 * D.G1 / (1.0 + exp(-(((double)t - 1.0) - 0.5 * D.E)));
}

// Per-registration set-up: statistics of the reference curvatures, masses
// and the constants of the force law.  One block, fixed-order reductions.
__device__ inline void prepare_body(const float* __restrict__ aX, const float* __restrict__ wX, int64_t N,
                                    const float* __restrict__ aY, const float* __restrict__ mY, int64_t M,
                                    const double* __restrict__ mom_t, const double* __restrict__ mom_r,
                                    const PrepParams& P, Derived* __restrict__ out, double* lds, double* red_max,
                                    double* abar_p) {
  double& abar_s = *abar_p;
  // aX == nullptr (and aY == nullptr): no scalar curvature (a caller that
  // weights pairs by other descriptors, or by the masses alone); the
  // curvature statistics are then 0 and sigma comes from the caller.
  double s[3] = {0, 0, 0};
  for (int64_t j = threadIdx.x; j < N; j += 1024) {
    s[0] += aX ? (double)aX[j] : 0.0;
    s[1] += wX ? (double)wX[j] : 1.0;
  }
  for (int64_t i = threadIdx.x; i < M; i += 1024) s[2] += mY ? (double)mY[i] : 1.0;
  block_sum<3, 1024>(s, lds);
  if (threadIdx.x == 0) abar_s = s[0] / (double)N;
  __syncthreads();
  const double abar = abar_s;
  double v[1] = {0};
  for (int64_t j = threadIdx.x; j < N && aX; j += 1024) {
    const double d = (double)aX[j] - abar;
    v[0] += d * d;
  }
  block_sum<1, 1024>(v, lds);
  // largest |a - abar| over both clouds and largest log2 weight: bound of the
  // expanded similarity exponent (checked below once sigma is known)
  // and the range of the reference curvatures
  double mx[4] = {0.0, -INFINITY, -INFINITY, -INFINITY};
  for (int64_t j = threadIdx.x; j < N; j += 1024) {
    const double a = aX ? (double)aX[j] : 0.0;
    mx[0] = fmax(mx[0], fabs(a - abar));
    double l = wX ? log2((double)wX[j]) : 0.0;
    if (P.g_mode == 1) l += log2(a / abar);
    mx[1] = fmax(mx[1], l);
    mx[2] = fmax(mx[2], a);
    mx[3] = fmax(mx[3], -a);
  }
  for (int64_t i = threadIdx.x; i < M && aY; i += 1024) mx[0] = fmax(mx[0], fabs((double)aY[i] - abar));
  for (int c = 0; c < 4; ++c) {
    double m = mx[c];
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red_max[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 16; ++w) m = fmax(m, red_max[w]);
      mx[c] = m;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  Derived D;
  int32_t st = 0;
  for (int c = 0; c < 3; ++c) D.xbar[c] = mom_r[c];
  D.lamX = mom_r[9];
  D.L = sqrt(D.lamX);
  for (int c = 0; c < 3; ++c) D.ybar0[c] = mom_t[c];
  for (int c = 0; c < 6; ++c) D.SigY0[c] = mom_t[3 + c];
  D.lamY0 = mom_t[9];
  D.abar = abar;
  const double sd = sqrt(v[0] / (double)N);
  D.sigma = (P.sigma > 0 ? P.sigma : sd) * P.sigma_scale;
  D.Z = s[1];
  D.Mtot = s[2];
  D.Mcount = (double)M;
  // sqrt(log2 e) / sigma; 0 for g = 1 (no shape term: every b is 0 and s = 1)
  D.bscale = (P.g_mode == 2 || !aX) ? 0.0 : sqrt(1.4426950408889634) / D.sigma;
  D.coefL = exp((1.0 - P.p) * log(D.L));
  D.hp = 0.5 * (P.p - 1.0);
  D.eps2 = P.eps * P.eps;
  D.G1 = P.G1;
  D.E = (double)P.E;
  D.dt2 = P.dt2 > 0 ? P.dt2 : 1.0 / P.G1;
  D.momentum = P.momentum;
  D.dprev[0] = D.dprev[1] = D.dprev[2] = 0.0;
  D.p = P.p;
  D.g_mode = (double)P.g_mode;
  {
    const double bmax = mx[0] * D.bscale;
    D.lw_max = fmax(mx[1], 0.0);
    D.bref_lo = (double)(float)((-mx[3] - abar) * D.bscale);
    D.bref_hi = (double)(float)((mx[2] - abar) * D.bscale);
    D.expand_ok = (bmax * bmax + D.lw_max <= 64.0) ? 1.0 : 0.0;
  }
  for (int e = 0; e < 9; ++e) D.Vw[e] = (e % 4 == 0) ? 1.0 : 0.0;
  D.pad2 = 0;
  D.cold_svd = P.cold_svd;
  if (!(D.lamX > 0) || !(D.lamY0 > 0) || (P.g_mode != 2 && aX && !(D.sigma > 0)) || !(D.Z > 0) || !(D.Mtot > 0) ||
      (P.g_mode == 1 && !(abar > 0)))
    st |= ST_DEGENERATE;
  D.status = st;
  D.pad = 0;
  *out = D;
}

__global__ __launch_bounds__(1024) void prepare_kernel(const float* __restrict__ aX, const float* __restrict__ wX,
                                                       int64_t N, const float* __restrict__ aY,
                                                       const float* __restrict__ mY, int64_t M,
                                                       const double* __restrict__ mom_t, const double* __restrict__ mom_r,
                                                       PrepParams P, Derived* __restrict__ out) {
  __shared__ double lds[16 * 3];
  __shared__ double red_max[16];
  __shared__ double abar_s;
  prepare_body(aX, wX, N, aY, mY, M, mom_t, mom_r, P, out, lds, red_max, &abar_s);
}

// One block per registration of a batch.
__global__ __launch_bounds__(1024) void prepare_batch_kernel(const PrepDesc* __restrict__ d, PrepParams P,
                                                             Derived* __restrict__ outs) {
  __shared__ double lds[16 * 3];
  __shared__ double red_max[16];
  __shared__ double abar_s;
  const PrepDesc g = prep_at(d, blockIdx.x);
  prepare_body(g.aX, g.wX, g.N, g.aY, g.mY, g.M, g.mom_t, g.mom_r, P, outs + blockIdx.x, lds, red_max, &abar_s);
}

// Template in the order the force kernel visits it: position ip holds the
// point perm[ip] as (x0, y0, z0, b) and (a, m), so that the kernel's loads
// are contiguous whatever the order.
__device__ inline void pack_tmpl_body(const float* __restrict__ x, const float* __restrict__ y,
                                      const float* __restrict__ z, const float* __restrict__ aY,
                                      const float* __restrict__ mY, int M, const int* __restrict__ perm,
                                      const Derived& D, float4* __restrict__ tm4, float2* __restrict__ tmx,
                                      int ip) {
  if (ip >= M) return;
  const int i = perm[ip];
  const float a = aY[i];
  tm4[ip] = make_float4(x[i], y[i], z[i], (float)(((double)a - D.abar) * D.bscale));
  tmx[ip] = make_float2(a, mY ? mY[i] : 1.f);
}

__global__ __launch_bounds__(256) void pack_tmpl_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                        const float* __restrict__ z, const float* __restrict__ aY,
                                                        const float* __restrict__ mY, int M,
                                                        const int* __restrict__ perm, const Derived* __restrict__ dv,
                                                        float4* __restrict__ tm4, float2* __restrict__ tmx) {
  pack_tmpl_body(x, y, z, aY, mY, M, perm, *dv, tm4, tmx, blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void pack_tmpl_batch_kernel(const RegDesc* __restrict__ regs,
                                                              const Derived* __restrict__ dvs) {
  const RegDesc g = reg_at(regs, blockIdx.y);
  for (int ip = blockIdx.x * 256 + threadIdx.x; ip < g.M; ip += gridDim.x * 256)
    pack_tmpl_body(g.y0x, g.y0y, g.y0z, g.aY, g.mY, g.M, g.perm, dvs[blockIdx.y], g.tm4, g.tmx, ip);
}

// Reference in the layout the pair loop reads: float4 (x - xbar, b) and
// the log2 weight lw (reference mass and, for g = a a s, a_j / abar).
__device__ inline void pack_ref_body(const float* __restrict__ X, const float* __restrict__ Y,
                                     const float* __restrict__ Zc, const float* __restrict__ aX,
                                     const float* __restrict__ wX, int64_t N, const Derived* __restrict__ dv,
                                     float4* __restrict__ ref4, float* __restrict__ lw, int64_t j) {
  if (j >= N) {
    ref4[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    lw[j] = -INFINITY;
    return;
  }
  const Derived& D = *dv;
  ref4[j] = make_float4((float)((double)X[j] - D.xbar[0]), (float)((double)Y[j] - D.xbar[1]),
                        (float)((double)Zc[j] - D.xbar[2]), (float)(((double)aX[j] - D.abar) * D.bscale));
  double l = wX ? log2((double)wX[j]) : 0.0;
  if (D.g_mode == 1.0) l += log2((double)aX[j] / D.abar);
  lw[j] = (float)l;
}

// The grid covers N rounded up to whole tiles of 256: the tail gets
// zero-weight padding (lw = -inf, so exp2 gives exactly 0).
__global__ __launch_bounds__(256) void pack_ref_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                       const float* __restrict__ Zc, const float* __restrict__ aX,
                                                       const float* __restrict__ wX, int64_t N,
                                                       const Derived* __restrict__ dv, float4* __restrict__ ref4,
                                                       float* __restrict__ lw) {
  pack_ref_body(X, Y, Zc, aX, wX, N, dv, ref4, lw, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void pack_batch_kernel(const PrepDesc* __restrict__ d, const int* __restrict__ blk2reg,
                                                         const Derived* __restrict__ dvs, float4* __restrict__ ref4,
                                                         float* __restrict__ lw) {
  const int r = blk2reg[blockIdx.x];
  const PrepDesc g = prep_at(d, r);
  pack_ref_body(g.xx, g.xy, g.xz, g.aX, g.wX, g.N, dvs + r, ref4 + g.ref_off, lw + g.ref_off,
                (int64_t)(blockIdx.x - g.blk0) * 256 + threadIdx.x);
}

template <int PM>
__device__ inline float pair_coef(float rx, float ry, float rz, float db, float lw, float eps2, float hp, float& q) {
  // exponent of the similarity x weight factor: lw - (b_i - b_j)^2
  const float t = __builtin_fmaf(-db, db, lw);
  q = __builtin_fmaf(rx, rx, __builtin_fmaf(ry, ry, __builtin_fmaf(rz, rz, eps2)));
  if constexpr (PM == 1) {
    return __builtin_amdgcn_exp2f(t);
  } else if constexpr (PM == 3) {
    return __builtin_amdgcn_exp2f(t) * q;
  } else {
    return __builtin_amdgcn_exp2f(__builtin_fmaf(hp, __builtin_amdgcn_logf(q), t));
  }
}

// SM = false: the reference tile is staged in LDS and read by broadcast.
// SM = true: every lane of a wave reads the same reference point, so the
// loads go through the scalar unit into SGPRs (no LDS, no barriers).
// One work item: template points [iblk*256*R, (iblk+1)*256*R) against the
// reference chunk `chunk`; writes its 13 wrench partials to wpart[slot].
// The pose as applied to a template point: y - xbar = sR (y0 - ybar0) + cv.
struct PoseRT {
  double sR[9], cv[3];
};

__device__ inline PoseRT pose_rt(const double* __restrict__ pose, const Derived& D) {
  PoseRT P;
  const double s = pose[0];
#pragma unroll
  for (int e = 0; e < 9; ++e) P.sR[e] = s * pose[1 + e];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    P.cv[r] = P.sR[3 * r] * D.ybar0[0] + P.sR[3 * r + 1] * D.ybar0[1] + P.sR[3 * r + 2] * D.ybar0[2] + pose[10 + r] -
              D.xbar[r];
  return P;
}

// Template point at visiting position ip < M: its index, its similarity
// coordinate b and its posed position relative to xbar (FP64 pose, rounded
// once to FP32).
__device__ inline int tmpl_index(const ForceArgs& A, int ip) { return A.perm ? A.perm[ip] : ip; }

__device__ inline float tmpl_b(const ForceArgs& A, const Derived& D, int ip) {
  if (A.tm4) return A.tm4[ip].w;
  return (float)(((double)A.aY[tmpl_index(A, ip)] - D.abar) * D.bscale);
}

__device__ inline void tmpl_posed(const ForceArgs& A, const Derived& D, const PoseRT& P, int ip, float& px, float& py,
                                  float& pz) {
  float x0, y0, z0;
  if (A.tm4) {
    const float4 T = A.tm4[ip];
    x0 = T.x;
    y0 = T.y;
    z0 = T.z;
  } else {
    const int i = tmpl_index(A, ip);
    x0 = A.y0x[i];
    y0 = A.y0y[i];
    z0 = A.y0z[i];
  }
  const double ex = (double)x0 - D.ybar0[0], ey = (double)y0 - D.ybar0[1], ez = (double)z0 - D.ybar0[2];
  px = (float)(P.sR[0] * ex + P.sR[1] * ey + P.sR[2] * ez + P.cv[0]);
  py = (float)(P.sR[3] * ex + P.sR[4] * ey + P.sR[5] * ez + P.cv[1]);
  pz = (float)(P.sR[6] * ex + P.sR[7] * ey + P.sR[8] * ez + P.cv[2]);
}

// SM = false: the reference tile is staged in LDS and read by broadcast.
// SM = true: every lane of a wave reads the same reference point, so the
// loads go through the scalar unit into SGPRs (no LDS, no barriers).
// One work item: template points at visiting positions [iblk*256*R,
// (iblk+1)*256*R) against reference points [j0, j1); writes its 13 wrench
// partials to wpart[slot] and, with WF, its per-point forces to
// fpart[chunk].
//
// FP64 running sums per point.  r-form: (tx, ty, tz) = sum_j c_ij r_ij (and
// tu = sum_j c_ij q_ij).  Moment form (p = 1): t0 = sum_j c, (tx, ty, tz) =
// sum_j c x_j and tq = sum_j c |x_j|^2, so that sum_j c r = y_i t0 - t and
// sum_j c q = |y_i|^2 t0 - 2 y_i.t + tq + eps^2 t0; the pair loop needs
// neither r_ij nor y_i, and the posed points are formed after it, so that
// nothing but b and the sums occupies registers across the loop.  Its
// exponent is either lw_j - (b_i - b_j)^2 (one sub and one FMA: 6 VALU + 1
// exp2 per pair) or the expanded form below (one FMA: 5 VALU + 1 exp2).
template <int R, int PM, bool WU, bool WF, bool SM>
__device__ inline void force_block(const ForceArgs& A, int iblk, int j0, int j1, int chunk, int slot, float4* s_ref,
                                   float* s_lw, double* s_red, float* s_y) {
  const Derived& D = *A.dv;
  constexpr bool MOM = (PM == 1);
  const int ip0 = iblk * F_BT * R + threadIdx.x;
  const float eps2 = (float)D.eps2;
  const float hp = (float)D.hp;

  // Posed points: in registers for the r-form, whose pair loop reads them;
  // parked in LDS (s_y, [3][R*256]) for the moment form, whose loop does not.
  float bi[R], yx[R], yy[R], yz[R];
  {
    const PoseRT P = pose_rt(A.pose, D);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int ip = ip0 + r * F_BT;
      bi[r] = 0.f;
      yx[r] = yy[r] = yz[r] = 0.f;
      if (ip < A.M) {
        bi[r] = tmpl_b(A, D, ip);
        tmpl_posed(A, D, P, ip, yx[r], yy[r], yz[r]);
      }
      if constexpr (MOM) {
        s_y[r * F_BT + threadIdx.x] = yx[r];
        s_y[(R + r) * F_BT + threadIdx.x] = yy[r];
        s_y[(2 * R + r) * F_BT + threadIdx.x] = yz[r];
      }
    }
  }

  double t0[R], tx[R], ty[R], tz[R], tu[R];
#pragma unroll
  for (int r = 0; r < R; ++r) t0[r] = tx[r] = ty[r] = tz[r] = tu[r] = 0.0;
  // Expanded exponent centred on beta (see expanded_centre): one FMA per
  // pair; the LDS form stages d_j = b_j - beta and lw_j - d_j^2 with the
  // tile, the scalar form keeps beta = 0 and reads the packed reference.
  float beta = 0.f;
  bool expd = false;
  {
    float lo = INFINITY, hi = -INFINITY;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (ip0 + r * F_BT < A.M) {
        lo = fminf(lo, bi[r]);
        hi = fmaxf(hi, bi[r]);
      }
    block_range<F_BT>(lo, hi, s_red);
    // r-form: the distance law adds hp log2(q) to the exponent; for hp < 0 it
    // is largest at q = eps^2 (p < 1 needs eps > 0); p = 3 multiplies by q
    // outside the exponent
    const double extra = (!MOM && PM != 3 && D.hp < 0.0 && D.eps2 > 0.0) ? D.hp * log2(D.eps2) : 0.0;
    expd = expanded_centre(lo, hi, D, SM, beta, extra);
  }
  float al[R];
#pragma unroll
  for (int r = 0; r < R; ++r) al[r] = 2.f * (bi[r] - beta);

  for (int base = j0; base < j1; base += F_TJ) {
    // points of this tile, rounded up to even (the padding has zero weight)
    const int tn = (min(F_TJ, j1 - base) + 1) & ~1;
    // reference point jj of this tile (the packed arrays are padded to whole
    // tiles with zero-weight points, so no bounds test is needed)
    const float4* __restrict__ gref = A.ref4 + base;
    const float* __restrict__ glw = A.reflw + base;
    if constexpr (!SM) {
      __syncthreads();
      {
        const int j = base + threadIdx.x;
        float4 X = make_float4(0.f, 0.f, 0.f, 0.f);  // beyond this range: zero weight
        float l = -INFINITY;                            // (exp2(-inf) = 0), finite coordinates
        if (j < j1) {
          X = gref[threadIdx.x];
          l = glw[threadIdx.x];
        }
        if (expd) {
          // |d_j| is capped at 1e18 so that 2 d_i d_j stays finite; such a
          // term has lw_j - d_j^2 = -1e36 and weight 0 either way (NaN stays NaN)
          float d = X.w - beta;
          if (fabsf(d) > 1e18f) d = copysignf(1e18f, d);
          X.w = d;
          l = __builtin_fmaf(-d, d, l);
        }
        s_ref[threadIdx.x] = X;
        s_lw[threadIdx.x] = l;
      }
      __syncthreads();
    }
    if constexpr (MOM) {
      float a0[R], ax[R], ay[R], az[R], aq[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a0[r] = ax[r] = ay[r] = az[r] = aq[r] = 0.f;
      if (expd && !SM && !WU) {
        // two reference points per step: all 2R exponentials first, then
        // the accumulation, which leaves the exp2 latency off the FMA chains
#pragma unroll 2
        for (int jj = 0; jj < tn; jj += 2) {
          const float4 X0 = s_ref[jj], X1 = s_ref[jj + 1];
          const float c0 = s_lw[jj], c1 = s_lw[jj + 1];
          float w0[R], w1[R];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            w0[r] = __builtin_amdgcn_exp2f(__builtin_fmaf(al[r], X0.w, c0));
            w1[r] = __builtin_amdgcn_exp2f(__builtin_fmaf(al[r], X1.w, c1));
          }
#pragma unroll
          for (int r = 0; r < R; ++r) {
            a0[r] += w0[r] + w1[r];
            ax[r] = __builtin_fmaf(w0[r], X0.x, __builtin_fmaf(w1[r], X1.x, ax[r]));
            ay[r] = __builtin_fmaf(w0[r], X0.y, __builtin_fmaf(w1[r], X1.y, ay[r]));
            az[r] = __builtin_fmaf(w0[r], X0.z, __builtin_fmaf(w1[r], X1.z, az[r]));
          }
        }
      } else if (expd) {
#pragma unroll 2
        for (int jj = 0; jj < tn; ++jj) {
          const float4 X = SM ? gref[jj] : s_ref[jj];
          const float cj = SM ? __builtin_fmaf(-X.w, X.w, glw[jj]) : s_lw[jj];
          float x2 = 0.f;
          if constexpr (WU) x2 = __builtin_fmaf(X.x, X.x, __builtin_fmaf(X.y, X.y, X.z * X.z));
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const float c = __builtin_amdgcn_exp2f(__builtin_fmaf(al[r], X.w, cj));
            a0[r] += c;
            ax[r] = __builtin_fmaf(c, X.x, ax[r]);
            ay[r] = __builtin_fmaf(c, X.y, ay[r]);
            az[r] = __builtin_fmaf(c, X.z, az[r]);
            if constexpr (WU) aq[r] = __builtin_fmaf(c, x2, aq[r]);
          }
        }
      } else {
#pragma unroll 2
        for (int jj = 0; jj < tn; ++jj) {
          const float4 X = SM ? gref[jj] : s_ref[jj];
          const float lw = SM ? glw[jj] : s_lw[jj];
          float x2 = 0.f;
          if constexpr (WU) x2 = __builtin_fmaf(X.x, X.x, __builtin_fmaf(X.y, X.y, X.z * X.z));
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const float db = bi[r] - X.w;
            const float c = __builtin_amdgcn_exp2f(__builtin_fmaf(-db, db, lw));
            a0[r] += c;
            ax[r] = __builtin_fmaf(c, X.x, ax[r]);
            ay[r] = __builtin_fmaf(c, X.y, ay[r]);
            az[r] = __builtin_fmaf(c, X.z, az[r]);
            if constexpr (WU) aq[r] = __builtin_fmaf(c, x2, aq[r]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        t0[r] += (double)a0[r];
        tx[r] += (double)ax[r];
        ty[r] += (double)ay[r];
        tz[r] += (double)az[r];
        if constexpr (WU) tu[r] += (double)aq[r];
      }
    } else {
      float ax[R], ay[R], az[R], au[R];
#pragma unroll
      for (int r = 0; r < R; ++r) ax[r] = ay[r] = az[r] = au[r] = 0.f;
      if (expd) {
        // block-centred expanded similarity exponent: one FMA, the factor
        // exp2(-d_i^2) is applied in FP64 after the loop
#pragma unroll 2
        for (int jj = 0; jj < tn; ++jj) {
          const float4 X = SM ? gref[jj] : s_ref[jj];
          const float cj = SM ? __builtin_fmaf(-X.w, X.w, glw[jj]) : s_lw[jj];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const float rx = yx[r] - X.x, ry = yy[r] - X.y, rz = yz[r] - X.z;
            const float q = __builtin_fmaf(rx, rx, __builtin_fmaf(ry, ry, __builtin_fmaf(rz, rz, eps2)));
            const float e = __builtin_fmaf(al[r], X.w, cj);
            float c;
            if constexpr (PM == 3)
              c = __builtin_amdgcn_exp2f(e) * q;
            else
              c = __builtin_amdgcn_exp2f(__builtin_fmaf(hp, __builtin_amdgcn_logf(q), e));
            ax[r] = __builtin_fmaf(c, rx, ax[r]);
            ay[r] = __builtin_fmaf(c, ry, ay[r]);
            az[r] = __builtin_fmaf(c, rz, az[r]);
            if constexpr (WU) au[r] = __builtin_fmaf(c, q, au[r]);
          }
        }
      } else {
#pragma unroll 2
        for (int jj = 0; jj < tn; ++jj) {
          const float4 X = SM ? gref[jj] : s_ref[jj];
          const float lw = SM ? glw[jj] : s_lw[jj];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const float rx = yx[r] - X.x, ry = yy[r] - X.y, rz = yz[r] - X.z;
            float q;
            const float c = pair_coef<PM>(rx, ry, rz, bi[r] - X.w, lw, eps2, hp, q);
            ax[r] = __builtin_fmaf(c, rx, ax[r]);
            ay[r] = __builtin_fmaf(c, ry, ay[r]);
            az[r] = __builtin_fmaf(c, rz, az[r]);
            if constexpr (WU) au[r] = __builtin_fmaf(c, q, au[r]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        tx[r] += (double)ax[r];
        ty[r] += (double)ay[r];
        tz[r] += (double)az[r];
        if constexpr (WU) tu[r] += (double)au[r];
      }
    }
  }

  // Per-point force and its contributions to F, K, U.
  double cv[3];
  {
    const PoseRT P = pose_rt(A.pose, D);
#pragma unroll
    for (int c = 0; c < 3; ++c) cv[c] = P.cv[c];
  }
  const double G = A.G > 0 ? A.G : G_at(D, A.t);
  const double coef = -(G / D.Z) * D.coefL;
  const double ucoef = (G / D.Z) * D.coefL / (D.p + 1.0);
  double w[13];
#pragma unroll
  for (int e = 0; e < 13; ++e) w[e] = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int ip = ip0 + r * F_BT;
    if (ip >= A.M) continue;
    if constexpr (!MOM) {
      if (expd) {
        const double dl = (double)(bi[r] - beta);
        const double sc = exp2(-dl * dl);
        tx[r] *= sc;
        ty[r] *= sc;
        tz[r] *= sc;
        if constexpr (WU) tu[r] *= sc;
      }
    }
    if constexpr (MOM) {
      yx[r] = s_y[r * F_BT + threadIdx.x];
      yy[r] = s_y[(R + r) * F_BT + threadIdx.x];
      yz[r] = s_y[(2 * R + r) * F_BT + threadIdx.x];
      const double dl = (double)(bi[r] - beta);
      const double sc = expd ? exp2(-dl * dl) : 1.0;
      const double py = yx[r], pyy = yy[r], pz = yz[r];
      if constexpr (WU)
        tu[r] = sc * ((py * py + pyy * pyy + pz * pz + D.eps2) * t0[r] - 2.0 * (py * tx[r] + pyy * ty[r] + pz * tz[r]) +
                      tu[r]);
      tx[r] = sc * (py * t0[r] - tx[r]);
      ty[r] = sc * (pyy * t0[r] - ty[r]);
      tz[r] = sc * (pz * t0[r] - tz[r]);
    }
    double ai, mi;
    if (A.tmx) {
      const float2 T = A.tmx[ip];
      ai = (double)T.x;
      mi = (double)T.y;
    } else {
      const int i = tmpl_index(A, ip);
      ai = (double)A.aY[i];
      mi = A.mY ? (double)A.mY[i] : 1.0;
    }
    const double gi = D.g_mode == 1.0 ? ai / D.abar : 1.0;
    const double fx = coef * gi * tx[r], fy = coef * gi * ty[r], fz = coef * gi * tz[r];
    // lever arm y_i - ybar = sR (y0_i - ybar0), from the posed FP32 point
    // (relative rounding 2^-24)
    const double cx = (double)yx[r] - cv[0], cy = (double)yy[r] - cv[1], cz = (double)yz[r] - cv[2];
    w[WR_F + 0] += mi * fx;
    w[WR_F + 1] += mi * fy;
    w[WR_F + 2] += mi * fz;
    w[WR_K + 0] += fx * cx;
    w[WR_K + 1] += fx * cy;
    w[WR_K + 2] += fx * cz;
    w[WR_K + 3] += fy * cx;
    w[WR_K + 4] += fy * cy;
    w[WR_K + 5] += fy * cz;
    w[WR_K + 6] += fz * cx;
    w[WR_K + 7] += fz * cy;
    w[WR_K + 8] += fz * cz;
    if constexpr (WU) w[WR_U] += ucoef * gi * tu[r];
    if constexpr (WF) {
      double* fp = A.fpart + ((int64_t)chunk * A.M + ip) * 3;  // visiting order
      fp[0] = fx;
      fp[1] = fy;
      fp[2] = fz;
    }
  }
  block_sum<13, F_BT>(w, s_red);
  if (threadIdx.x == 0) {
    double* o = A.wpart + (int64_t)slot * WR_STRIDE;
#pragma unroll
    for (int e = 0; e < 13; ++e) o[e] = w[e];
  }
}

template <int R, int PM, bool WU, bool WF, bool SM>
__global__ __launch_bounds__(F_BT) void force_kernel(ForceArgs A) {
  __shared__ float4 s_ref[SM ? 1 : F_TJ];
  __shared__ float s_lw[SM ? 1 : F_TJ];
  __shared__ double s_red[(F_BT / 64) * 13];
  __shared__ float s_y[PM == 1 ? 3 * R * F_BT : 1];
  const int n_iblk = (A.M + F_BT * R - 1) / (F_BT * R);
  const int chunk = blockIdx.x / n_iblk;
  int j0, j1;
  if (A.chunk_len > 0) {
    j0 = chunk * A.chunk_len;
    j1 = min(A.N, j0 + A.chunk_len);
  } else {
    // balanced chunks: chunk c covers the F_GRAN-point groups [c n / C, (c + 1) n / C)
    const int64_t n_sub = (A.N + F_GRAN - 1) / F_GRAN;
    j0 = (int)(chunk * n_sub / A.n_chunks) * F_GRAN;
    j1 = min(A.N, (int)((chunk + 1) * n_sub / A.n_chunks) * F_GRAN);
  }
  force_block<R, PM, WU, WF, SM>(A, blockIdx.x % n_iblk, j0, j1, chunk, blockIdx.x, s_ref, s_lw, s_red, s_y);
}

// Persistent form over a batch of registrations: the grid strides over a
// work list of (registration, template block, reference chunk) items, sorted
// by decreasing cost; each item writes the partial wrench to its own slot,
// so the per-registration sums do not depend on the execution order.
template <int R, int PM, bool WU>
__global__ __launch_bounds__(F_BT) void force_batch_kernel(BatchArgs B) {
  __shared__ float4 s_ref[F_TJ];
  __shared__ float s_lw[F_TJ];
  __shared__ double s_red[(F_BT / 64) * 13];
  __shared__ float s_y[PM == 1 ? 3 * R * F_BT : 1];
  for (int it = blockIdx.x; it < B.n_items; it += gridDim.x) {
    const int4 item = B.items[it];  // (registration, template block, chunk, output slot)
    const RegDesc g = reg_at(B.regs, item.x);
    ForceArgs A{g.y0x, g.y0y, g.y0z, g.aY, g.mY, B.ref4 + g.ref_off, B.reflw + g.ref_off,
                B.poses + (int64_t)13 * item.x, B.dvs + item.x, g.M, g.N, B.chunk_len, 0, B.t, 0.0, B.wpart, nullptr,
                g.perm, g.tm4, g.tmx};
    const int j0 = item.z * B.chunk_len;
    force_block<R, PM, WU, false, false>(A, item.y, j0, min(g.N, j0 + B.chunk_len), item.z, item.w, s_ref, s_lw,
                                         s_red, s_y);
  }
}

// f_out[perm[ip]] = sum over chunks of the per-chunk forces of visiting
// position ip (fixed order); perm may be null (identity).
__global__ __launch_bounds__(256) void reduce_f_kernel(const double* __restrict__ fpart, int n_chunks, int M,
                                                       const int* __restrict__ perm, float* __restrict__ f_out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * 3) return;
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += fpart[(int64_t)c * M * 3 + e];
  const int64_t ip = e / 3;
  f_out[(perm ? (int64_t)perm[ip] : ip) * 3 + (e - ip * 3)] = (float)s;
}

hipError_t launch_prepare(const float* aX, const float* wX, int64_t N, const float* aY, const float* mY, int64_t M,
                          const double* mom_t, const double* mom_r, const PrepParams& P, Derived* out, hipStream_t st) {
  hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(1024), 0, st, aX, wX, N, aY, mY, M, mom_t, mom_r, P, out);
  return hipGetLastError();
}

hipError_t launch_pack_tmpl(const float* x, const float* y, const float* z, const float* aY, const float* mY, int M,
                            const int* perm, const Derived* dv, float4* tm4, float2* tmx, hipStream_t st) {
  hipLaunchKernelGGL(pack_tmpl_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, x, y, z, aY, mY, M, perm,
                     dv, tm4, tmx);
  return hipGetLastError();
}

hipError_t launch_pack_tmpl_batch(const RegDesc* regs, int B, int max_M, const Derived* dvs, hipStream_t st) {
  const unsigned gx = (unsigned)std::min(64, (max_M + 255) / 256);
  hipLaunchKernelGGL(pack_tmpl_batch_kernel, dim3(gx, (unsigned)B), dim3(256), 0, st, regs, dvs);
  return hipGetLastError();
}

hipError_t launch_prepare_batch(const PrepDesc* d, int B, const PrepParams& P, Derived* outs, hipStream_t st) {
  hipLaunchKernelGGL(prepare_batch_kernel, dim3(B), dim3(1024), 0, st, d, P, outs);
  return hipGetLastError();
}

hipError_t launch_pack_batch(const PrepDesc* d, const int* blk2reg, int n_blocks, const Derived* dvs, float4* ref4,
                             float* lw, hipStream_t st) {
  hipLaunchKernelGGL(pack_batch_kernel, dim3(n_blocks), dim3(256), 0, st, d, blk2reg, dvs, ref4, lw);
  return hipGetLastError();
}

hipError_t launch_pack_ref(const float* x, const float* y, const float* z, const float* aX, const float* wX, int64_t N,
                           const Derived* dv, float4* ref4, float* lw, hipStream_t st) {
  hipLaunchKernelGGL(pack_ref_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, x, y, z, aX, wX, N, dv, ref4,
                     lw);
  return hipGetLastError();
}

template <int R, int PM, bool SM>
static void launch_force_rps(const ForceArgs& A, int nblk, bool wu, bool wf, hipStream_t st) {
  if (wu && wf)
    hipLaunchKernelGGL((force_kernel<R, PM, true, true, SM>), dim3(nblk), dim3(F_BT), 0, st, A);
  else if (wu)
    hipLaunchKernelGGL((force_kernel<R, PM, true, false, SM>), dim3(nblk), dim3(F_BT), 0, st, A);
  else if (wf)
    hipLaunchKernelGGL((force_kernel<R, PM, false, true, SM>), dim3(nblk), dim3(F_BT), 0, st, A);
  else
    hipLaunchKernelGGL((force_kernel<R, PM, false, false, SM>), dim3(nblk), dim3(F_BT), 0, st, A);
}

template <int R>
static void launch_force_r(const ForceArgs& A, int pm, bool sm, int nblk, bool wu, bool wf, hipStream_t st) {
  if (sm) {
    if (pm == 1)
      launch_force_rps<R, 1, true>(A, nblk, wu, wf, st);
    else if (pm == 3)
      launch_force_rps<R, 3, true>(A, nblk, wu, wf, st);
    else
      launch_force_rps<R, 0, true>(A, nblk, wu, wf, st);
  } else {
    if (pm == 1)
      launch_force_rps<R, 1, false>(A, nblk, wu, wf, st);
    else if (pm == 3)
      launch_force_rps<R, 3, false>(A, nblk, wu, wf, st);
    else
      launch_force_rps<R, 0, false>(A, nblk, wu, wf, st);
  }
}

// Resident blocks per CU of the force kernel (cached per instantiation).
template <int R, int PM, bool SM>
static int force_occ() {
  static int occ = 0;
  if (occ == 0) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, force_kernel<R, PM, false, false, SM>, F_BT, 0) !=
            hipSuccess ||
        n < 1)
      n = 1;
    occ = n;
  }
  return occ;
}

template <int R>
static int force_occ_r(int pm, bool sm) {
  if (pm == 1) return sm ? force_occ<R, 1, true>() : force_occ<R, 1, false>();
  if (pm == 3) return sm ? force_occ<R, 3, true>() : force_occ<R, 3, false>();
  return sm ? force_occ<R, 0, true>() : force_occ<R, 0, false>();
}

int force_blocks_per_cu(int R, int pm, bool sm) {
  switch (R) {
    case 1: return force_occ_r<1>(pm, sm);
    case 2: return force_occ_r<2>(pm, sm);
    case 4: return force_occ_r<4>(pm, sm);
    case 8: return force_occ_r<8>(pm, sm);
    default: return 1;
  }
}

int force_points_per_block(int R) { return F_BT * R; }
int force_chunk_gran() { return F_GRAN; }
int force_tile_j() { return F_TJ; }

hipError_t launch_force(const ForceArgs& A, int R, int pm, bool want_u, bool want_f, hipStream_t st, bool sm) {
  const int n_iblk = (A.M + F_BT * R - 1) / (F_BT * R);
  const int nblk = n_iblk * A.n_chunks;
  switch (R) {
    case 1: launch_force_r<1>(A, pm, sm, nblk, want_u, want_f, st); break;
    case 2: launch_force_r<2>(A, pm, sm, nblk, want_u, want_f, st); break;
    case 4: launch_force_r<4>(A, pm, sm, nblk, want_u, want_f, st); break;
    case 8: launch_force_r<8>(A, pm, sm, nblk, want_u, want_f, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_force_batch(const BatchArgs& B, int R, int pm, bool want_u, int grid, hipStream_t st) {
#define SGR_FB(RR, PP, UU) hipLaunchKernelGGL((force_batch_kernel<RR, PP, UU>), dim3(grid), dim3(F_BT), 0, st, B)
#define SGR_FB_R(RR)                      \
  do {                                     \
    if (pm == 1) {                         \
      if (want_u) SGR_FB(RR, 1, true);     \
      else SGR_FB(RR, 1, false);           \
    } else if (pm == 3) {                  \
      if (want_u) SGR_FB(RR, 3, true);     \
      else SGR_FB(RR, 3, false);           \
    } else {                               \
      if (want_u) SGR_FB(RR, 0, true);     \
      else SGR_FB(RR, 0, false);           \
    }                                      \
  } while (0)
  switch (R) {
    case 1: SGR_FB_R(1); break;
    case 2: SGR_FB_R(2); break;
    case 4: SGR_FB_R(4); break;
    default: return hipErrorInvalidValue;
  }
#undef SGR_FB_R
#undef SGR_FB
  return hipGetLastError();
}

hipError_t launch_reduce_f(const double* fpart, int n_chunks, int M, const int* perm, float* f_out, hipStream_t st) {
  const int64_t n = (int64_t)M * 3;
  hipLaunchKernelGGL(reduce_f_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, fpart, n_chunks, M, perm,
                     f_out);
  return hipGetLastError();
}

}  // namespace sgr
