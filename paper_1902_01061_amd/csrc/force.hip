// Shape-weighted all-pairs force (eqs. 3, 5, 10, 11) reduced to the net
// force F and moment matrix K that drive the rigid update.
//
//   f_i = -(G/Z) L^(1-p) g'_i sum_j exp2( hp log2(q_ij) + lw_j - (b_i - b_j)^2 ) r_ij
//   r_ij = y_i - x_j,  q_ij = |r_ij|^2 + eps^2,  hp = (p-1)/2,
//   b = a sqrt(log2 e)/sigma  (so exp2(-(b_i-b_j)^2) is the RBF similarity s_ij),
//   lw_j = log2(w_j) [+ log2(a_j/abar) for g = a a s],  g'_i = 1 [or a_i/abar].
//
// All similarity, mass and distance-law factors of one pair fold into a
// single exponent, so a pair costs 3 sub + 3 fma (q) + 1 sub + 2 fma + one
// log2 + one exp2 + 3 fma (accumulate) on the FP32 VALU for p != 1, and no
// log2 / q for p = 1.  Each lane holds R template points in registers (R
// independent dependency chains hide transcendental latency); the
// reference streams through LDS in tiles of 256 points that every lane reads
// by broadcast.  Per-tile FP32 partial sums (256 terms) are flushed into
// FP64 accumulators, and the per-point forces are reduced to the 13 wrench
// values with FP64 wave shuffles and a fixed-order block sum.  The
// reference is split into chunks across blocks (F and K are linear in the
// per-chunk partial forces), and a second kernel sums the block partials in
// a fixed order, so results are bitwise reproducible.
#include "common.h"
#include "launch.h"

namespace sgr {

constexpr int F_BT = 256;  // threads per block
constexpr int F_TJ = 256;  // reference points per LDS tile

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
  double s[3] = {0, 0, 0};
  for (int64_t j = threadIdx.x; j < N; j += 1024) {
    s[0] += (double)aX[j];
    s[1] += wX ? (double)wX[j] : 1.0;
  }
  for (int64_t i = threadIdx.x; i < M; i += 1024) s[2] += mY ? (double)mY[i] : 1.0;
  block_sum<3, 1024>(s, lds);
  if (threadIdx.x == 0) abar_s = s[0] / (double)N;
  __syncthreads();
  const double abar = abar_s;
  double v[1] = {0};
  for (int64_t j = threadIdx.x; j < N; j += 1024) {
    const double d = (double)aX[j] - abar;
    v[0] += d * d;
  }
  block_sum<1, 1024>(v, lds);
  // largest |a - abar| over both clouds and largest log2 weight: bound of the
  // expanded similarity exponent (checked below once sigma is known)
  double mx[2] = {0.0, -INFINITY};
  for (int64_t j = threadIdx.x; j < N; j += 1024) {
    mx[0] = fmax(mx[0], fabs((double)aX[j] - abar));
    double l = wX ? log2((double)wX[j]) : 0.0;
    if (P.g_mode == 1) l += log2((double)aX[j] / abar);
    mx[1] = fmax(mx[1], l);
  }
  for (int64_t i = threadIdx.x; i < M; i += 1024) mx[0] = fmax(mx[0], fabs((double)aY[i] - abar));
  for (int c = 0; c < 2; ++c) {
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
  D.sigma = P.sigma > 0 ? P.sigma : sd;
  D.Z = s[1];
  D.Mtot = s[2];
  D.Mcount = (double)M;
  D.bscale = sqrt(1.4426950408889634) / D.sigma;  // sqrt(log2 e) / sigma
  D.coefL = exp((1.0 - P.p) * log(D.L));
  D.hp = 0.5 * (P.p - 1.0);
  D.eps2 = P.eps * P.eps;
  D.G1 = P.G1;
  D.E = (double)P.E;
  D.dt2 = P.dt2 > 0 ? P.dt2 : 1.0 / P.G1;
  D.p = P.p;
  D.g_mode = (double)P.g_mode;
  {
    const double bmax = mx[0] * D.bscale;
    D.lw_max = fmax(mx[1], 0.0);
    D.expand_ok = (bmax * bmax + D.lw_max <= 64.0) ? 1.0 : 0.0;
  }
  for (int e = 0; e < 9; ++e) D.Vw[e] = (e % 4 == 0) ? 1.0 : 0.0;
  D.n_safe = 0;
  D.pad2 = 0;
  if (!(D.lamX > 0) || !(D.lamY0 > 0) || !(D.sigma > 0) || !(D.Z > 0) || !(D.Mtot > 0) ||
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
  const PrepDesc& g = d[blockIdx.x];
  prepare_body(g.aX, g.wX, g.N, g.aY, g.mY, g.M, g.mom_t, g.mom_r, P, outs + blockIdx.x, lds, red_max, &abar_s);
}

// Stable partition of the template points: those whose expanded similarity
// exponent stays below 64 for every reference point (b_i^2 + lw_max <= 64)
// first, the rest after; n_safe counts the first group.  A block of the
// force kernel whose points all lie in the first group can use the
// one-FMA exponent.  One block, deterministic.
__device__ inline void partition_body(const float* __restrict__ aY, int M, Derived* __restrict__ dv,
                                      int* __restrict__ perm, int* s_cnt) {
  const Derived& D = *dv;
  const int C = (M + 1023) / 1024;
  const int lo = min(M, (int)threadIdx.x * C), hi = min(M, lo + C);
  auto safe = [&](int i) {
    const double b = (double)(float)(((double)aY[i] - D.abar) * D.bscale);
    return b * b + D.lw_max <= 64.0;
  };
  int cnt = 0;
  for (int i = lo; i < hi; ++i) cnt += safe(i) ? 1 : 0;
  s_cnt[threadIdx.x] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int t = 0; t < 1024; ++t) {
      const int v = s_cnt[t];
      s_cnt[t] = acc;
      acc += v;
    }
    s_cnt[1024] = acc;
  }
  __syncthreads();
  const int total = s_cnt[1024];
  int ps = s_cnt[threadIdx.x];
  int pu = total + (lo - s_cnt[threadIdx.x]);
  for (int i = lo; i < hi; ++i) {
    if (safe(i))
      perm[ps++] = i;
    else
      perm[pu++] = i;
  }
  if (threadIdx.x == 0) dv->n_safe = total;
}

__global__ __launch_bounds__(1024) void partition_kernel(const float* __restrict__ aY, int M, Derived* __restrict__ dv,
                                                         int* __restrict__ perm) {
  __shared__ int s_cnt[1025];
  partition_body(aY, M, dv, perm, s_cnt);
}

__global__ __launch_bounds__(1024) void partition_batch_kernel(const RegDesc* __restrict__ regs,
                                                               Derived* __restrict__ dvs) {
  __shared__ int s_cnt[1025];
  const RegDesc& g = regs[blockIdx.x];
  partition_body(g.aY, g.M, dvs + blockIdx.x, g.perm, s_cnt);
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
  const PrepDesc& g = d[r];
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
template <int R, int PM, bool WU, bool WF, bool SM>
__device__ inline void force_block(const ForceArgs& A, int iblk, int chunk, int slot, float4* s_ref, float* s_lw,
                                   double* s_red) {
  const Derived& D = *A.dv;

  // pose: y - xbar = sR (y0 - ybar0) + (sR ybar0 + t - xbar)
  double sR[9], cv[3];
  {
    const double s = A.pose[0];
#pragma unroll
    for (int e = 0; e < 9; ++e) sR[e] = s * A.pose[1 + e];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      cv[r] = sR[3 * r] * D.ybar0[0] + sR[3 * r + 1] * D.ybar0[1] + sR[3 * r + 2] * D.ybar0[2] + A.pose[10 + r] -
              D.xbar[r];
  }
  const float eps2 = (float)D.eps2;
  const float hp = (float)D.hp;

  float yx[R], yy[R], yz[R], bi[R];
  int ii[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int ip = iblk * F_BT * R + r * F_BT + threadIdx.x;
    const int i = ip < A.M ? (A.perm ? A.perm[ip] : ip) : A.M;
    ii[r] = i;
    if (i < A.M) {
      const double ex = (double)A.y0x[i] - D.ybar0[0], ey = (double)A.y0y[i] - D.ybar0[1],
                   ez = (double)A.y0z[i] - D.ybar0[2];
      yx[r] = (float)(sR[0] * ex + sR[1] * ey + sR[2] * ez + cv[0]);
      yy[r] = (float)(sR[3] * ex + sR[4] * ey + sR[5] * ez + cv[1]);
      yz[r] = (float)(sR[6] * ex + sR[7] * ey + sR[8] * ez + cv[2]);
      bi[r] = (float)(((double)A.aY[i] - D.abar) * D.bscale);
    } else {
      yx[r] = yy[r] = yz[r] = 0.f;
      bi[r] = 0.f;
    }
  }

  // FP64 running sums per point.  r-form: (tx, ty, tz) = sum_j c_ij r_ij
  // (and tu = sum_j c_ij q_ij).  Moment form (p = 1): t0 = sum_j c, (tx, ty,
  // tz) = sum_j c x_j and tq = sum_j c |x_j|^2, so that sum_j c r =
  // y_i t0 - t and sum_j c q = |y_i|^2 t0 - 2 y_i.t + tq + eps^2 t0; it needs
  // no r_ij.  Its exponent is either lw_j - (b_i - b_j)^2 (one sub and one
  // FMA: 6 VALU + 1 exp2 per pair) or, when the prepare kernel has shown it
  // cannot overflow (expand_ok), the expanded 2 b_i b_j + (lw_j - b_j^2)
  // (one FMA: 5 VALU + 1 exp2), whose extra factor exp2(b_i^2) is divided
  // out in FP64 at the end.
  double t0[R], tx[R], ty[R], tz[R], tu[R];
#pragma unroll
  for (int r = 0; r < R; ++r) t0[r] = tx[r] = ty[r] = tz[r] = tu[r] = 0.0;
  constexpr bool MOM = (PM == 1);
  // expanded exponent: every point of this block must admit it
  const bool expd = MOM && (D.expand_ok != 0.0 || (A.perm && min(A.M, (iblk + 1) * F_BT * R) <= D.n_safe));
  float al[R];
#pragma unroll
  for (int r = 0; r < R; ++r) al[r] = 2.f * bi[r];

  const int j0 = chunk * A.chunk_len;
  const int j1 = min(A.N, j0 + A.chunk_len);
  for (int base = j0; base < j1; base += F_TJ) {
    // reference point jj of this tile (the packed arrays are padded to whole
    // tiles with zero-weight points, so no bounds test is needed)
    const float4* __restrict__ gref = A.ref4 + base;
    const float* __restrict__ glw = A.reflw + base;
    if constexpr (!SM) {
      __syncthreads();
      {
        const int j = base + threadIdx.x;
        if (j < j1) {
          s_ref[threadIdx.x] = gref[threadIdx.x];
          s_lw[threadIdx.x] = glw[threadIdx.x];
        } else {  // beyond this chunk: zero weight (exp2(-inf) = 0), finite coordinates
          s_ref[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
          s_lw[threadIdx.x] = -INFINITY;
        }
      }
      __syncthreads();
    }
    if constexpr (MOM) {
      float a0[R], ax[R], ay[R], az[R], aq[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a0[r] = ax[r] = ay[r] = az[r] = aq[r] = 0.f;
      if (expd) {
#pragma unroll 2
        for (int jj = 0; jj < F_TJ; ++jj) {
          const float4 X = SM ? gref[jj] : s_ref[jj];
          const float beta = __builtin_fmaf(-X.w, X.w, SM ? glw[jj] : s_lw[jj]);
          float x2 = 0.f;
          if constexpr (WU) x2 = __builtin_fmaf(X.x, X.x, __builtin_fmaf(X.y, X.y, X.z * X.z));
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const float c = __builtin_amdgcn_exp2f(__builtin_fmaf(al[r], X.w, beta));
            a0[r] += c;
            ax[r] = __builtin_fmaf(c, X.x, ax[r]);
            ay[r] = __builtin_fmaf(c, X.y, ay[r]);
            az[r] = __builtin_fmaf(c, X.z, az[r]);
            if constexpr (WU) aq[r] = __builtin_fmaf(c, x2, aq[r]);
          }
        }
      } else {
#pragma unroll 2
        for (int jj = 0; jj < F_TJ; ++jj) {
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
#pragma unroll 2
      for (int jj = 0; jj < F_TJ; ++jj) {
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
#pragma unroll
      for (int r = 0; r < R; ++r) {
        tx[r] += (double)ax[r];
        ty[r] += (double)ay[r];
        tz[r] += (double)az[r];
        if constexpr (WU) tu[r] += (double)au[r];
      }
    }
  }
  if constexpr (MOM) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double sc = expd ? exp2(-(double)bi[r] * (double)bi[r]) : 1.0;
      const double py = yx[r], pyy = yy[r], pz = yz[r];
      if constexpr (WU)
        tu[r] = sc * ((py * py + pyy * pyy + pz * pz + D.eps2) * t0[r] - 2.0 * (py * tx[r] + pyy * ty[r] + pz * tz[r]) +
                      tu[r]);
      tx[r] = sc * (py * t0[r] - tx[r]);
      ty[r] = sc * (pyy * t0[r] - ty[r]);
      tz[r] = sc * (pz * t0[r] - tz[r]);
    }
  }


  // Per-point force and its contributions to F, K, U.
  const double G = A.G > 0 ? A.G : G_at(D, A.t);
  const double coef = -(G / D.Z) * D.coefL;
  const double ucoef = (G / D.Z) * D.coefL / (D.p + 1.0);
  double w[13];
#pragma unroll
  for (int e = 0; e < 13; ++e) w[e] = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = ii[r];
    if (i >= A.M) continue;
    double gi = 1.0;
    if (D.g_mode == 1.0) gi = (double)A.aY[i] / D.abar;
    const double fx = coef * gi * tx[r], fy = coef * gi * ty[r], fz = coef * gi * tz[r];
    const double mi = A.mY ? (double)A.mY[i] : 1.0;
    const double ex = (double)A.y0x[i] - D.ybar0[0], ey = (double)A.y0y[i] - D.ybar0[1],
                 ez = (double)A.y0z[i] - D.ybar0[2];
    const double cx = sR[0] * ex + sR[1] * ey + sR[2] * ez;
    const double cy = sR[3] * ex + sR[4] * ey + sR[5] * ez;
    const double cz = sR[6] * ex + sR[7] * ey + sR[8] * ez;
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
      double* fp = A.fpart + ((int64_t)chunk * A.M + i) * 3;
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
  const int n_iblk = (A.M + F_BT * R - 1) / (F_BT * R);
  force_block<R, PM, WU, WF, SM>(A, blockIdx.x % n_iblk, blockIdx.x / n_iblk, blockIdx.x, s_ref, s_lw, s_red);
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
  for (int it = blockIdx.x; it < B.n_items; it += gridDim.x) {
    const int4 item = B.items[it];  // (registration, template block, chunk, output slot)
    const RegDesc& g = B.regs[item.x];
    ForceArgs A{g.y0x, g.y0y, g.y0z, g.aY, g.mY, B.ref4 + g.ref_off, B.reflw + g.ref_off,
                B.poses + (int64_t)13 * item.x, B.dvs + item.x, g.M, g.N, B.chunk_len, 0, B.t, 0.0, B.wpart, nullptr,
                g.perm};
    force_block<R, PM, WU, false, false>(A, item.y, item.z, item.w, s_ref, s_lw, s_red);
  }
}

// f_out[i] = sum over chunks of the per-chunk forces (fixed order).
__global__ __launch_bounds__(256) void reduce_f_kernel(const double* __restrict__ fpart, int n_chunks, int M,
                                                       float* __restrict__ f_out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * 3) return;
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += fpart[(int64_t)c * M * 3 + e];
  f_out[e] = (float)s;
}

hipError_t launch_prepare(const float* aX, const float* wX, int64_t N, const float* aY, const float* mY, int64_t M,
                          const double* mom_t, const double* mom_r, const PrepParams& P, Derived* out, hipStream_t st) {
  hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(1024), 0, st, aX, wX, N, aY, mY, M, mom_t, mom_r, P, out);
  return hipGetLastError();
}

hipError_t launch_partition(const float* aY, int M, Derived* dv, int* perm, hipStream_t st) {
  hipLaunchKernelGGL(partition_kernel, dim3(1), dim3(1024), 0, st, aY, M, dv, perm);
  return hipGetLastError();
}

hipError_t launch_partition_batch(const RegDesc* regs, int B, Derived* dvs, hipStream_t st) {
  hipLaunchKernelGGL(partition_batch_kernel, dim3(B), dim3(1024), 0, st, regs, dvs);
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

int force_points_per_block(int R) { return F_BT * R; }
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

hipError_t launch_reduce_f(const double* fpart, int n_chunks, int M, float* f_out, hipStream_t st) {
  const int64_t n = (int64_t)M * 3;
  hipLaunchKernelGGL(reduce_f_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, fpart, n_chunks, M, f_out);
  return hipGetLastError();
}

}  // namespace sgr
