// Rigid update of Sec. III-B in FP64: sum the block wrench partials in a
// fixed order, then one thread applies
//   translation (eq. 5.5):  d = dt2 F / sum_i m_i           (v = 0, Sec. IV)
//   rotation (eq. 6):       C = Y_D^T Y = M Sigma_Y + dt2 K, Kabsch on C
//                           (Y_D = Y + dt2 f, both centred; K = sum_i f_i (y_i - ybar)^T)
//   scale (eq. 8):          c = sqrt(lambda_max(Sigma_X) / lambda_max(Sigma_Y(t))),
//                           lambda_max(Sigma_Y(t)) = s^2 lambda_max(Sigma_Y0)
//   update (eq. 9):         Y(t+1) = c (Y - ybar) R + ybar + d   (row vectors)
// folded into the pose T(y) = s R y + t of the input template, then
// re-orthonormalised (one Newton-Schulz step).  A non-finite or rank-deficient
// update leaves the pose unchanged and sets the device status word.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace sgr {

__device__ inline double G_sched(const Derived& D, int t) {
  return 0.1 * D.G1 + 0.9 * D.G1 / (1.0 + exp(-(((double)t - 1.0) - 0.5 * D.E)));
}

// Sum of `n` wrench partial rows (WR_STRIDE doubles each) starting at
// `wpart` (16-byte aligned), in a fixed order; the result W[0..12] is valid
// in thread 0 only.  The rows are read as one contiguous array of double
// pairs: thread t always takes the pair 2 (t % 8), 2 (t % 8) + 1 (BT is a
// multiple of 64 and WR_STRIDE is 16) of rows t / 8, t / 8 + BT / 8, ...,
// U loads in flight per thread, since the rows were written by blocks on
// every XCD and each round trip is long.  The eight lanes of a wave that
// hold the same pair are added by shuffles, then the waves in order through
// LDS (lds: BT / 4 doubles).  Components 13..15 are padding and are summed
// but not used.
template <int BT, int U>
__device__ inline void sum_partials(const double* __restrict__ wpart, int n, double* lds, double W[13]) {
  static_assert(WR_STRIDE == 16 && BT % 64 == 0, "one component pair per lane");
  const double2* __restrict__ p = reinterpret_cast<const double2*>(wpart);
  const int total = n * (WR_STRIDE / 2);
  double a = 0.0, b = 0.0;
  for (int base = threadIdx.x; base < total; base += U * BT) {
    double2 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int e = base + k * BT;
      v[k] = e < total ? p[e] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      a += v[k].x;
      b += v[k].y;
    }
  }
#pragma unroll
  for (int off = 8; off < 64; off <<= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane < 8) {
    lds[w * 16 + 2 * lane] = a;
    lds[w * 16 + 2 * lane + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int e = 0; e < 13; ++e) {
      double s = 0.0;
      for (int ww = 0; ww < BT / 64; ++ww) s += lds[ww * 16 + e];
      W[e] = s;
    }
  }
}

// The update itself (one thread).  Every field of the constant block it
// reads is loaded into registers first, and the three it changes (status,
// warm-start vectors, previous translation) are stored at the end: reading
// them in place would order each later load behind those stores.  pose_in
// and pose_out may be the same array (the pose is updated in place), so
// neither is declared __restrict__; the pose is read into registers before
// anything is stored.
__device__ void pose_update(const double W[13], const double* pose_in, double* pose_out,
                            Derived* __restrict__ dv, int t, double G_fixed, int do_update,
                            double* __restrict__ wrench_out, double* __restrict__ stats_row) {
  const double G = G_fixed > 0 ? G_fixed : G_sched(*dv, t);
  const bool cold = dv->cold_svd != 0;
  double ybar0[3], SigY0[6], Vw[9], dprev[3];
  for (int e = 0; e < 3; ++e) ybar0[e] = dv->ybar0[e];
  for (int e = 0; e < 6; ++e) SigY0[e] = dv->SigY0[e];
  // cold: the SVD starts from the identity, which is what it does without a
  // warm start, to the bit
  for (int e = 0; e < 9; ++e) Vw[e] = cold ? ((e % 4 == 0) ? 1.0 : 0.0) : dv->Vw[e];
  for (int e = 0; e < 3; ++e) dprev[e] = dv->dprev[e];
  const double Mcount = dv->Mcount, dt2 = dv->dt2, lamX = dv->lamX, lamY0 = dv->lamY0, Mtot = dv->Mtot,
               momentum = dv->momentum;
  if (wrench_out) {
    for (int e = 0; e < 13; ++e) wrench_out[e] = W[e];
  }
  double P[13];
  for (int e = 0; e < 13; ++e) P[e] = pose_in[e];
  double Pn[13];
  for (int e = 0; e < 13; ++e) Pn[e] = P[e];
  double c = 1.0;
  int32_t st = dv->status;
  if (do_update && st == 0) {
    const double s = P[0];
    const double* R = P + 1;
    const double* tv = P + 10;
    bool ok = true;
    for (int e = 0; e < 12; ++e) ok &= isfinite(W[e]);
    // ybar = s R ybar0 + t ; Sigma_Y = s^2 R Sigma_Y0 R^T
    double yb[3];
    for (int r = 0; r < 3; ++r)
      yb[r] = s * (R[3 * r] * ybar0[0] + R[3 * r + 1] * ybar0[1] + R[3 * r + 2] * ybar0[2]) + tv[r];
    const double S0[9] = {SigY0[0], SigY0[3], SigY0[4], SigY0[3], SigY0[1],
                          SigY0[5], SigY0[4], SigY0[5], SigY0[2]};
    double RS[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) RS[3 * r + q] = R[3 * r] * S0[q] + R[3 * r + 1] * S0[3 + q] + R[3 * r + 2] * S0[6 + q];
    double C[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        const double sig = s * s * (RS[3 * r] * R[3 * q] + RS[3 * r + 1] * R[3 * q + 1] + RS[3 * r + 2] * R[3 * q + 2]);
        C[3 * r + q] = Mcount * sig + dt2 * W[WR_K + 3 * r + q];
      }
    for (int e = 0; e < 9; ++e) ok &= isfinite(C[e]);
    double Rk[9];
    if (!ok) {
      st |= ST_NONFINITE;
    } else if (!kabsch_rot(C, Rk, Vw)) {
      st |= ST_SINGULAR;
    } else {
      c = sqrt(lamX / (s * s * lamY0));
      double d[3];
      for (int r = 0; r < 3; ++r) d[r] = dt2 * W[WR_F + r] / Mtot;
      // velocity state: the share momentum of the previous translation
      if (momentum != 0.0)
        for (int r = 0; r < 3; ++r) d[r] += momentum * dprev[r];
      // column form: y' = c Rk^T (y - ybar) + ybar + d
      double Rn[9];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) Rn[3 * r + q] = Rk[r] * R[q] + Rk[3 + r] * R[3 + q] + Rk[6 + r] * R[6 + q];
      // one Newton-Schulz step towards the nearest rotation: Rn (3I - Rn^T Rn)/2
      double RtR[9];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) RtR[3 * r + q] = Rn[r] * Rn[q] + Rn[3 + r] * Rn[3 + q] + Rn[6 + r] * Rn[6 + q];
      double Ro[9];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k) acc += Rn[3 * r + k] * ((k == q ? 3.0 : 0.0) - RtR[3 * k + q]);
          Ro[3 * r + q] = 0.5 * acc;
        }
      double tn[3];
      for (int r = 0; r < 3; ++r) {
        const double dv0 = tv[0] - yb[0], dv1 = tv[1] - yb[1], dv2 = tv[2] - yb[2];
        tn[r] = c * (Rk[r] * dv0 + Rk[3 + r] * dv1 + Rk[6 + r] * dv2) + yb[r] + d[r];
      }
      const double sn = c * s;
      bool fin = isfinite(sn);
      for (int e = 0; e < 9; ++e) fin &= isfinite(Ro[e]);
      for (int e = 0; e < 3; ++e) fin &= isfinite(tn[e]);
      if (!fin) {
        st |= ST_NONFINITE;
      } else if (!(sn > 1e-6 && sn < 1e6)) {
        st |= ST_SCALE;
      } else {
        Pn[0] = sn;
        for (int e = 0; e < 9; ++e) Pn[1 + e] = Ro[e];
        for (int e = 0; e < 3; ++e) Pn[10 + e] = tn[e];
        for (int e = 0; e < 3; ++e) dprev[e] = d[e];
      }
    }
    dv->status = st;
    if (!cold)
      for (int e = 0; e < 9; ++e) dv->Vw[e] = Vw[e];
    for (int e = 0; e < 3; ++e) dv->dprev[e] = dprev[e];
  }
  if (pose_out) {
    for (int e = 0; e < 13; ++e) pose_out[e] = Pn[e];
  }
  if (stats_row) {
    stats_row[ST_G] = G;
    for (int e = 0; e < 12; ++e) stats_row[ST_F + e] = W[e];
    stats_row[ST_U] = W[WR_U];
    for (int e = 0; e < 13; ++e) stats_row[ST_POSE + e] = Pn[e];
    stats_row[ST_C] = c;
    stats_row[ST_STATUS] = (double)st;
    for (int e = ST_STATUS + 1; e < STATS_STRIDE; ++e) stats_row[e] = 0.0;
  }
}

// 512 threads: the single-thread update keeps its FP64 state in registers
// (a 1024-thread block would cap it at 128 VGPRs and spill), and 32 loads in
// flight per thread still read up to 2048 partial rows in one round.
__global__ __launch_bounds__(512) void update_kernel(const double* __restrict__ wpart, int nblk,
                                                      const double* pose_in, double* pose_out,
                                                      Derived* __restrict__ dv, int t, double G_fixed, int do_update,
                                                      double* __restrict__ wrench_out, double* __restrict__ stats_row) {
  __shared__ double lds[512 / 4];
  double W[13];
  sum_partials<512, 32>(wpart, nblk, lds, W);
  if (threadIdx.x == 0) pose_update(W, pose_in, pose_out, dv, t, G_fixed, do_update, wrench_out, stats_row);
}

// One block per registration of a batch; its items own the wrench slots
// [wslot0, wslot0 + n_items).  energy_out[r] (nullable) receives U.
__global__ __launch_bounds__(256) void update_batch_kernel(const double* __restrict__ wpart,
                                                           const RegDesc* __restrict__ regs, double* poses,
                                                           Derived* __restrict__ dvs, int t, int do_update,
                                                           double* __restrict__ energy_out, double* __restrict__ stats,
                                                           int E) {
  __shared__ double lds[256 / 4];
  const int r = blockIdx.x;
  const RegDesc& g = regs[r];
  double W[13];
  sum_partials<256, 16>(wpart + (int64_t)g.wslot0 * WR_STRIDE, g.n_items, lds, W);
  if (threadIdx.x == 0) {
    double* pose = poses + 13 * (int64_t)r;
    pose_update(W, pose, pose, dvs + r, t, 0.0, do_update, nullptr,
                stats ? stats + ((int64_t)r * E + t) * STATS_STRIDE : nullptr);
    if (energy_out) energy_out[r] = W[WR_U];
  }
}

// Multi-start initial poses: rotate the template by R0[s] about its centroid.
__global__ void init_multistart_kernel(const double* __restrict__ R0, int S, const double* __restrict__ mom_t,
                                       double* __restrict__ poses) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const double* R = R0 + 9 * (int64_t)s;
  double* P = poses + 13 * (int64_t)s;
  P[0] = 1.0;
  for (int e = 0; e < 9; ++e) P[1 + e] = R[e];
  for (int r = 0; r < 3; ++r)
    P[10 + r] = mom_t[r] - (R[3 * r] * mom_t[0] + R[3 * r + 1] * mom_t[1] + R[3 * r + 2] * mom_t[2]);
}

// Index of the smallest value (ties: the lowest index; NaN never wins).
__global__ void argmin_kernel(const double* __restrict__ v, int n, int32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  int best = -1;
  for (int i = 0; i < n; ++i)
    if (!isnan(v[i]) && (best < 0 || v[i] < v[best])) best = i;
  out[0] = best;
}

hipError_t launch_update_batch(const double* wpart, const RegDesc* regs, int B, double* poses, Derived* dvs, int t,
                               int do_update, double* energy_out, double* stats, int E, hipStream_t st) {
  hipLaunchKernelGGL(update_batch_kernel, dim3(B), dim3(256), 0, st, wpart, regs, poses, dvs, t, do_update, energy_out,
                     stats, E);
  return hipGetLastError();
}

hipError_t launch_init_multistart(const double* R0, int S, const double* mom_t, double* poses, hipStream_t st) {
  hipLaunchKernelGGL(init_multistart_kernel, dim3((S + 63) / 64), dim3(64), 0, st, R0, S, mom_t, poses);
  return hipGetLastError();
}

hipError_t launch_argmin(const double* v, int n, int32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(argmin_kernel, dim3(1), dim3(64), 0, st, v, n, out);
  return hipGetLastError();
}


__global__ void fill_kernel(double* __restrict__ p, int n, double v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_f_kernel(float* __restrict__ p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_i_kernel(int* __restrict__ p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t launch_fill_i(int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(fill_i_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

__global__ void identity_pose_kernel(double* __restrict__ pose) {
  const int e = threadIdx.x;
  if (e < 13) pose[e] = (e == 0 || e == 1 || e == 5 || e == 9) ? 1.0 : 0.0;
}

hipError_t launch_fill(double* p, int n, double v, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f(float* p, int64_t n, float v, hipStream_t st) {
  hipLaunchKernelGGL(fill_f_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_identity_pose(double* pose, hipStream_t st) {
  hipLaunchKernelGGL(identity_pose_kernel, dim3(1), dim3(64), 0, st, pose);
  return hipGetLastError();
}

hipError_t launch_update(const double* wpart, int nblk, const double* pose_in, double* pose_out, Derived* dv, int t,
                         double G_fixed, int do_update, double* wrench_out, double* stats_row, hipStream_t st) {
  hipLaunchKernelGGL(update_kernel, dim3(1), dim3(512), 0, st, wpart, nblk, pose_in, pose_out, dv, t, G_fixed,
                     do_update, wrench_out, stats_row);
  return hipGetLastError();
}


// ---------------------------------------------------------------- adjoint
// Reverse-mode derivative of one rigid update (Sec. III-B, eqs. 5.5, 6, 8,
// 9 as in pose_update) with respect to the pose it starts from and the
// wrench (F, K) it consumes, given the cotangent of the pose it produces.
// With Q the Kabsch rotation, i.e. the orthogonal polar factor of C^T
// (C^T = Q H, H = U' S' U'^T with the signed singular values of C), a
// cotangent Qbar pulls back to Cbar = -2 Z Q^T, where Z = [z]x is the skew
// solution of H Z + Z H = skew(Q^T Qbar): (tr H I - H) z = s.  The new
// scale c s = sqrt(lambda_X / lambda_Y0) does not depend on the pose, and
// the Newton-Schulz step Ro = Rn (3I - Rn^T Rn) / 2 is differentiated as
// written.  Assumes the forward update was applied (status 0).
__global__ void update_bwd_kernel(const double* __restrict__ pose_in, const double* __restrict__ W,
                                  const double* __restrict__ gpose_out, const Derived* __restrict__ dv,
                                  double* __restrict__ gpose_in, double* __restrict__ gW) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const Derived& D = *dv;
  const double s = pose_in[0];
  double R[9], tv[3];
  for (int e = 0; e < 9; ++e) R[e] = pose_in[1 + e];
  for (int e = 0; e < 3; ++e) tv[e] = pose_in[10 + e];
  const double S0[9] = {D.SigY0[0], D.SigY0[3], D.SigY0[4], D.SigY0[3], D.SigY0[1],
                        D.SigY0[5], D.SigY0[4], D.SigY0[5], D.SigY0[2]};
  // forward quantities
  double yb[3], Ry0[3];
  for (int r = 0; r < 3; ++r) {
    Ry0[r] = R[3 * r] * D.ybar0[0] + R[3 * r + 1] * D.ybar0[1] + R[3 * r + 2] * D.ybar0[2];
    yb[r] = s * Ry0[r] + tv[r];
  }
  double RS[9], RSRt[9], C[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) RS[3 * r + q] = R[3 * r] * S0[q] + R[3 * r + 1] * S0[3 + q] + R[3 * r + 2] * S0[6 + q];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) {
      RSRt[3 * r + q] = RS[3 * r] * R[3 * q] + RS[3 * r + 1] * R[3 * q + 1] + RS[3 * r + 2] * R[3 * q + 2];
      C[3 * r + q] = D.Mcount * s * s * RSRt[3 * r + q] + D.dt2 * W[WR_K + 3 * r + q];
    }
  double sv[3], u[3][3], v[3][3];
  svd3(C, sv, u, v);
  double u3[3], v3[3];
  cross3(u[0], u[1], u3);
  cross3(v[0], v[1], v3);
  const double sg = ((u3[0] * u[2][0] + u3[1] * u[2][1] + u3[2] * u[2][2]) < 0 ? -1.0 : 1.0) *
                    ((v3[0] * v[2][0] + v3[1] * v[2][1] + v3[2] * v[2][2]) < 0 ? -1.0 : 1.0);
  const double s1 = sv[0], s2 = sv[1], s3 = sg * sv[2];  // C = U' diag(s1, s2, s3) V'^T
  const double* Uc[3] = {u[0], u[1], u3};
  double Q[9];
  for (int r = 0; r < 3; ++r)
    for (int c2 = 0; c2 < 3; ++c2) Q[3 * r + c2] = v[0][r] * u[0][c2] + v[1][r] * u[1][c2] + v3[r] * u3[c2];
  const double c = sqrt(D.lamX / (s * s * D.lamY0));
  double Rn[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) Rn[3 * r + q] = Q[r] * R[q] + Q[3 + r] * R[3 + q] + Q[6 + r] * R[6 + q];
  double RtR[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) RtR[3 * r + q] = Rn[r] * Rn[q] + Rn[3 + r] * Rn[3 + q] + Rn[6 + r] * Rn[6 + q];
  // cotangents of the output pose
  double Rob[9], tnb[3];
  for (int e = 0; e < 9; ++e) Rob[e] = gpose_out[1 + e];
  for (int e = 0; e < 3; ++e) tnb[e] = gpose_out[10 + e];
  // Newton-Schulz: Rnb = (Rob B - Rn Rob^T Rn - Rn Rn^T Rob) / 2, B = 3I - Rn^T Rn
  double Rnb[9];
  {
    double T1[9], RoRn[9], RnRnt[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        double a = 0.0, b = 0.0, d = 0.0;
        for (int k = 0; k < 3; ++k) {
          a += Rob[3 * r + k] * ((k == q ? 3.0 : 0.0) - RtR[3 * k + q]);
          b += Rob[3 * k + r] * Rn[3 * k + q];  // (Rob^T Rn)[r][q]
          d += Rn[3 * r + k] * Rn[3 * q + k];   // (Rn Rn^T)[r][q]
        }
        T1[3 * r + q] = a;
        RoRn[3 * r + q] = b;
        RnRnt[3 * r + q] = d;
      }
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        double x = 0.0, y = 0.0;
        for (int k = 0; k < 3; ++k) {
          x += Rn[3 * r + k] * RoRn[3 * k + q];
          y += RnRnt[3 * r + k] * Rob[3 * k + q];
        }
        Rnb[3 * r + q] = 0.5 * (T1[3 * r + q] - x - y);
      }
  }
  // Rn = Q^T R
  double Rb[9], Qb[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < 3; ++k) {
        a += Q[3 * r + k] * Rnb[3 * k + q];
        b += R[3 * r + k] * Rnb[3 * q + k];
      }
      Rb[3 * r + q] = a;
      Qb[3 * r + q] = b;
    }
  // tn = c Q^T (t - ybar) + ybar + d
  double vv[3], vb[3], QTv[3];
  for (int r = 0; r < 3; ++r) vv[r] = tv[r] - yb[r];
  for (int r = 0; r < 3; ++r) {
    vb[r] = c * (Q[3 * r] * tnb[0] + Q[3 * r + 1] * tnb[1] + Q[3 * r + 2] * tnb[2]);
    QTv[r] = Q[r] * vv[0] + Q[3 + r] * vv[1] + Q[6 + r] * vv[2];
  }
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) Qb[3 * r + q] += c * vv[r] * tnb[q];
  const double cb = tnb[0] * QTv[0] + tnb[1] * QTv[1] + tnb[2] * QTv[2];
  double ybb[3], tb[3];
  for (int r = 0; r < 3; ++r) {
    ybb[r] = tnb[r] - vb[r];
    tb[r] = vb[r];
  }
  double sb = -cb * c / s;  // c = sqrt(lambda_X / lambda_Y0) / s
  // polar factor: Cb = -2 Z Q^T, (tr H I - H) z = skew(Q^T Qb)
  double Cb[9];
  {
    double M1[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) M1[3 * r + q] = Q[r] * Qb[q] + Q[3 + r] * Qb[3 + q] + Q[6 + r] * Qb[6 + q];
    const double sk[3] = {0.5 * (M1[7] - M1[5]), 0.5 * (M1[2] - M1[6]), 0.5 * (M1[3] - M1[1])};
    const double den[3] = {s2 + s3, s1 + s3, s1 + s2};
    double z[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 3; ++k) {
      const double w = (Uc[k][0] * sk[0] + Uc[k][1] * sk[1] + Uc[k][2] * sk[2]) / den[k];
      for (int r = 0; r < 3; ++r) z[r] += w * Uc[k][r];
    }
    const double Z[9] = {0.0, -z[2], z[1], z[2], 0.0, -z[0], -z[1], z[0], 0.0};
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q)
        Cb[3 * r + q] = -2.0 * (Z[3 * r] * Q[3 * q] + Z[3 * r + 1] * Q[3 * q + 1] + Z[3 * r + 2] * Q[3 * q + 2]);
  }
  // C = Mcount s^2 R S0 R^T + dt2 K
  {
    double sig = 0.0;
    for (int e = 0; e < 9; ++e) sig += Cb[e] * RSRt[e];
    sb += 2.0 * s * D.Mcount * sig;
    double Sb[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) Sb[3 * r + q] = D.Mcount * s * s * (Cb[3 * r + q] + Cb[3 * q + r]);
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) Rb[3 * r + q] += Sb[3 * r] * RS[q] + Sb[3 * r + 1] * RS[3 + q] + Sb[3 * r + 2] * RS[6 + q];
  }
  // ybar = s R ybar0 + t
  sb += ybb[0] * Ry0[0] + ybb[1] * Ry0[1] + ybb[2] * Ry0[2];
  for (int r = 0; r < 3; ++r) {
    for (int q = 0; q < 3; ++q) Rb[3 * r + q] += s * ybb[r] * D.ybar0[q];
    tb[r] += ybb[r];
  }
  gpose_in[0] = sb;
  for (int e = 0; e < 9; ++e) gpose_in[1 + e] = Rb[e];
  for (int e = 0; e < 3; ++e) gpose_in[10 + e] = tb[e];
  for (int e = 0; e < 3; ++e) gW[WR_F + e] = D.dt2 / D.Mtot * tnb[e];
  for (int e = 0; e < 9; ++e) gW[WR_K + e] = D.dt2 * Cb[e];
  for (int e = 12; e < WR_STRIDE; ++e) gW[e] = 0.0;
}

// World coordinates of the posed template, s R y0 + t (FP64, rounded once).
__global__ __launch_bounds__(256) void pose_points_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                          const float* __restrict__ z, int M,
                                                          const double* __restrict__ pose, float* __restrict__ ox,
                                                          float* __restrict__ oy, float* __restrict__ oz) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const double s = pose[0];
  const double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
  double o[3];
  for (int r = 0; r < 3; ++r) o[r] = s * (pose[1 + 3 * r] * p[0] + pose[2 + 3 * r] * p[1] + pose[3 + 3 * r] * p[2]) + pose[10 + r];
  ox[i] = (float)o[0];
  oy[i] = (float)o[1];
  oz[i] = (float)o[2];
}

// Per-block sums of gy_i y0_i^T (9) and gy_i (3) over the template points.
__global__ __launch_bounds__(256) void pose_grad_partial_kernel(const float* __restrict__ gy, const float* __restrict__ x,
                                                                const float* __restrict__ y,
                                                                const float* __restrict__ z, int M,
                                                                double* __restrict__ part) {
  __shared__ double lds[4 * 12];
  double v[12];
  for (int e = 0; e < 12; ++e) v[e] = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < M; i += gridDim.x * 256) {
    const double g[3] = {(double)gy[3 * i], (double)gy[3 * i + 1], (double)gy[3 * i + 2]};
    const double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
    for (int r = 0; r < 3; ++r) {
      for (int q = 0; q < 3; ++q) v[3 * r + q] += g[r] * p[q];
      v[9 + r] += g[r];
    }
  }
  block_sum<12, 256>(v, lds);
  if (threadIdx.x == 0)
    for (int e = 0; e < 12; ++e) part[(int64_t)blockIdx.x * 12 + e] = v[e];
}

// gpose += the pose cotangent of y_i = s R y0_i + t: sbar += <A, R>,
// Rbar += s A, tbar += g, with A = sum_i gy_i y0_i^T, g = sum_i gy_i.
__global__ __launch_bounds__(256) void pose_grad_final_kernel(const double* __restrict__ part, int nb,
                                                              const double* __restrict__ pose,
                                                              double* __restrict__ gpose) {
  __shared__ double lds[4 * 12];
  double v[12];
  for (int e = 0; e < 12; ++e) v[e] = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256)
    for (int e = 0; e < 12; ++e) v[e] += part[(int64_t)b * 12 + e];
  block_sum<12, 256>(v, lds);
  if (threadIdx.x != 0) return;
  double sA = 0.0;
  for (int e = 0; e < 9; ++e) sA += v[e] * pose[1 + e];
  gpose[0] += sA;
  for (int e = 0; e < 9; ++e) gpose[1 + e] += pose[0] * v[e];
  for (int e = 0; e < 3; ++e) gpose[10 + e] += v[9 + e];
}

__global__ void axpy_kernel(const double* __restrict__ x, int n, double* __restrict__ y) {
  if (threadIdx.x < n) y[threadIdx.x] += x[threadIdx.x];
}

hipError_t launch_update_bwd(const double* pose_in, const double* W, const double* gpose_out, const Derived* dv,
                             double* gpose_in, double* gW, hipStream_t st) {
  hipLaunchKernelGGL(update_bwd_kernel, dim3(1), dim3(64), 0, st, pose_in, W, gpose_out, dv, gpose_in, gW);
  return hipGetLastError();
}

hipError_t launch_pose_points(const float* x, const float* y, const float* z, int M, const double* pose, float* ox,
                              float* oy, float* oz, hipStream_t st) {
  hipLaunchKernelGGL(pose_points_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, x, y, z, M, pose, ox, oy,
                     oz);
  return hipGetLastError();
}

int pose_grad_blocks(int M) { return std::min(256, (M + 255) / 256); }

hipError_t launch_pose_grad(const float* gy, const float* x, const float* y, const float* z, int M, const double* pose,
                            double* part, double* gpose, hipStream_t st) {
  const int nb = pose_grad_blocks(M);
  hipLaunchKernelGGL(pose_grad_partial_kernel, dim3(nb), dim3(256), 0, st, gy, x, y, z, M, part);
  hipLaunchKernelGGL(pose_grad_final_kernel, dim3(1), dim3(256), 0, st, (const double*)part, nb, pose, gpose);
  return hipGetLastError();
}

hipError_t launch_axpy(const double* x, int n, double* y, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3(1), dim3(64), 0, st, x, n, y);
  return hipGetLastError();
}

}  // namespace sgr
