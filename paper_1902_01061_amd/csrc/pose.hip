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
#include "common.h"
#include "launch.h"

namespace sgr {

__device__ inline double G_sched(const Derived& D, int t) {
  return 0.1 * D.G1 + 0.9 * D.G1 / (1.0 + exp(-(((double)t - 1.0) - 0.5 * D.E)));
}

// Sum of `n` wrench partial rows starting at `wpart` (fixed order); result in
// W[0..12], valid for thread 0 only.
__device__ inline void sum_partials(const double* __restrict__ wpart, int n, double* lds, double W[13]) {
  double v[13];
#pragma unroll
  for (int e = 0; e < 13; ++e) v[e] = 0.0;
  for (int b = threadIdx.x; b < n; b += 256) {
    const double* src = wpart + (int64_t)b * WR_STRIDE;
#pragma unroll
    for (int e = 0; e < 13; ++e) v[e] += src[e];
  }
  block_sum<13, 256>(v, lds);
#pragma unroll
  for (int e = 0; e < 13; ++e) W[e] = v[e];
}

// The update itself (one thread).
__device__ void pose_update(const double W[13], const double* __restrict__ pose_in, double* __restrict__ pose_out,
                            Derived* __restrict__ dv, int t, double G_fixed, int do_update,
                            double* __restrict__ wrench_out, double* __restrict__ stats_row) {
  Derived& D = *dv;
  const double G = G_fixed > 0 ? G_fixed : G_sched(D, t);
  if (wrench_out) {
    for (int e = 0; e < 13; ++e) wrench_out[e] = W[e];
  }
  double P[13];
  for (int e = 0; e < 13; ++e) P[e] = pose_in[e];
  double Pn[13];
  for (int e = 0; e < 13; ++e) Pn[e] = P[e];
  double c = 1.0;
  int32_t st = D.status;
  if (do_update && st == 0) {
    const double s = P[0];
    const double* R = P + 1;
    const double* tv = P + 10;
    bool ok = true;
    for (int e = 0; e < 12; ++e) ok &= isfinite(W[e]);
    // ybar = s R ybar0 + t ; Sigma_Y = s^2 R Sigma_Y0 R^T
    double yb[3];
    for (int r = 0; r < 3; ++r)
      yb[r] = s * (R[3 * r] * D.ybar0[0] + R[3 * r + 1] * D.ybar0[1] + R[3 * r + 2] * D.ybar0[2]) + tv[r];
    const double S0[9] = {D.SigY0[0], D.SigY0[3], D.SigY0[4], D.SigY0[3], D.SigY0[1],
                          D.SigY0[5], D.SigY0[4], D.SigY0[5], D.SigY0[2]};
    double RS[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) RS[3 * r + q] = R[3 * r] * S0[q] + R[3 * r + 1] * S0[3 + q] + R[3 * r + 2] * S0[6 + q];
    double C[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        const double sig = s * s * (RS[3 * r] * R[3 * q] + RS[3 * r + 1] * R[3 * q + 1] + RS[3 * r + 2] * R[3 * q + 2]);
        C[3 * r + q] = D.Mcount * sig + D.dt2 * W[WR_K + 3 * r + q];
      }
    for (int e = 0; e < 9; ++e) ok &= isfinite(C[e]);
    double Rk[9];
    if (!ok) {
      st |= ST_NONFINITE;
    } else if (!kabsch_rot(C, Rk, D.Vw)) {
      st |= ST_SINGULAR;
    } else {
      c = sqrt(D.lamX / (s * s * D.lamY0));
      double d[3];
      for (int r = 0; r < 3; ++r) d[r] = D.dt2 * W[WR_F + r] / D.Mtot;
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
      }
    }
    D.status = st;
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

__global__ __launch_bounds__(256) void update_kernel(const double* __restrict__ wpart, int nblk,
                                                     const double* __restrict__ pose_in, double* __restrict__ pose_out,
                                                     Derived* __restrict__ dv, int t, double G_fixed, int do_update,
                                                     double* __restrict__ wrench_out, double* __restrict__ stats_row) {
  __shared__ double lds[4 * 13];
  double W[13];
  sum_partials(wpart, nblk, lds, W);
  if (threadIdx.x == 0) pose_update(W, pose_in, pose_out, dv, t, G_fixed, do_update, wrench_out, stats_row);
}

// One block per registration of a batch; its items own the wrench slots
// [wslot0, wslot0 + n_items).  energy_out[r] (nullable) receives U.
__global__ __launch_bounds__(256) void update_batch_kernel(const double* __restrict__ wpart,
                                                           const RegDesc* __restrict__ regs, double* __restrict__ poses,
                                                           Derived* __restrict__ dvs, int t, int do_update,
                                                           double* __restrict__ energy_out, double* __restrict__ stats,
                                                           int E) {
  __shared__ double lds[4 * 13];
  const int r = blockIdx.x;
  const RegDesc& g = regs[r];
  double W[13];
  sum_partials(wpart + (int64_t)g.wslot0 * WR_STRIDE, g.n_items, lds, W);
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
  hipLaunchKernelGGL(update_kernel, dim3(1), dim3(256), 0, st, wpart, nblk, pose_in, pose_out, dv, t, G_fixed,
                     do_update, wrench_out, stats_row);
  return hipGetLastError();
}

}  // namespace sgr
