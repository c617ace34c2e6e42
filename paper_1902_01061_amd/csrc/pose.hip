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
#include "update.h"

namespace sgr {

// 512 threads: the single-thread update keeps its FP64 state in registers
// (a 1024-thread block would cap it at 128 VGPRs and spill); its other inputs
// are loaded before the partial rows are summed, with 16 loads in flight per
// thread (up to 1024 rows per round).
__global__ __launch_bounds__(512) void update_kernel(const double* __restrict__ wpart, int nblk,
                                                      const double* pose_in, double* pose_out,
                                                      Derived* __restrict__ dv, int t, double G_fixed, int do_update,
                                                      double* __restrict__ wrench_out, double* __restrict__ stats_row) {
  __shared__ double lds[512 / 4];
  UpdateIn u;
  if (threadIdx.x == 0) update_load(dv, pose_in, t, G_fixed, u);
  double W[13];
  sum_partials<512, 16>(wpart, nblk, lds, W);
  if (threadIdx.x == 0) update_apply(W, u, pose_out, dv, do_update, wrench_out, stats_row);
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
  double* pose = poses + 13 * (int64_t)r;
  UpdateIn u;
  if (threadIdx.x == 0) update_load(dvs + r, pose, t, 0.0, u);
  double W[13];
  sum_partials<256, 16>(wpart + (int64_t)g.wslot0 * WR_STRIDE, g.n_items, lds, W);
  if (threadIdx.x == 0) {
    update_apply(W, u, pose, dvs + r, do_update, nullptr, stats ? stats + ((int64_t)r * E + t) * STATS_STRIDE : nullptr);
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
// One wave (its launch): the bound lets the single thread keep its FP64
// state in registers (the default bound of 1 024 threads spilled it).
__global__ __launch_bounds__(64) void update_bwd_kernel(const double* __restrict__ pose_in,
                                                        const double* __restrict__ W,
                                                        const double* __restrict__ gpose_out,
                                                        const Derived* __restrict__ dv, double* __restrict__ gpose_in,
                                                        double* __restrict__ gW) {
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
