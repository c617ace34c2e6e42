// The rigid update of Sec. III-B (FP64, one thread) and the fixed-order sum
// of the wrench partials that feeds it; included by the update kernels.
#pragma once
#include "common.h"

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

// Everything the update reads besides the wrench.  The thread that runs
// the update loads it before the wrench rows are summed (update_load), so
// that both sets of loads are in flight together, then applies the update
// (update_apply).  Every field of the constant block it reads is loaded into
// registers first, and the three it changes (status, warm-start vectors,
// previous translation) are stored at the end: reading them in place would
// order each later load behind those stores.  pose_in and pose_out may be
// the same array (the pose is updated in place), so neither is declared
// __restrict__; the pose is read into registers before anything is stored.
struct UpdateIn {
  double G;
  double ybar0[3], SigY0[6], Vw[9], dprev[3];
  double Mcount, dt2, lamX, lamY0, Mtot, momentum;
  double P[13];
  int32_t status;
  bool cold;
};

__device__ inline void update_load(const Derived* __restrict__ dv, const double* pose_in, int t, double G_fixed,
                                   UpdateIn& u) {
  u.G = G_fixed > 0 ? G_fixed : G_sched(*dv, t);
  u.cold = dv->cold_svd != 0;
  for (int e = 0; e < 3; ++e) u.ybar0[e] = dv->ybar0[e];
  for (int e = 0; e < 6; ++e) u.SigY0[e] = dv->SigY0[e];
  // cold: the SVD starts from the identity, which is what it does without a
  // warm start, to the bit
  for (int e = 0; e < 9; ++e) u.Vw[e] = u.cold ? ((e % 4 == 0) ? 1.0 : 0.0) : dv->Vw[e];
  for (int e = 0; e < 3; ++e) u.dprev[e] = dv->dprev[e];
  u.Mcount = dv->Mcount;
  u.dt2 = dv->dt2;
  u.lamX = dv->lamX;
  u.lamY0 = dv->lamY0;
  u.Mtot = dv->Mtot;
  u.momentum = dv->momentum;
  for (int e = 0; e < 13; ++e) u.P[e] = pose_in[e];
  u.status = dv->status;
}

// The update itself (one thread).
__device__ inline void update_apply(const double W[13], const UpdateIn& u, double* pose_out,
                                    Derived* __restrict__ dv, int do_update, double* __restrict__ wrench_out,
                                    double* __restrict__ stats_row) {
  const double G = u.G;
  const bool cold = u.cold;
  double ybar0[3], SigY0[6], Vw[9], dprev[3];
  for (int e = 0; e < 3; ++e) ybar0[e] = u.ybar0[e];
  for (int e = 0; e < 6; ++e) SigY0[e] = u.SigY0[e];
  for (int e = 0; e < 9; ++e) Vw[e] = u.Vw[e];
  for (int e = 0; e < 3; ++e) dprev[e] = u.dprev[e];
  const double Mcount = u.Mcount, dt2 = u.dt2, lamX = u.lamX, lamY0 = u.lamY0, Mtot = u.Mtot, momentum = u.momentum;
  if (wrench_out) {
    for (int e = 0; e < 13; ++e) wrench_out[e] = W[e];
  }
  double P[13];
  for (int e = 0; e < 13; ++e) P[e] = u.P[e];
  double Pn[13];
  for (int e = 0; e < 13; ++e) Pn[e] = P[e];
  double c = 1.0;
  int32_t st = u.status;
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
      const double dt2_m = dt2 / Mtot;
      for (int r = 0; r < 3; ++r) d[r] = dt2_m * W[WR_F + r];
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

__device__ inline void pose_update(const double W[13], const double* pose_in, double* pose_out,
                                   Derived* __restrict__ dv, int t, double G_fixed, int do_update,
                                   double* __restrict__ wrench_out, double* __restrict__ stats_row) {
  UpdateIn u;
  update_load(dv, pose_in, t, G_fixed, u);
  update_apply(W, u, pose_out, dv, do_update, wrench_out, stats_row);
}

}  // namespace sgr
