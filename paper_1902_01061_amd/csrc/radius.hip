// Curvature of radius neighbourhoods (Sec. IV: neighbourhood radius sqrt(eX)
// for the reference and sqrt(eY) for the template, eX and eY the largest
// covariance eigenvalues of Sec. III-B).
//
// With the paper's radius a neighbourhood holds a large part of the cloud,
// so a spatial grid would visit nearly every cell: the kernel scans every
// point.  A block owns 64 queries (one per lane) and its four waves split
// each LDS tile of 256 points four ways, so a cloud of n points gives n/64
// blocks and every SIMD has several waves.  Membership is the key of the
// nearest-neighbour search, float32 ((dx*dx + dy*dy) + dz*dz) with every
// operation rounded on its own (this file is compiled without contraction),
// compared with the float32 threshold r2; the query itself is a member.
// Each member adds its offset from the query (the difference of two floats,
// exact in FP64 for coordinates of comparable magnitude) to FP64 moments:
// count, first and second.  The four waves' moments are then added in a
// fixed order, so the result does not depend on scheduling, and the
// covariance (1/n, centred at the members' mean) gives the surface variation
// lambda_min / trace.
#include "common.h"
#include "launch.h"

namespace sgr {

namespace {

constexpr int RD_BT = 256;  // threads per block
constexpr int RD_Q = 64;    // queries per block
constexpr int RD_TILE = 256;

struct Mom {
  double s[3];
  double c[6];  // xx, yy, zz, xy, xz, yz
  int n;
};

__global__ __launch_bounds__(RD_BT) void radius_desc_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                            const float* __restrict__ Zc, int n,
                                                            const double* __restrict__ mom, double scale2, float r2_in,
                                                            float* __restrict__ a_out, int32_t* __restrict__ cnt_out) {
  __shared__ float4 tf[RD_TILE];
  __shared__ double td[RD_TILE][3];
  __shared__ double red[3][10][RD_Q];
  __shared__ int redn[3][RD_Q];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = blockIdx.x * RD_Q + lane;
  const bool valid = q < n;
  const float r2 = mom ? (float)(scale2 * mom[9]) : r2_in;
  const float qx = valid ? X[q] : 0.f, qy = valid ? Y[q] : 0.f, qz = valid ? Zc[q] : 0.f;
  const double qxd = qx, qyd = qy, qzd = qz;
  Mom m = {{0, 0, 0}, {0, 0, 0, 0, 0, 0}, 0};
  for (int base = 0; base < n; base += RD_TILE) {
    const int j = base + threadIdx.x;
    __syncthreads();
    if (j < n) {
      const float x = X[j], y = Y[j], z = Zc[j];
      tf[threadIdx.x] = make_float4(x, y, z, 0.f);
      td[threadIdx.x][0] = x;
      td[threadIdx.x][1] = y;
      td[threadIdx.x][2] = z;
    }
    __syncthreads();
    // wave w takes points w, w + 4, w + 8, ... of the tile
    const int cnt = min(RD_TILE, n - base);
    for (int jj = w; jj < cnt; jj += 4) {
      const float4 p = tf[jj];
      const float dx = p.x - qx, dy = p.y - qy, dz = p.z - qz;
      const float key = (dx * dx + dy * dy) + dz * dz;
      if (key <= r2) {
        const double ex = td[jj][0] - qxd, ey = td[jj][1] - qyd, ez = td[jj][2] - qzd;
        m.n += 1;
        m.s[0] += ex;
        m.s[1] += ey;
        m.s[2] += ez;
        m.c[0] = fma(ex, ex, m.c[0]);
        m.c[1] = fma(ey, ey, m.c[1]);
        m.c[2] = fma(ez, ez, m.c[2]);
        m.c[3] = fma(ex, ey, m.c[3]);
        m.c[4] = fma(ex, ez, m.c[4]);
        m.c[5] = fma(ey, ez, m.c[5]);
      }
    }
  }
  if (w > 0) {
    for (int c = 0; c < 3; ++c) red[w - 1][c][lane] = m.s[c];
    for (int c = 0; c < 6; ++c) red[w - 1][3 + c][lane] = m.c[c];
    redn[w - 1][lane] = m.n;
  }
  __syncthreads();
  if (w > 0 || !valid) return;
  for (int v = 0; v < 3; ++v) {
    for (int c = 0; c < 3; ++c) m.s[c] += red[v][c][lane];
    for (int c = 0; c < 6; ++c) m.c[c] += red[v][3 + c][lane];
    m.n += redn[v][lane];
  }
  float a = NAN;  // no member: a non-finite query
  if (m.n > 0) {
    const double inv = 1.0 / (double)m.n;
    const double mx = m.s[0] * inv, my = m.s[1] * inv, mz = m.s[2] * inv;
    double C[6] = {m.c[0] * inv - mx * mx, m.c[1] * inv - my * my, m.c[2] * inv - mz * mz,
                   m.c[3] * inv - mx * my, m.c[4] * inv - mx * mz, m.c[5] * inv - my * mz};
    double lam[3];
    eig_psd3(C, lam);
    const double tr = C[0] + C[1] + C[2];
    a = (tr > 0.0) ? (float)(lam[2] / tr) : 0.f;
  }
  if (a_out) a_out[q] = a;
  if (cnt_out) cnt_out[q] = m.n;
}

}  // namespace

hipError_t launch_radius_desc(const float* x, const float* y, const float* z, int n, const double* mom, double scale2,
                              float r2, float* a_out, int32_t* cnt_out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(radius_desc_kernel, dim3((unsigned)((n + RD_Q - 1) / RD_Q)), dim3(RD_BT), 0, st, x, y, z, n,
                     mom, scale2, r2, a_out, cnt_out);
  return hipGetLastError();
}

}  // namespace sgr
