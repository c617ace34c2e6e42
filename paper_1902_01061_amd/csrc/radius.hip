// Curvature of radius neighbourhoods (Sec. IV: neighbourhood radius sqrt(eX)
// for the reference and sqrt(eY) for the template, eX and eY the largest
// covariance eigenvalues of Sec. III-B).
//
// Membership is the key of the nearest-neighbour search, float32
// ((dx*dx + dy*dy) + dz*dz) with every operation rounded on its own (this
// file is compiled without contraction), compared with the float32 threshold
// r2; the query itself is a member.  Each member adds its offset from the
// query (the difference of two floats, exact in FP64 for coordinates of
// comparable magnitude) to FP64 moments: count, first and second.  The
// covariance (1/n, centred at the members' mean) gives the surface variation
// lambda_min / trace.
//
// With the paper's radius a neighbourhood holds about a tenth of a scan, so
// a cell grid would visit most cells, yet most pairs are still far apart.
// The points are put in Morton order (30-bit codes on the cloud's bounding
// cube, radix-sorted, ties by index) and cut into tiles of 64 with a
// bounding box each.  A block of 16 waves owns 64 consecutive queries of
// that order (one per lane).  A tile whose box lies farther than r from the
// box of the block's queries holds no member.  The test is taken in float32
// against r2 (1 + 2^-16) + 2^-100: if the computed squared gap g2 exceeds
// it, the exact one exceeds r2 (1 + 2^-17) + 2^-101 (five roundings of at
// most 2^-24 relative, underflow of at most 2^-149 absolute), and so does
// the exact squared distance of every pair, whose float32 key (five roundings
// again) then exceeds r2.  A tile is never skipped that holds a member, and
// member counts are those of the full scan.  The block first lists the tiles that pass (one
// tile per thread, compacted in tile order), then its waves take the list
// round-robin.  Every lane of a wave reads the same tile point, so the points
// (float32, and an FP64 copy for the member offsets) come through the scalar
// unit into SGPRs.  Points with a non-finite coordinate are members of no
// neighbourhood (their keys are inf or NaN) and are left out of the boxes.
// Each wave visits its tiles in a fixed order and the waves' moments are
// added by a fixed tree, so results do not depend on scheduling.
#include <hipcub/hipcub.hpp>

#include "common.h"
#include "launch.h"

namespace sgr {

namespace {

constexpr int RD_WAVES = 16;
constexpr int RD_BT = 64 * RD_WAVES;  // threads per block
constexpr int RD_Q = 64;              // queries per block
constexpr int RD_TILE = 64;
constexpr int RD_LIST = RD_BT;        // tiles tested per pass, one per thread
constexpr int RD_U = 4;  // tile points loaded ahead
constexpr int BOX_NB = 64;  // blocks of the partial bounding boxes
// Code of a point with a non-finite coordinate: such a point is a member of
// no neighbourhood, so where it sorts changes no result.
constexpr uint32_t CODE_NONFINITE = 0x3fffffffu;
constexpr size_t kAlign = 256;

size_t up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

size_t sort_temp_bytes(int n) {
  size_t tb = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tb, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int*)nullptr, (int*)nullptr, n, 0, 30, (hipStream_t)0);
  return tb;
}

struct RadiusWs {
  float4* P;     // points in Morton order (x, y, z, 0)
  double4* Pd;   // the same in FP64
  int* perm;     // P[q] is point perm[q]
  uint32_t* code_in;
  uint32_t* code_out;
  int* idx;
  float4* tbox;  // per tile: lo, hi
  float* box;    // per block of cloud_box_kernel: lo[3], hi[3]
  void* tmp;
  size_t tmp_bytes;
};

RadiusWs carve(void* ws, int n) {
  char* p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + kAlign - 1) & ~(uintptr_t)(kAlign - 1));
  RadiusWs w;
  const int ntile = (n + RD_TILE - 1) / RD_TILE;
  const size_t npad = (size_t)ntile * RD_TILE;
  w.P = reinterpret_cast<float4*>(p);
  p += up(npad * 16);
  w.Pd = reinterpret_cast<double4*>(p);
  p += up(npad * 32);
  w.perm = reinterpret_cast<int*>(p);
  p += up((size_t)n * 4);
  w.code_in = reinterpret_cast<uint32_t*>(p);
  p += up((size_t)n * 4);
  w.code_out = reinterpret_cast<uint32_t*>(p);
  p += up((size_t)n * 4);
  w.idx = reinterpret_cast<int*>(p);
  p += up((size_t)n * 4);
  w.tbox = reinterpret_cast<float4*>(p);
  p += up((size_t)ntile * 32);
  w.box = reinterpret_cast<float*>(p);
  p += up(BOX_NB * 6 * sizeof(float));
  w.tmp = p;
  w.tmp_bytes = sort_temp_bytes(n);
  return w;
}

__device__ inline bool finite3(float x, float y, float z) { return isfinite(x) && isfinite(y) && isfinite(z); }

__device__ inline float wave_min(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ inline float wave_max(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// Bounding boxes of the finite points of BOX_NB interleaved parts of the
// cloud (block b takes points b*256 + t + k*BOX_NB*256).
__global__ __launch_bounds__(256) void cloud_box_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                        const float* __restrict__ Zc, int n,
                                                        float* __restrict__ box) {
  __shared__ double lds[2 * 256 / 64];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += BOX_NB * 256) {
    const float p[3] = {X[i], Y[i], Zc[i]};
    if (finite3(p[0], p[1], p[2]))
      for (int c = 0; c < 3; ++c) {
        lo[c] = fminf(lo[c], p[c]);
        hi[c] = fmaxf(hi[c], p[c]);
      }
  }
  for (int c = 0; c < 3; ++c) block_range<256>(lo[c], hi[c], lds);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) {
      box[blockIdx.x * 6 + c] = lo[c];
      box[blockIdx.x * 6 + 3 + c] = hi[c];
    }
}

// Ten low bits of v spread to every third bit.
__device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Morton code of every point on the cloud's bounding cube, 1024 cells a side
// (the box: the smallest and largest of the BOX_NB partial boxes).
__global__ __launch_bounds__(256) void morton_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                     const float* __restrict__ Zc, int n,
                                                     const float* __restrict__ part, uint32_t* __restrict__ code,
                                                     int* __restrict__ idx) {
  static_assert(BOX_NB == 64, "one wave reduces the partial boxes");
  __shared__ float s_box[6];
  if (threadIdx.x < 64) {
    float v[6];
    for (int c = 0; c < 6; ++c) v[c] = part[threadIdx.x * 6 + c];
    for (int c = 0; c < 3; ++c) {
      v[c] = wave_min(v[c]);
      v[3 + c] = wave_max(v[3 + c]);
    }
    if (threadIdx.x == 0)
      for (int c = 0; c < 6; ++c) s_box[c] = v[c];
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float p[3] = {X[i], Y[i], Zc[i]};
  uint32_t c = CODE_NONFINITE;
  if (finite3(p[0], p[1], p[2])) {
    const float ext = fmaxf(fmaxf(s_box[3] - s_box[0], s_box[4] - s_box[1]), s_box[5] - s_box[2]);
    // an infinite extent (overflow) or a single point: every code 0
    const float inv = (ext > 0.f && isfinite(ext)) ? 1023.f / ext : 0.f;
    c = 0;
    for (int a = 0; a < 3; ++a) {
      const float f = fminf(1023.f, fmaxf(0.f, (p[a] - s_box[a]) * inv));  // NaN (inf * 0) gives 0
      c |= spread3((uint32_t)f) << a;
    }
  }
  code[i] = c;
  idx[i] = i;
}

// Points in Morton order, padded to whole tiles with NaN points (members of
// no neighbourhood), and the bounding box of each tile of RD_TILE (one wave
// per tile).
__global__ __launch_bounds__(256) void gather_tiles_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                           const float* __restrict__ Zc, int n,
                                                           const int* __restrict__ perm, float4* __restrict__ P,
                                                           double4* __restrict__ Pd, float4* __restrict__ tbox) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int tile = q / RD_TILE;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (q < n) {
    const int j = perm[q];
    const float p[3] = {X[j], Y[j], Zc[j]};
    P[q] = make_float4(p[0], p[1], p[2], 0.f);
    Pd[q] = make_double4(p[0], p[1], p[2], 0.0);
    if (finite3(p[0], p[1], p[2]))
      for (int c = 0; c < 3; ++c) lo[c] = hi[c] = p[c];
  } else if (tile * RD_TILE < n) {
    P[q] = make_float4(NAN, NAN, NAN, 0.f);
    Pd[q] = make_double4(NAN, NAN, NAN, 0.0);
  }
  for (int c = 0; c < 3; ++c) {
    lo[c] = wave_min(lo[c]);
    hi[c] = wave_max(hi[c]);
  }
  if ((threadIdx.x & 63) == 0 && tile * RD_TILE < n) {
    tbox[2 * tile] = make_float4(lo[0], lo[1], lo[2], 0.f);
    tbox[2 * tile + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
  }
}

struct Mom {
  double s[3];
  double c[6];  // xx, yy, zz, xy, xz, yz
  int n;
};

// A value that every lane of the wave holds, in an SGPR.
__device__ inline float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Lower bound of the distance between two boxes along one axis (0 when they
// overlap; +inf when either box is empty), one rounding.
__device__ inline float axis_gap(float lo_a, float hi_a, float lo_b, float hi_b) {
  return fmaxf(0.f, fmaxf(lo_a - hi_b, lo_b - hi_a));
}

__device__ inline void add_member(Mom& m, double ex, double ey, double ez) {
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

__global__ __launch_bounds__(RD_BT) void radius_desc_kernel(const float4* __restrict__ P,
                                                            const double4* __restrict__ Pd,
                                                            const int* __restrict__ perm,
                                                            const float4* __restrict__ tbox, int n,
                                                            const double* __restrict__ mom, double scale2, float r2_in,
                                                            float* __restrict__ a_out, int32_t* __restrict__ cnt_out) {
  __shared__ int s_list[RD_LIST];
  __shared__ int s_cnt[RD_WAVES];
  __shared__ double red[RD_WAVES / 2][10][RD_Q];
  __shared__ int redn[RD_WAVES / 2][RD_Q];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ws = __builtin_amdgcn_readfirstlane(w);  // the wave index, in an SGPR
  const int q = blockIdx.x * RD_Q + lane;
  const bool valid = q < n;
  const float r2 = mom ? (float)(scale2 * mom[9]) : r2_in;
  const float4 qp = valid ? P[q] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float qx = qp.x, qy = qp.y, qz = qp.z;
  const double qxd = qx, qyd = qy, qzd = qz;
  // box of the block's finite queries (the same in every wave)
  const bool fin = valid && finite3(qx, qy, qz);
  const float qlo_x = uniform(wave_min(fin ? qx : INFINITY)), qhi_x = uniform(wave_max(fin ? qx : -INFINITY));
  const float qlo_y = uniform(wave_min(fin ? qy : INFINITY)), qhi_y = uniform(wave_max(fin ? qy : -INFINITY));
  const float qlo_z = uniform(wave_min(fin ? qz : INFINITY)), qhi_z = uniform(wave_max(fin ? qz : -INFINITY));
  const float thr = r2 * (1.0f + 0x1p-16f) + 0x1p-100f;
  Mom m = {{0, 0, 0}, {0, 0, 0, 0, 0, 0}, 0};
  const int ntile = (n + RD_TILE - 1) / RD_TILE;
  for (int t0 = 0; t0 < ntile; t0 += RD_LIST) {
    // the tiles of this pass that may hold a member, listed in tile order
    const int t = t0 + (int)threadIdx.x;
    bool keep = false;
    if (t < ntile) {
      const float4 lo = tbox[2 * t], hi = tbox[2 * t + 1];
      const float gx = axis_gap(lo.x, hi.x, qlo_x, qhi_x);
      const float gy = axis_gap(lo.y, hi.y, qlo_y, qhi_y);
      const float gz = axis_gap(lo.z, hi.z, qlo_z, qhi_z);
      keep = !((gx * gx + gy * gy) + gz * gz > thr);
    }
    const unsigned long long bal = __ballot(keep);
    if (lane == 0) s_cnt[w] = __popcll(bal);
    __syncthreads();
    int off = 0, total = 0;
#pragma unroll 1
    for (int v = 0; v < RD_WAVES; ++v) {
      const int c = s_cnt[v];
      off += v < w ? c : 0;
      total += c;
    }
    if (keep) s_list[off + __popcll(bal & ((1ull << lane) - 1ull))] = t;
    __syncthreads();
    total = __builtin_amdgcn_readfirstlane(total);
    for (int e = ws; e < total; e += RD_WAVES) {
      const int tile = __builtin_amdgcn_readfirstlane(s_list[e]);
      const float4* __restrict__ tp = P + tile * RD_TILE;
      const double4* __restrict__ tpd = Pd + tile * RD_TILE;
#pragma unroll 1
      for (int jj = 0; jj < RD_TILE; jj += RD_U) {
        float4 p[RD_U];
        double4 pd[RD_U];
#pragma unroll
        for (int u = 0; u < RD_U; ++u) {
          p[u] = tp[jj + u];
          pd[u] = tpd[jj + u];
        }
#pragma unroll
        for (int u = 0; u < RD_U; ++u) {
          const float dx = p[u].x - qx, dy = p[u].y - qy, dz = p[u].z - qz;
          const float key = (dx * dx + dy * dy) + dz * dz;
          if (key <= r2) add_member(m, pd[u].x - qxd, pd[u].y - qyd, pd[u].z - qzd);
        }
      }
    }
    __syncthreads();  // the list is rewritten by the next pass
  }
  // fixed tree: wave w < h adds wave w + h's moments, h = 8, 4, 2, 1
  for (int h = RD_WAVES / 2; h >= 1; h >>= 1) {
    if (w >= h && w < 2 * h) {
      for (int c = 0; c < 3; ++c) red[w - h][c][lane] = m.s[c];
      for (int c = 0; c < 6; ++c) red[w - h][3 + c][lane] = m.c[c];
      redn[w - h][lane] = m.n;
    }
    __syncthreads();
    if (w < h) {
      for (int c = 0; c < 3; ++c) m.s[c] += red[w][c][lane];
      for (int c = 0; c < 6; ++c) m.c[c] += red[w][3 + c][lane];
      m.n += redn[w][lane];
    }
    __syncthreads();
  }
  if (w > 0 || !valid) return;
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
  const int o = perm[q];
  if (a_out) a_out[o] = a;
  if (cnt_out) cnt_out[o] = m.n;
}

}  // namespace

size_t radius_desc_workspace(int n) {
  const size_t ntile = ((size_t)n + RD_TILE - 1) / RD_TILE;
  return kAlign + up(ntile * RD_TILE * 16) + up(ntile * RD_TILE * 32) + 4 * up((size_t)n * 4) + up(ntile * 32) + up(BOX_NB * 6 * sizeof(float)) +
         up(sort_temp_bytes(n));
}

hipError_t launch_radius_desc(const float* x, const float* y, const float* z, int n, const double* mom, double scale2,
                              float r2, float* a_out, int32_t* cnt_out, void* ws, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  RadiusWs w = carve(ws, n);
  hipLaunchKernelGGL(cloud_box_kernel, dim3(BOX_NB), dim3(256), 0, st, x, y, z, n, w.box);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned g256 = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(morton_kernel, dim3(g256), dim3(256), 0, st, x, y, z, n, (const float*)w.box, w.code_in, w.idx);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t tb = w.tmp_bytes;
  e = hipcub::DeviceRadixSort::SortPairs(w.tmp, tb, w.code_in, w.code_out, w.idx, w.perm, n, 0, 30, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gather_tiles_kernel, dim3(g256), dim3(256), 0, st, x, y, z, n, (const int*)w.perm, w.P, w.Pd, w.tbox);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(radius_desc_kernel, dim3((unsigned)((n + RD_Q - 1) / RD_Q)), dim3(RD_BT), 0, st,
                     (const float4*)w.P, (const double4*)w.Pd, (const int*)w.perm, (const float4*)w.tbox, n, mom,
                     scale2, r2, a_out, cnt_out);
  return hipGetLastError();
}

}  // namespace sgr
