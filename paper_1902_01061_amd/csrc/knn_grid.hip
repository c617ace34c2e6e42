// Exact k nearest neighbours through a uniform grid (the same lists as a
// search over all points: float32 squared distance ((dx*dx + dy*dy) + dz*dz),
// every operation rounded, ties by index), followed by the FP64
// neighbourhood covariance and curvature (Sec. III-A).
//
// 1. grid_setup: bounding box of the finite points and a cell size h with
//    about two points per cell of the bounding volume (fewer cells than the
//    allocated maximum), shrunk for surfaces after a first count;
// 2. counting sort of the points by cell (cell counts, exclusive scan,
//    scatter); the order inside a cell does not matter because candidates
//    are ranked by the (distance, index) key;
// 3. one query per lane, in cell order (neighbouring lanes search the same
//    cells): shells of cells at Chebyshev radius 0, 1, 2, ... are scanned
//    until the current k-th distance is below the distance from the query to
//    the unsearched region (with a margin that covers the float32 rounding
//    of cell assignment and of the key), so no closer point can be missed;
//    a query still open after shell 1 is handed over with its list and
//    resumed where it stopped (a wave per query; in a batch, a lane per
//    query for shell 2, then a wave per query).
#include <utility>
#include <vector>

#include "common.h"
#include "launch.h"

namespace sgr {

struct GridInfo {
  float lo[3];
  float h;
  int dims[3];
  int ncells;
  double ext[3];  // bounding-box extents (for re-sizing the cells)
};

// Cell counts per axis for cell size h, grown by 10 % steps until the grid
// has at most max_cells cells.
__device__ inline void grid_dims(GridInfo& G, double h, int max_cells) {
  int d[3];
  for (int it = 0; it < 200; ++it) {
    long long tot = 1;
    for (int a = 0; a < 3; ++a) {
      d[a] = (int)fmin(1024.0, floor(G.ext[a] / h) + 1.0);
      tot *= d[a];
    }
    if (tot <= max_cells) break;
    h *= 1.1;
  }
  G.h = (float)h;
  for (int a = 0; a < 3; ++a) G.dims[a] = d[a];
  G.ncells = d[0] * d[1] * d[2];
}

constexpr int GQ_BT = 256;
constexpr int KNN_RCAP = 1;  // last shell the one-lane pass searches before handing a query over
constexpr int SCAN_B = 1024;

// Bodies of the grid kernels, shared by the one-cloud kernels and their
// batched forms (a table of clouds, one launch per phase for all of them).
__device__ inline void grid_setup_body(const float* __restrict__ X, const float* __restrict__ Y,
                                       const float* __restrict__ Zc, int n, int max_cells, GridInfo* __restrict__ gi,
                                       int* __restrict__ far, int* __restrict__ far2) {
  // counts of the queries handed over by the one-lane pass (far) and, in a
  // batch, by the pass that resumes them for one more shell (far2)
  if (threadIdx.x == 0) {
    far[0] = 0;
    if (far2) far2[0] = 0;
  }
  __shared__ float red[16][6];
  float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  // the bounding box of the finite points (an infinite coordinate would
  // make the box infinite and the grid one row of cells)
  for (int i = threadIdx.x; i < n; i += 1024) {
    const float p[3] = {X[i], Y[i], Zc[i]};
    if (!(isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))) continue;
    for (int a = 0; a < 3; ++a) {
      v[a] = fminf(v[a], p[a]);
      v[3 + a] = fmaxf(v[3 + a], p[a]);
    }
  }
  for (int a = 0; a < 6; ++a) {
    float m = v[a];
    for (int off = 32; off > 0; off >>= 1) {
      const float o = __shfl_xor(m, off, 64);
      m = a < 3 ? fminf(m, o) : fmaxf(m, o);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][a] = m;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int a = 0; a < 6; ++a)
    for (int w = 1; w < 16; ++w) red[0][a] = a < 3 ? fminf(red[0][a], red[w][a]) : fmaxf(red[0][a], red[w][a]);
  GridInfo G;
  double e[3];
  for (int a = 0; a < 3; ++a) {
    const bool any = red[0][a] <= red[0][3 + a];  // some finite point
    G.lo[a] = any ? red[0][a] : 0.f;
    e[a] = any ? (double)red[0][3 + a] - (double)red[0][a] : 0.0;
  }
  // cell size for about two points per cell of the bounding volume; flat or
  // linear clouds fall back to their non-degenerate extents
  double s[3] = {e[0], e[1], e[2]};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2 - i; ++j)
      if (s[j] < s[j + 1]) {
        const double t = s[j];
        s[j] = s[j + 1];
        s[j + 1] = t;
      }
  // first guess: 2 points per cell of the bounding box (a volume); for
  // surfaces grid_refine_kernel then shrinks the cells
  const double rho = 2.0;
  for (int a = 0; a < 3; ++a) G.ext[a] = e[a];
  double h;
  if (s[2] > 1e-6 * s[0])
    h = cbrt(s[0] * s[1] * s[2] * rho / n);
  else if (s[1] > 1e-6 * s[0])
    h = sqrt(s[0] * s[1] * rho / n);
  else
    h = s[0] * rho / n;
  if (!(h > 0) || !isfinite(h)) h = 1.0;
  grid_dims(G, h, max_cells);
  *gi = G;
}

__global__ __launch_bounds__(1024) void grid_setup_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                          const float* __restrict__ Zc, int n, int max_cells,
                                                          GridInfo* __restrict__ gi, int* __restrict__ far) {
  grid_setup_body(X, Y, Zc, n, max_cells, gi, far, nullptr);
}

// Second look at the cell size, from the first count: scans are surfaces
// (often with dense clusters), whose occupied cells hold many more points
// than the 2 per cell of a volume, and a query inside them meets hundreds of
// candidates.  With mu the mean count of the occupied cells, the cell side
// is scaled by sqrt(6 / mu) when mu > 6 (surface scaling: counts go with
// the side squared), and left as it is for volume-like clouds.  The caller
// counts again with the new grid.  (Measured on the scan clouds: queries in
// their clusters dominate the search time at 2 points per cell.)
__device__ inline void grid_refine_body(const int* __restrict__ counts, int n, int max_cells,
                                        GridInfo* __restrict__ gi) {
  __shared__ int red[16];
  const GridInfo G0 = *gi;
  int occ = 0;
  for (int c = threadIdx.x; c < G0.ncells; c += 1024) occ += counts[c] > 0;
  for (int off = 32; off > 0; off >>= 1) occ += __shfl_xor(occ, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = occ;
  __syncthreads();
  if (threadIdx.x != 0) return;
  occ = 0;
  for (int w = 0; w < 16; ++w) occ += red[w];
  const double mu = (double)n / (double)max(occ, 1);
  if (!(mu > 6.0)) return;
  GridInfo G = G0;
  grid_dims(G, (double)G0.h * sqrt(6.0 / mu), max_cells);
  *gi = G;
}

__global__ __launch_bounds__(1024) void grid_refine_kernel(const int* __restrict__ counts, int n, int max_cells,
                                                           GridInfo* __restrict__ gi) {
  grid_refine_body(counts, n, max_cells, gi);
}

// Cell coordinates and cell faces are computed in FP64 so that rounding
// cannot move a point across a face by more than a negligible fraction of a
// cell, whatever the offset of the cloud from the origin.
__device__ inline int cell_coord(float p, float lo, float h, int dim) {
  const double u = floor(((double)p - (double)lo) / (double)h);
  const int c = u < 0.0 ? 0 : (u >= (double)dim ? dim - 1 : (int)u);
  return c;
}

__device__ inline void grid_count_point(const float* __restrict__ X, const float* __restrict__ Y,
                                        const float* __restrict__ Zc, int n, const GridInfo* __restrict__ gi,
                                        int* __restrict__ cell_of, int* __restrict__ counts, int i) {
  if (i >= n) return;
  const GridInfo& G = *gi;
  const int cx = cell_coord(X[i], G.lo[0], G.h, G.dims[0]);
  const int cy = cell_coord(Y[i], G.lo[1], G.h, G.dims[1]);
  const int cz = cell_coord(Zc[i], G.lo[2], G.h, G.dims[2]);
  const int c = (cz * G.dims[1] + cy) * G.dims[0] + cx;
  cell_of[i] = c;
  atomicAdd(&counts[c], 1);
}

__global__ __launch_bounds__(256) void grid_count_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                         const float* __restrict__ Zc, int n,
                                                         const GridInfo* __restrict__ gi, int* __restrict__ cell_of,
                                                         int* __restrict__ counts) {
  grid_count_point(X, Y, Zc, n, gi, cell_of, counts, blockIdx.x * 256 + threadIdx.x);
}

// Exclusive scan of counts[0, m) into starts[0, m], in three passes.
__global__ __launch_bounds__(SCAN_B) void scan_local_kernel(const int* __restrict__ in, int m, int* __restrict__ out,
                                                            int* __restrict__ bsum) {
  __shared__ int s[SCAN_B];
  const int i = blockIdx.x * SCAN_B + threadIdx.x;
  const int v = i < m ? in[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_B; off <<= 1) {
    const int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < m) out[i] = s[threadIdx.x] - v;
  if (threadIdx.x == SCAN_B - 1) bsum[blockIdx.x] = s[threadIdx.x];
}

__global__ __launch_bounds__(1024) void scan_blocks_kernel(int* __restrict__ bsum, int nb) {
  // serial over block sums in one thread per 1024-chunk, nb is small
  if (threadIdx.x != 0) return;
  int acc = 0;
  for (int b = 0; b < nb; ++b) {
    const int v = bsum[b];
    bsum[b] = acc;
    acc += v;
  }
  bsum[nb] = acc;
}

__global__ __launch_bounds__(SCAN_B) void scan_add_kernel(int* __restrict__ out, int m, const int* __restrict__ bsum,
                                                          int nb) {
  const int i = blockIdx.x * SCAN_B + threadIdx.x;
  if (i < m) out[i] += bsum[blockIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) out[m] = bsum[nb];
}

// Also packs the point, in its own order, as p4[i] = (x, y, z, 0): one
// 16-byte load per neighbour for the curvature instead of three.
__device__ inline void grid_scatter_point(const float* __restrict__ X, const float* __restrict__ Y,
                                          const float* __restrict__ Zc, int n, const int* __restrict__ cell_of,
                                          const int* __restrict__ starts, int* __restrict__ cursor,
                                          float4* __restrict__ spts, float4* __restrict__ p4, int i) {
  if (i >= n) return;
  const int c = cell_of[i];
  const int pos = starts[c] + atomicAdd(&cursor[c], 1);
  const float x = X[i], y = Y[i], z = Zc[i];
  spts[pos] = make_float4(x, y, z, __int_as_float(i));
  p4[i] = make_float4(x, y, z, 0.f);
}

__global__ __launch_bounds__(256) void grid_scatter_kernel(const float* __restrict__ X, const float* __restrict__ Y,
                                                           const float* __restrict__ Zc, int n,
                                                           const int* __restrict__ cell_of,
                                                           const int* __restrict__ starts, int* __restrict__ cursor,
                                                           float4* __restrict__ spts, float4* __restrict__ p4) {
  grid_scatter_point(X, Y, Zc, n, cell_of, starts, cursor, spts, p4, blockIdx.x * 256 + threadIdx.x);
}

__device__ inline bool key_less(float d, int i, float bd, int bi) { return d < bd || (d == bd && i < bi); }

// Visits spts[p0 .. p1) in order.  A lane searching far from its cell meets
// thousands of candidates, and with few waves per SIMD one dependent load
// per candidate would leave it waiting on memory for most of the kernel: the
// lane therefore issues SPAN_U independent loads, parks the points in its own
// LDS column (buf[u * GQ_BT], no other lane touches it, no barrier) and then
// processes them in a rolled loop, which keeps the per-candidate code (the
// top-k insertion) in one copy.  Six loads: with the 8-key candidate column
// a 256-thread block then needs 40 KB of LDS, so four blocks (four waves
// per SIMD, which the registers also allow) fit on a CU; with eight loads
// only three fit, and the batched search took 16 % longer (measured on the
// 512 clouds of the batch workload; four loads: 3 % longer).
constexpr int SPAN_U = 6;

template <class F>
__device__ inline void span_points(const float4* __restrict__ spts, int p0, int p1, float4* buf, F&& f) {
  for (int p = p0; p < p1; p += SPAN_U) {
#pragma unroll
    for (int u = 0; u < SPAN_U; ++u) buf[u * GQ_BT] = spts[min(p + u, p1 - 1)];
    const int nu = min(SPAN_U, p1 - p);
#pragma unroll 1
    for (int u = 0; u < nu; ++u) f(buf[u * GQ_BT]);
  }
}

// The points of row (dz, dy) of shell r around cell c (the cells with
// max(|dx|, |dy|, |dz|) = r in that row) as contiguous spans of the
// cell-sorted point array.  The cells of one (z, y) row are adjacent in that
// array, so a row on the shell's boundary is one span (two index loads,
// however many cells) and a row inside the shell contributes its two end
// cells.  Up to two spans are handed to a single call site (one inlined copy
// of the caller's per-candidate code), in the order in which visiting the
// cells one by one would meet the points.
__device__ inline void row_bounds(const int* __restrict__ starts, const GridInfo& G, const int c[3], int r, int dz,
                                  int dy, int& a0, int& a1, int& b0, int& b1) {
  a0 = a1 = b0 = b1 = 0;
  const int cz = c[2] + dz, cy = c[1] + dy;
  if (cz < 0 || cz >= G.dims[2] || cy < 0 || cy >= G.dims[1]) return;
  const int row = (cz * G.dims[1] + cy) * G.dims[0];
  const bool full = r == 0 || abs(dz) == r || abs(dy) == r;
  // first span: cells [c - r, c + r] of a boundary row (clipped to the
  // grid), or the cell c - r of an interior row; second span: the cell
  // c + r of an interior row.  (Each bound is loaded under one condition:
  // assignments of loaded values to a0..b1 on several paths made the
  // compiler keep them in scratch memory.)
  const int xa0 = max(0, c[0] - r);
  const int xa1 = full ? min(G.dims[0] - 1, c[0] + r) : c[0] - r;
  if (xa1 >= xa0) {
    a0 = starts[row + xa0];
    a1 = starts[row + xa1 + 1];
  }
  const int xb = c[0] + r;
  if (!full && xb < G.dims[0]) {
    b0 = starts[row + xb];
    b1 = starts[row + xb + 1];
  }
}

template <class F>
__device__ inline void row_spans(const int* __restrict__ starts, const GridInfo& G, const int c[3], int r, int dz,
                                 int dy, F&& f) {
  int a0, a1, b0, b1;
  row_bounds(starts, G, c, r, dz, dy, a0, a1, b0, b1);
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    const int q0 = h ? b0 : a0, q1 = h ? b1 : a1;
    if (q0 < q1) f(q0, q1);
  }
}

// Every point of shell r, row by row; far queries (outliers in empty space)
// touch about 3x fewer index words than cell by cell.
template <class F>
__device__ inline void shell_spans(const int* __restrict__ starts, const GridInfo& G, const int c[3], int r, F&& f) {
  for (int dz = -r; dz <= r; ++dz)
    for (int dy = -r; dy <= r; ++dy) row_spans(starts, G, c, r, dz, dy, f);
}

// After shell r has been searched: true when nothing outside the searched
// cube can beat the current k-th key (or no cell lies outside it).  Margin:
// 1e-3 of a cell for the face, 1e-5 relative for the float32 key; an
// incomplete list (key NaN) never stops the search.
__device__ inline bool shell_done(const GridInfo& G, const int c[3], const float qv[3], int r, float kth) {
  double lb = INFINITY;
  bool all = true;
  for (int a = 0; a < 3; ++a) {
    if (c[a] - r > 0) {
      lb = fmin(lb, (double)qv[a] - ((double)G.lo[a] + (double)(c[a] - r) * (double)G.h));
      all = false;
    }
    if (c[a] + r < G.dims[a] - 1) {
      lb = fmin(lb, ((double)G.lo[a] + (double)(c[a] + r + 1) * (double)G.h) - (double)qv[a]);
      all = false;
    }
  }
  if (all) return true;
  const double lbs = lb - 1e-3 * (double)G.h;
  return lbs > 0.0 && (double)kth * 1.00001 < lbs * lbs;
}

__device__ inline float key_of(uint64_t w) { return __uint_as_float((uint32_t)(w >> 32)); }

// Sorted insertion of a 64-bit (float32 key bits << 32 | index) word into
// L[0..KC): one compare and two selects per slot.
template <int KC>
__device__ inline void insert_key(uint64_t (&L)[KC], uint64_t key) {
  uint64_t ck = key;
#pragma unroll
  for (int s = 0; s < KC; ++s) {
    const uint64_t t = L[s];
    const bool sw = ck < t;
    L[s] = sw ? ck : t;
    ck = sw ? t : ck;
  }
}

// Compare-exchange of two keys into ascending order.
__device__ inline void cmp_swap(uint64_t& a, uint64_t& b) {
  const bool sw = b < a;
  const uint64_t lo = sw ? b : a, hi = sw ? a : b;
  a = lo;
  b = hi;
}

// f(integral_constant<int, I>) for I = 0 .. N-1, expanded at compile time (the
// networks below index register arrays, which must never be indexed at run
// time).
template <class F, int... I>
__device__ inline void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ inline void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// Sorts a bitonic sequence (ascending, then descending) into ascending order
// (Batcher's bitonic merger: half-cleaners of width N/2, N/4, ..., 1).
template <int N, int J = N / 2>
__device__ inline void bitonic_merge(uint64_t (&v)[N]) {
  if constexpr (J > 0) {
    static_for<N>([&](auto i) {
      if constexpr ((i & J) == 0) cmp_swap(v[i], v[i | J]);
    });
    bitonic_merge<N, J / 2>(v);
  }
}

// Sorts 8 keys ascending (bitonic sort: merges of width 2, 4, 8 with
// alternating directions).
template <int W = 2, int J = 1>
__device__ inline void bitonic_sort8(uint64_t (&v)[8]) {
  if constexpr (W <= 8) {
    static_for<8>([&](auto i) {
      if constexpr ((i & J) == 0) {
        if constexpr ((i & W) == 0)
          cmp_swap(v[i], v[i | J]);
        else
          cmp_swap(v[i | J], v[i]);
      }
    });
    if constexpr (J > 1)
      bitonic_sort8<W, J / 2>(v);
    else
      bitonic_sort8<W * 2, W>(v);
  }
}

// Merges up to 8 keys cand[0 .. cnt) (the lane's LDS column) into the sorted
// list L, keeping its KC smallest.  A flush runs in every lane of the wave
// at once, and with one sorted insertion per key it would cost the largest
// cnt of the wave times 7 KC operations; the keys instead go through one
// network: the buffer, padded with all-ones keys, is sorted; with L and the
// buffer both ascending and padded to a power of two P >= KC, the
// element-wise minimum of L and the reversed buffer is a bitonic sequence
// that holds the P smallest keys of the two, and a bitonic merger sorts it.
// Keys are (key bits, index) words, so the result is the same list as that
// of the insertions.
template <int KC>
__device__ inline void flush_keys(uint64_t (&L)[KC], const uint64_t* cand, int cnt) {
  uint64_t B[8];
  static_for<8>([&](auto u) { B[u] = u < cnt ? cand[u * GQ_BT] : ~0ull; });
  bitonic_sort8(B);
  if constexpr ((KC & (KC - 1)) == 0) {
    // P = KC: only the last 8 slots meet a buffered key; merged in place
    static_for<8>([&](auto u) {
      const uint64_t b = B[u];
      L[KC - 1 - u] = b < L[KC - 1 - u] ? b : L[KC - 1 - u];
    });
    bitonic_merge<KC>(L);
  } else {
    // KC = 24, P = 32: L's padding is all ones, so the sequence is L
    // followed by the reversed buffer
    static_assert(KC == 24, "list sizes are 8, 16, 24 or 32");
    uint64_t D[32];
    static_for<24>([&](auto i) { D[i] = L[i]; });
    static_for<8>([&](auto u) { D[24 + u] = B[7 - u]; });
    bitonic_merge<32>(D);
    static_for<24>([&](auto i) { L[i] = D[i]; });
  }
}

// Order in which a lane visits the rows (dz, dy) of shell r: the rows
// nearest the query's cell first (by |dz| + |dy|, then max(|dz|, |dy|)), so
// that the k-th key falls early and fewer later candidates are buffered.  Any
// order visits the same points before the stopping test.
__device__ inline void shell_row(int r, int ri, int& dz, int& dy) {
  if (r == 1) {
    // (0,0) (0,-1) (0,1) (-1,0) (1,0) (-1,-1) (-1,1) (1,-1) (1,1), as
    // 2-bit fields of dz + 1 and dy + 1 (no table in memory)
    dz = ((0x28215 >> (2 * ri)) & 3) - 1;
    dy = ((0x22161 >> (2 * ri)) & 3) - 1;
    return;
  }
  const int w = 2 * r + 1;
  dz = ri / w - r;
  dy = ri % w - r;
}

// Writes the k neighbour indices of every point (row = original index,
// sorted by key; -1 where fewer than k finite points exist).  With a far
// list, a query whose search is not finished after shell rcap (an outlier in
// empty space, whose lane would otherwise sweep many cells alone and hold up
// its wave) is appended to it instead, for grid_knn_far_kernel.
// Candidates a lane buffers before they are inserted.  A candidate is
// buffered when its key is below the k-th key of the list as it stood at the
// last insertion; that key only decreases, so a rejected candidate could never
// have entered.  Each lane's buffer is its own LDS column.  The active lanes
// of a wave insert their buffers together as soon as one of them is full (and
// at the end of every shell, before the stopping test): in a dense cluster
// some lane accepts a candidate at almost every step, and inserting at once
// would make the wave run the 5 KC-operation insertion at almost every step.
constexpr int KNN_CB = 8;
static_assert(KNN_CB == 8, "flush_keys sorts a buffer of 8 keys");

// Query t (a position in the cell-sorted array); buf and cand are the lane's
// LDS columns (stride GQ_BT).  No barriers.  The search starts at shell r0:
// with r0 > 0 it resumes a query handed over after shell r0 - 1, whose list
// of the k best of shells 0 .. r0 - 1 is in its output row (see below).
template <int KC>
__device__ inline void grid_knn_query(const float4* __restrict__ spts, const float4* __restrict__ p4,
                                      const int* __restrict__ starts, const GridInfo* __restrict__ gi, int n, int k,
                                      int rcap, int* __restrict__ far, int32_t* __restrict__ idx_out, int t,
                                      float4* buf, uint64_t* cand, int r0) {
  if (t >= n) return;
  const GridInfo G = *gi;
  const float4 q = spts[t];
  const int qi = __float_as_int(q.w);
  // a query with a non-finite coordinate has no finite key to any point:
  // its list is empty (and searching for one would visit every shell)
  if (!(isfinite(q.x) && isfinite(q.y) && isfinite(q.z))) {
    for (int s = 0; s < k; ++s) idx_out[(int64_t)qi * k + s] = -1;
    return;
  }
  const float qv[3] = {q.x, q.y, q.z};
  int c[3];
  for (int a = 0; a < 3; ++a) c[a] = cell_coord(qv[a], G.lo[a], G.h, G.dims[a]);
  // The running top k as sorted 64-bit keys (float32 key bits << 32 |
  // index): for keys >= 0 the bit pattern orders like the value, so one
  // unsigned compare gives the (key, index) order.  Slots [0, KC - k) hold
  // the sentinel 0, which no candidate undercuts, so slot KC - 1 is always
  // the k-th best; empty slots hold all ones (key NaN, index -1).
  // Candidates whose key is not below +inf (non-finite points, overflowing
  // distances) never enter.
  uint64_t L[KC];
#pragma unroll
  for (int s = 0; s < KC; ++s) L[s] = (s < KC - k) ? 0ull : ~0ull;
  if (r0 > 0) {
    // the row's indices in key order (-1: empty); their keys are rebuilt
    // from the packed points with the same float32 arithmetic
    const int64_t o = (int64_t)qi * k;
#pragma unroll
    for (int s = 0; s < KC; ++s) {
      if (s >= KC - k) {
        const int id = idx_out[o + (s - (KC - k))];
        if (id >= 0) {
          const float4 P = p4[id];
          const float ex = __fsub_rn(P.x, q.x), ey = __fsub_rn(P.y, q.y), ez = __fsub_rn(P.z, q.z);
          const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(ex, ex), __fmul_rn(ey, ey)), __fmul_rn(ez, ez));
          L[s] = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)id;
        }
      }
    }
  }
  int cnt = 0;  // buffered candidates of this lane
  const int rmax = max(G.dims[0], max(G.dims[1], G.dims[2]));
  for (int r = r0; r <= rmax; ++r) {
    // the rows of shell r (see row_spans), then one end row that visits no
    // point and empties the buffers through the same insertion code, so that
    // this code exists once
    const int w = 2 * r + 1, nrow = w * w;
#pragma unroll 1
    for (int ri = 0; ri <= nrow; ++ri) {
      const bool end = ri == nrow;
      int a0 = 0, a1 = 1, b0 = 0, b1 = 0;
      if (!end) {
        int dz, dy;
        shell_row(r, ri, dz, dy);
        row_bounds(starts, G, c, r, dz, dy, a0, a1, b0, b1);
      }
#pragma unroll 1
      for (int h = 0; h < 2; ++h) {
        const int q0 = h ? b0 : a0, q1 = h ? b1 : a1;
#pragma unroll 1
        for (int p = q0; p < q1; p += SPAN_U) {
          if (!end) {
#pragma unroll
            for (int u = 0; u < SPAN_U; ++u) buf[u * GQ_BT] = spts[min(p + u, q1 - 1)];
          }
          const int nu = min(SPAN_U, q1 - p);
#pragma unroll 1
          for (int u = 0; u < nu; ++u) {
            if (!end) {
              const float4 P = buf[u * GQ_BT];
              const float ex = __fsub_rn(P.x, q.x), ey = __fsub_rn(P.y, q.y), ez = __fsub_rn(P.z, q.z);
              const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(ex, ex), __fmul_rn(ey, ey)), __fmul_rn(ez, ez));
              const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)__float_as_int(P.w);
              if (d2 < INFINITY && key < L[KC - 1]) {
                cand[cnt * GQ_BT] = key;
                ++cnt;
              }
            }
            if (__any(cnt == KNN_CB || (end && cnt > 0))) {
              flush_keys<KC>(L, cand, cnt);
              cnt = 0;
            }
          }
        }
      }
    }
    if (shell_done(G, c, qv, r, key_of(L[KC - 1]))) break;
    // handed to the far pass, which continues from shell rcap + 1 with the
    // list written below (the k best of the shells searched here)
    if (far && r >= rcap) {
      far[1 + atomicAdd(far, 1)] = t;
      break;
    }
  }
  // static slot indices only (a runtime index would put L in scratch memory)
  const int64_t o = (int64_t)qi * k;
#pragma unroll
  for (int s = 0; s < KC; ++s)
    if (s >= KC - k) idx_out[o + (s - (KC - k))] = (int32_t)(uint32_t)L[s];
}

template <int KC>
__global__ __launch_bounds__(GQ_BT) void grid_knn_kernel(const float4* __restrict__ spts, const int* __restrict__ starts,
                                                         const GridInfo* __restrict__ gi, int n, int k, int rcap,
                                                         int* __restrict__ far, int32_t* __restrict__ idx_out) {
  __shared__ float4 s_buf[SPAN_U * GQ_BT];
  __shared__ uint64_t s_cand[KNN_CB * GQ_BT];
  grid_knn_query<KC>(spts, nullptr, starts, gi, n, k, rcap, far, idx_out, blockIdx.x * GQ_BT + threadIdx.x,
                     s_buf + threadIdx.x, s_cand + threadIdx.x, 0);
}

// The queries grid_knn_kernel left unfinished, one wave per query (a
// wave-uniform loop over the far list).  Lane l scans rows l, l + 64, ... of
// each shell into its own sorted list of the KC best keys it has met (every
// slot real, no sentinels); after the shell the wave merges the 64 lists into
// the KC best of their union by KC rounds of a wave-wide minimum (keys are
// unique, so exactly the lanes holding the minimum pop it, and duplicates of
// a merged entry are popped together), and every lane continues from the
// merged list (a shell in which no lane took a key leaves every list equal
// to the merged one, and skips the merge).  The stopping test is
// grid_knn_kernel's on the merged k-th key, so the neighbour list is the
// same exact one.  This is far query t (a position in the cell-sorted
// array) of the grid G, searched by the calling wave.
template <int KC>
__device__ inline void grid_knn_far_query(const float4* __restrict__ spts, const float4* __restrict__ p4,
                                          const int* __restrict__ starts, const GridInfo& G, int k, int t,
                                          int32_t* __restrict__ idx_out, float4* buf, int r0) {
  const int lane = threadIdx.x & 63;
  const int rmax = max(G.dims[0], max(G.dims[1], G.dims[2]));
  const float4 q = spts[t];
  const int qi = __float_as_int(q.w);
  const float qv[3] = {q.x, q.y, q.z};
  int c[3];
  for (int a = 0; a < 3; ++a) c[a] = cell_coord(qv[a], G.lo[a], G.h, G.dims[a]);
  // The lane passes searched shells 0 .. r0 - 1 and left the k best of
  // them in the query's output row (index -1 for an empty slot): lane s < k
  // rebuilds entry s's key from the packed points (the same float32
  // arithmetic as the key was made with), and every lane starts from that
  // list, as after a merge.  Slots k .. KC-1 start empty; they never hold
  // one of the k best.
  uint64_t L[KC];
  {
    uint64_t mine = ~0ull;
    if (lane < k) {
      const int id = idx_out[(int64_t)qi * k + lane];
      if (id >= 0) {
        const float4 P = p4[id];
        const float ex = __fsub_rn(P.x, q.x), ey = __fsub_rn(P.y, q.y), ez = __fsub_rn(P.z, q.z);
        const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(ex, ex), __fmul_rn(ey, ey)), __fmul_rn(ez, ez));
        mine = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)id;
      }
    }
#pragma unroll
    for (int s = 0; s < KC; ++s) L[s] = s < k ? __shfl(mine, s, 64) : ~0ull;
  }
  float kth = key_of(~0ull);  // the k-th key of the merged list (NaN: fewer than k yet)
#pragma unroll
  for (int s = 0; s < KC; ++s)
    if (s == k - 1) kth = key_of(L[s]);
  for (int r = r0; r <= rmax; ++r) {
    const int side = 2 * r + 1;
    bool took = false;
    for (int row = lane; row < side * side; row += 64) {
      row_spans(starts, G, c, r, row / side - r, row % side - r, [&](int p0, int p1) {
        span_points(spts, p0, p1, buf, [&](const float4& P) {
          const float ex = __fsub_rn(P.x, q.x), ey = __fsub_rn(P.y, q.y), ez = __fsub_rn(P.z, q.z);
          const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(ex, ex), __fmul_rn(ey, ey)), __fmul_rn(ez, ez));
          const uint64_t key = ((uint64_t)__float_as_uint(d2) << 32) | (uint32_t)__float_as_int(P.w);
          if (d2 < INFINITY && key < L[KC - 1]) {
            insert_key(L, key);
            took = true;
          }
        });
      });
    }
    // no lane took a key in this shell: every lane's list is still the
    // merged list of the last shell, which the merge would return again
    if (__ballot(took) == 0) {
      if (shell_done(G, c, qv, r, kth)) break;
      continue;
    }
    // merge the 64 lists: M collects the successive wave minima in order
    uint64_t M[KC];
#pragma unroll
    for (int s = 0; s < KC; ++s) M[s] = ~0ull;
#pragma unroll 1
    for (int round = 0; round < KC; ++round) {
      const uint64_t h = L[0];
      uint64_t m = h;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t o = __shfl_xor(m, off, 64);
        m = o < m ? o : m;
      }
      const bool pop = h == m;
#pragma unroll
      for (int s = 0; s < KC - 1; ++s) L[s] = pop ? L[s + 1] : L[s];
      L[KC - 1] = pop ? ~0ull : L[KC - 1];
#pragma unroll
      for (int s = 0; s < KC - 1; ++s) M[s] = M[s + 1];
      M[KC - 1] = m;
    }
#pragma unroll
    for (int s = 0; s < KC; ++s) {
      L[s] = M[s];
      if (s == k - 1) kth = key_of(M[s]);
    }
    if (shell_done(G, c, qv, r, kth)) break;
  }
  if (lane == 0) {
    const int64_t o = (int64_t)qi * k;
#pragma unroll
    for (int s = 0; s < KC; ++s)
      if (s < k) idx_out[o + s] = (int32_t)(uint32_t)L[s];
  }
}

// Wave `wave` of n_waves takes the far queries wave, wave + n_waves, ...
template <int KC>
__device__ inline void grid_knn_far_waves(const float4* __restrict__ spts, const float4* __restrict__ p4,
                                          const int* __restrict__ starts,
                                          const GridInfo* __restrict__ gi, int k, const int* __restrict__ far,
                                          int32_t* __restrict__ idx_out, int wave, int n_waves, float4* buf) {
  const int cnt = far[0];
  const GridInfo G = *gi;
  for (int f = wave; f < cnt; f += n_waves)
    grid_knn_far_query<KC>(spts, p4, starts, G, k, far[1 + f], idx_out, buf, KNN_RCAP + 1);
}

template <int KC>
__global__ __launch_bounds__(GQ_BT) void grid_knn_far_kernel(const float4* __restrict__ spts,
                                                             const float4* __restrict__ p4,
                                                             const int* __restrict__ starts,
                                                             const GridInfo* __restrict__ gi, int k,
                                                             const int* __restrict__ far,
                                                             int32_t* __restrict__ idx_out) {
  __shared__ float4 s_buf[SPAN_U * GQ_BT];
  grid_knn_far_waves<KC>(spts, p4, starts, gi, k, far, idx_out, (blockIdx.x * GQ_BT + threadIdx.x) >> 6,
                         (gridDim.x * GQ_BT) >> 6, s_buf + threadIdx.x);
}

// Curvature from the neighbour lists (FP64 covariance, 1/k, centred), one
// block of CURV_BT points.  A point's list is k consecutive indices, so with
// one point per thread every load instruction of a wave would touch 64
// different rows; the block's rows (contiguous in memory) are therefore
// copied into LDS with coalesced loads first, at an odd row stride so that
// the threads' reads of their own rows meet no bank conflict.  The
// neighbours' packed coordinates (p4) are then read in groups of CURV_G, each
// group's loads all requested before the first is used, in one pass: the
// sums are taken of the offsets from the list's first point (the query
// itself unless duplicates come first), C = S2 / k - (S1 / k)(S1 / k)^T,
// which is the centred covariance for any shift and, with a shift inside the
// neighbourhood, keeps the FP64 cancellation at the rounding of the offsets.
constexpr int CURV_BT = 256;
constexpr int CURV_G = 8;

__device__ inline int curv_stride(int k) { return k | 1; }

// Points [b CURV_BT, min(n, (b + 1) CURV_BT)); lds holds CURV_BT rows of
// curv_stride(k) ints.  Every thread reaches the barrier.
__device__ inline void curvature_block(const float4* __restrict__ p4, int n, int k, const int32_t* __restrict__ idx,
                                       float* __restrict__ a_out, int b, int* lds) {
  const int p0 = b * CURV_BT;
  const int cnt = min(CURV_BT, n - p0);
  const int st = curv_stride(k);
  {
    // element e = threadIdx.x + CURV_BT i of the block's cnt k indices is
    // column c of row r; (r, c) advance by (CURV_BT / k, CURV_BT % k)
    const int32_t* src = idx + (int64_t)p0 * k;
    const int dr = CURV_BT / k, dc = CURV_BT % k;
    int r = threadIdx.x / k, c = threadIdx.x % k;
#pragma unroll 4
    for (int e = threadIdx.x; e < cnt * k; e += CURV_BT) {
      lds[r * st + c] = src[e];
      r += dr;
      c += dc;
      if (c >= k) {
        c -= k;
        ++r;
      }
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= cnt) return;
  const int q = p0 + t;
  const int* nb = lds + t * st;
  bool missing = false;
  double sh[3] = {0, 0, 0}, S1[3] = {0, 0, 0}, S2[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll 1
  for (int s0 = 0; s0 < k; s0 += CURV_G) {
    int id[CURV_G];
#pragma unroll
    for (int u = 0; u < CURV_G; ++u) id[u] = s0 + u < k ? nb[s0 + u] : 0;
    float4 P[CURV_G];
#pragma unroll
    for (int u = 0; u < CURV_G; ++u) P[u] = p4[max(id[u], 0)];
    if (s0 == 0) {
      sh[0] = (double)P[0].x;
      sh[1] = (double)P[0].y;
      sh[2] = (double)P[0].z;
    }
#pragma unroll
    for (int u = 0; u < CURV_G; ++u) {
      if (s0 + u < k) {
        missing |= id[u] < 0;
        const double dx = (double)P[u].x - sh[0], dy = (double)P[u].y - sh[1], dz = (double)P[u].z - sh[2];
        S1[0] += dx;
        S1[1] += dy;
        S1[2] += dz;
        S2[0] += dx * dx;
        S2[1] += dy * dy;
        S2[2] += dz * dz;
        S2[3] += dx * dy;
        S2[4] += dx * dz;
        S2[5] += dy * dz;
      }
    }
  }
  if (missing) {
    a_out[q] = NAN;
    return;
  }
  const double invk = 1.0 / (double)k;
  const double mx = S1[0] * invk, my = S1[1] * invk, mz = S1[2] * invk;
  const double C[6] = {S2[0] * invk - mx * mx, S2[1] * invk - my * my, S2[2] * invk - mz * mz,
                       S2[3] * invk - mx * my, S2[4] * invk - mx * mz, S2[5] * invk - my * mz};
  double lam[3];
  eig_psd3(C, lam);
  const double tr = C[0] + C[1] + C[2];
  a_out[q] = (tr > 0.0) ? (float)(lam[2] / tr) : 0.f;
}

// Dynamic LDS of the curvature kernels: CURV_BT rows of curv_stride(k) ints.
inline size_t curv_lds_bytes(int k) { return sizeof(int) * (size_t)CURV_BT * (size_t)(k | 1); }

__global__ __launch_bounds__(CURV_BT) void curvature_kernel(const float4* __restrict__ p4, int n, int k,
                                                            const int32_t* __restrict__ idx,
                                                            float* __restrict__ a_out) {
  extern __shared__ int s_nb[];
  curvature_block(p4, n, k, idx, a_out, blockIdx.x, s_nb);
}

int grid_max_cells(int n) {
  int m = 1024;
  while (m < 2 * n && m < (1 << 24)) m <<= 1;
  return m;
}

size_t grid_knn_workspace(int n, int k) {
  const int max_cells = grid_max_cells(n);
  const int nb = (max_cells + SCAN_B - 1) / SCAN_B;
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  add(sizeof(GridInfo));
  add(sizeof(int) * (size_t)n);            // cell_of
  add(sizeof(int) * (size_t)max_cells);    // counts
  add(sizeof(int) * (size_t)max_cells);    // cursor
  add(sizeof(int) * ((size_t)max_cells + 1));  // starts
  add(sizeof(int) * ((size_t)nb + 1));     // block sums
  add(sizeof(float4) * (size_t)n);         // sorted points
  add(sizeof(float4) * (size_t)n);         // packed points
  add(sizeof(int32_t) * (size_t)n * k);    // neighbour lists
  add(sizeof(int) * ((size_t)n + 1));      // far-query list
  add(sizeof(int) * ((size_t)n + 1));      // second far-query list (batches)
  return b;
}

namespace {

struct GridBufs {
  GridInfo* gi;
  int* cell_of;
  int* counts;
  int* cursor;
  int* starts;
  int* bsum;
  float4* spts;
  float4* p4;  // the points in their own order, (x, y, z, 0)
  int32_t* nbr;
  int* far;  // [0]: count, [1..n]: sorted positions of the queries left to the far pass
  int* far2;  // the same for the batch's second hand-over
};

GridBufs carve_grid(void* ws, int n, int k) {
  const int max_cells = grid_max_cells(n);
  const int nb = (max_cells + SCAN_B - 1) / SCAN_B;
  char* p = (char*)ws;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~size_t(255);
    return (void*)r;
  };
  GridBufs B;
  B.gi = (GridInfo*)take(sizeof(GridInfo));
  B.cell_of = (int*)take(sizeof(int) * (size_t)n);
  B.counts = (int*)take(sizeof(int) * (size_t)max_cells);
  B.cursor = (int*)take(sizeof(int) * (size_t)max_cells);
  B.starts = (int*)take(sizeof(int) * ((size_t)max_cells + 1));
  B.bsum = (int*)take(sizeof(int) * ((size_t)nb + 1));
  B.spts = (float4*)take(sizeof(float4) * (size_t)n);
  B.p4 = (float4*)take(sizeof(float4) * (size_t)n);
  B.nbr = (int32_t*)take(sizeof(int32_t) * (size_t)n * k);
  B.far = (int*)take(sizeof(int) * ((size_t)n + 1));
  B.far2 = (int*)take(sizeof(int) * ((size_t)n + 1));
  return B;
}

// Uniform grid of the points, counting-sorted by cell.
hipError_t build_grid(const float* x, const float* y, const float* z, int n, const GridBufs& B, hipStream_t st) {
  const int max_cells = grid_max_cells(n);
  const int nb = (max_cells + SCAN_B - 1) / SCAN_B;
  const dim3 gn((n + 255) / 256), b256(256);
  hipLaunchKernelGGL(grid_setup_kernel, dim3(1), dim3(1024), 0, st, x, y, z, n, max_cells, B.gi, B.far);
  if (hipError_t e = launch_fill_i(B.counts, max_cells, st)) return e;
  hipLaunchKernelGGL(grid_count_kernel, gn, b256, 0, st, x, y, z, n, B.gi, B.cell_of, B.counts);
  hipLaunchKernelGGL(grid_refine_kernel, dim3(1), dim3(1024), 0, st, B.counts, n, max_cells, B.gi);
  if (hipError_t e = launch_fill_i(B.counts, max_cells, st)) return e;
  if (hipError_t e = launch_fill_i(B.cursor, max_cells, st)) return e;
  hipLaunchKernelGGL(grid_count_kernel, gn, b256, 0, st, x, y, z, n, B.gi, B.cell_of, B.counts);
  hipLaunchKernelGGL(scan_local_kernel, dim3(nb), dim3(SCAN_B), 0, st, B.counts, max_cells, B.starts, B.bsum);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(64), 0, st, B.bsum, nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(SCAN_B), 0, st, B.starts, max_cells, B.bsum, nb);
  hipLaunchKernelGGL(grid_scatter_kernel, gn, b256, 0, st, x, y, z, n, B.cell_of, B.starts, B.cursor, B.spts,
                     B.p4);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_knn(const float* x, const float* y, const float* z, int n, int k, float* a_out,
                           int32_t* idx_out, void* ws, hipStream_t st) {
  const GridBufs B = carve_grid(ws, n, k);
  if (hipError_t e = build_grid(x, y, z, n, B, st)) return e;
  int32_t* lists = idx_out ? idx_out : B.nbr;
  const dim3 gn((n + 255) / 256), b256(256);
  const dim3 gq((n + GQ_BT - 1) / GQ_BT), bq(GQ_BT);
  // pass 1: one lane per query up to shell KNN_RCAP; pass 2: one wave per
  // query left over (a fixed grid of waves loops over the device-side list)
  const dim3 gf(512);
  if (k <= 8) {
    hipLaunchKernelGGL(grid_knn_kernel<8>, gq, bq, 0, st, B.spts, B.starts, B.gi, n, k, KNN_RCAP, B.far, lists);
    hipLaunchKernelGGL(grid_knn_far_kernel<8>, gf, bq, 0, st, B.spts, B.p4, B.starts, B.gi, k, B.far, lists);
  } else if (k <= 16) {
    hipLaunchKernelGGL(grid_knn_kernel<16>, gq, bq, 0, st, B.spts, B.starts, B.gi, n, k, KNN_RCAP, B.far, lists);
    hipLaunchKernelGGL(grid_knn_far_kernel<16>, gf, bq, 0, st, B.spts, B.p4, B.starts, B.gi, k, B.far, lists);
  } else if (k <= 24) {
    hipLaunchKernelGGL(grid_knn_kernel<24>, gq, bq, 0, st, B.spts, B.starts, B.gi, n, k, KNN_RCAP, B.far, lists);
    hipLaunchKernelGGL(grid_knn_far_kernel<24>, gf, bq, 0, st, B.spts, B.p4, B.starts, B.gi, k, B.far, lists);
  } else {
    hipLaunchKernelGGL(grid_knn_kernel<32>, gq, bq, 0, st, B.spts, B.starts, B.gi, n, k, KNN_RCAP, B.far, lists);
    hipLaunchKernelGGL(grid_knn_far_kernel<32>, gf, bq, 0, st, B.spts, B.p4, B.starts, B.gi, k, B.far, lists);
  }
  if (a_out)
    hipLaunchKernelGGL(curvature_kernel, gn, dim3(CURV_BT), curv_lds_bytes(k), st, B.p4, n, k, lists, a_out);
  return hipGetLastError();
}

// Nearest point of the grid's cloud to each query (any points, inside or
// outside the grid's box) among the points whose key is <= max_key: the
// same shell search and (key, index) order as grid_knn_kernel with k = 1,
// stopped once the unsearched cells lie beyond max_key.  A query with no
// such point, or with a non-finite coordinate, gets index -1 and key +inf.
__global__ __launch_bounds__(GQ_BT) void grid_nn_kernel(const float4* __restrict__ spts, const int* __restrict__ starts,
                                                        const GridInfo* __restrict__ gi, const float* __restrict__ qx,
                                                        const float* __restrict__ qy, const float* __restrict__ qz,
                                                        int nq, float max_key, int32_t* __restrict__ nn,
                                                        float* __restrict__ key) {
  __shared__ float4 s_buf[SPAN_U * GQ_BT];
  float4* buf = s_buf + threadIdx.x;
  const int t = blockIdx.x * GQ_BT + threadIdx.x;
  if (t >= nq) return;  // no barriers below
  const GridInfo G = *gi;
  const float qv[3] = {qx[t], qy[t], qz[t]};
  float bd = INFINITY;
  int bi = -1;
  if (isfinite(qv[0]) && isfinite(qv[1]) && isfinite(qv[2])) {
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = cell_coord(qv[a], G.lo[a], G.h, G.dims[a]);
    const int rmax = max(G.dims[0], max(G.dims[1], G.dims[2]));
    for (int r = 0; r <= rmax; ++r) {
      shell_spans(starts, G, c, r, [&](int p0, int p1) {
        span_points(spts, p0, p1, buf, [&](const float4& P) {
          const int j = __float_as_int(P.w);
          const float ex = __fsub_rn(P.x, qv[0]), ey = __fsub_rn(P.y, qv[1]), ez = __fsub_rn(P.z, qv[2]);
          const float d2 = __fadd_rn(__fadd_rn(__fmul_rn(ex, ex), __fmul_rn(ey, ey)), __fmul_rn(ez, ez));
          if (key_less(d2, j, bd, bi)) {
            bd = d2;
            bi = j;
          }
        });
      });
      // distance from the query to any cell outside the searched cube
      double lb = INFINITY;
      bool all = true;
      for (int a = 0; a < 3; ++a) {
        if (c[a] - r > 0) {
          lb = fmin(lb, (double)qv[a] - ((double)G.lo[a] + (double)(c[a] - r) * (double)G.h));
          all = false;
        }
        if (c[a] + r < G.dims[a] - 1) {
          lb = fmin(lb, ((double)G.lo[a] + (double)(c[a] + r + 1) * (double)G.h) - (double)qv[a]);
          all = false;
        }
      }
      if (all) break;
      const double lbs = lb - 1e-3 * (double)G.h;
      // nothing unsearched can beat the current best, or reach max_key
      if (lbs > 0.0 && fmin((double)bd, (double)max_key) * 1.00001 < lbs * lbs) break;
    }
  }
  if (!(bd <= max_key)) {
    bd = INFINITY;
    bi = -1;
  }
  nn[t] = bi;
  key[t] = bd;
}

// ---------------------------------------------------------------- batches
// The same exact search for many clouds (one launch per phase for all of
// them): every cloud has its own grid and workspace region, and blocks are
// mapped to clouds through a job table and a (cloud, block) list.
struct GridJob {
  const float* x;
  const float* y;
  const float* z;
  float* a_out;
  int n, max_cells;
  GridInfo* gi;
  int* cell_of;
  int* counts;
  int* cursor;
  int* starts;
  float4* spts;
  float4* p4;
  int32_t* nbr;
  int* far;
  int* far2;
};

// Job c of the table, with its pointers marked as global memory (gptr).
__device__ inline GridJob job_at(const GridJob* jobs, int c) {
  GridJob J = jobs[c];
  J.x = gptr(J.x), J.y = gptr(J.y), J.z = gptr(J.z), J.a_out = gptr(J.a_out), J.gi = gptr(J.gi);
  J.cell_of = gptr(J.cell_of), J.counts = gptr(J.counts), J.cursor = gptr(J.cursor), J.starts = gptr(J.starts);
  J.spts = gptr(J.spts), J.p4 = gptr(J.p4), J.nbr = gptr(J.nbr), J.far = gptr(J.far), J.far2 = gptr(J.far2);
  return J;
}

__global__ __launch_bounds__(1024) void grid_setup_batch_kernel(const GridJob* __restrict__ jobs) {
  const GridJob J = job_at(jobs, blockIdx.x);
  grid_setup_body(J.x, J.y, J.z, J.n, J.max_cells, J.gi, J.far, J.far2);
}

__global__ __launch_bounds__(1024) void grid_refine_batch_kernel(const GridJob* __restrict__ jobs) {
  const GridJob J = job_at(jobs, blockIdx.x);
  grid_refine_body(J.counts, J.n, J.max_cells, J.gi);
}

// counts (and, with both, cursor) of every cell set to 0; grid (clouds, splits)
__global__ __launch_bounds__(1024) void grid_clear_batch_kernel(const GridJob* __restrict__ jobs, int both) {
  const GridJob J = job_at(jobs, blockIdx.x);
  for (int c = blockIdx.y * 1024 + threadIdx.x; c < J.max_cells; c += gridDim.y * 1024) {
    J.counts[c] = 0;
    if (both) J.cursor[c] = 0;
  }
}

__global__ __launch_bounds__(256) void grid_count_batch_kernel(const GridJob* __restrict__ jobs,
                                                               const int2* __restrict__ bmap) {
  const int2 cb = bmap[blockIdx.x];
  const GridJob J = job_at(jobs, cb.x);
  grid_count_point(J.x, J.y, J.z, J.n, J.gi, J.cell_of, J.counts, cb.y * 256 + threadIdx.x);
}

// Exclusive scan of one cloud's cell counts into starts[0, max_cells], one
// block per cloud, 1024 cells per step: wave scans by shuffles, then the
// wave totals, then the running carry.
__global__ __launch_bounds__(1024) void grid_scan_batch_kernel(const GridJob* __restrict__ jobs) {
  __shared__ int s_w[16];
  __shared__ int s_carry;
  const GridJob J = job_at(jobs, blockIdx.x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < J.max_cells; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < J.max_cells ? J.counts[i] : 0;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(x, off, 64);
      if (lane >= off) x += o;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    int before = s_carry;
    for (int u = 0; u < w; ++u) before += s_w[u];
    if (i < J.max_cells) J.starts[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int u = 0; u < 16; ++u) tot += s_w[u];
      s_carry += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) J.starts[J.max_cells] = s_carry;
}

__global__ __launch_bounds__(256) void grid_scatter_batch_kernel(const GridJob* __restrict__ jobs,
                                                                 const int2* __restrict__ bmap) {
  const int2 cb = bmap[blockIdx.x];
  const GridJob J = job_at(jobs, cb.x);
  grid_scatter_point(J.x, J.y, J.z, J.n, J.cell_of, J.starts, J.cursor, J.spts, J.p4, cb.y * 256 + threadIdx.x);
}

template <int KC>
__global__ __launch_bounds__(GQ_BT) void grid_knn_batch_kernel(const GridJob* __restrict__ jobs,
                                                               const int2* __restrict__ bmap, int k) {
  __shared__ float4 s_buf[SPAN_U * GQ_BT];
  __shared__ uint64_t s_cand[KNN_CB * GQ_BT];
  const int2 cb = bmap[blockIdx.x];
  const GridJob J = job_at(jobs, cb.x);
  grid_knn_query<KC>(J.spts, nullptr, J.starts, J.gi, J.n, k, KNN_RCAP, J.far, J.nbr, cb.y * GQ_BT + threadIdx.x,
                     s_buf + threadIdx.x, s_cand + threadIdx.x, 0);
}

// The far queries of all clouds as one list: positions [off[c], off[c + 1])
// are cloud c's far list (far, or far2 with `second`), with off (fq + 2,
// n_clouds + 1 entries) the exclusive scan of their counts.  One block.
__global__ __launch_bounds__(1024) void far_scan_batch_kernel(const GridJob* __restrict__ jobs, int n_clouds,
                                                              int* __restrict__ fq, int second) {
  __shared__ int s_w[16];
  __shared__ int s_carry;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int* off = fq + 2;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < n_clouds; base += 1024) {
    const int c = base + threadIdx.x;
    const int v = c < n_clouds ? gptr(second ? jobs[c].far2 : jobs[c].far)[0] : 0;
    int x = v;
    for (int d = 1; d < 64; d <<= 1) {
      const int o = __shfl_up(x, d, 64);
      if (lane >= d) x += o;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    int before = s_carry;
    for (int u = 0; u < w; ++u) before += s_w[u];
    if (c < n_clouds) off[c] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int u = 0; u < 16; ++u) tot += s_w[u];
      s_carry += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) off[n_clouds] = s_carry;
}

// Cloud of far-list position g: the last c with off[c] <= g (a cloud without
// far queries shares its offset with the next one, so the last such c is
// the one whose range holds g), by bisection (off[n_clouds] = total > g).
__device__ inline int far_cloud_of(const int* __restrict__ off, int n_clouds, int g) {
  int lo = 0, hi = n_clouds;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The handed-over queries of all clouds, one lane each: lane g of the grid
// takes positions g, g + grid size, ... of the concatenated lists (far) and
// resumes the one-lane search at shell r0; a query not finished after shell
// r0 is handed over again, to far2, so that the few deep searches do not
// hold up waves of queries that need one shell more.  (A lane per query suits the batch's many handed-over
// queries; the one-cloud pass keeps a wave per query, which finishes a few
// of them sooner.)
template <int KC>
__global__ __launch_bounds__(GQ_BT) void grid_knn_far_lanes_kernel(const GridJob* __restrict__ jobs, int n_clouds,
                                                                   const int* __restrict__ fq, int k, int r0) {
  __shared__ float4 s_buf[SPAN_U * GQ_BT];
  __shared__ uint64_t s_cand[KNN_CB * GQ_BT];
  const int* off = fq + 2;
  const int total = off[n_clouds];
  for (int g = blockIdx.x * GQ_BT + threadIdx.x; g < total; g += gridDim.x * GQ_BT) {
    const int c = far_cloud_of(off, n_clouds, g);
    const GridJob J = job_at(jobs, c);
    grid_knn_query<KC>(J.spts, J.p4, J.starts, J.gi, J.n, k, r0, J.far2, J.nbr, J.far[1 + (g - off[c])],
                       s_buf + threadIdx.x, s_cand + threadIdx.x, r0);
  }
}

// The queries still open after the lane pass, one wave each (deep searches,
// which one lane would take long over): wave w of the grid takes positions
// w, w + number of waves, ... of the concatenated lists (far2), resuming at
// shell r0.
template <int KC>
__global__ __launch_bounds__(GQ_BT) void grid_knn_far_waves_batch_kernel(const GridJob* __restrict__ jobs,
                                                                         int n_clouds, const int* __restrict__ fq,
                                                                         int k, int r0) {
  __shared__ float4 s_buf[SPAN_U * GQ_BT];
  const int* off = fq + 2;
  const int total = off[n_clouds];
  const int n_waves = (gridDim.x * GQ_BT) >> 6;
  for (int g = (blockIdx.x * GQ_BT + threadIdx.x) >> 6; g < total; g += n_waves) {
    const int c = far_cloud_of(off, n_clouds, g);
    const GridJob J = job_at(jobs, c);
    const GridInfo G = *J.gi;
    grid_knn_far_query<KC>(J.spts, J.p4, J.starts, G, k, J.far2[1 + (g - off[c])], J.nbr, s_buf + threadIdx.x, r0);
  }
}

// Block (cloud, block) of the list: CURV_BT points of one cloud, as
// curvature_kernel.
static_assert(CURV_BT == 256, "the (cloud, block) list counts blocks of 256 points");
__global__ __launch_bounds__(CURV_BT) void curvature_batch_kernel(const GridJob* __restrict__ jobs,
                                                                  const int2* __restrict__ bmap, int k) {
  extern __shared__ int s_nb[];
  const int2 cb = bmap[blockIdx.x];
  const GridJob J = job_at(jobs, cb.x);
  if (J.a_out) curvature_block(J.p4, J.n, k, J.nbr, J.a_out, cb.y, s_nb);
}

// The handed-over queries of a batch: shell KNN_RCAP + 1 with a lane per
// query (far -> far2), then those still open with a wave per query.  The lane
// pass gets more blocks than fit at once, so that every CU holds as many
// waves as its LDS allows while the list lasts.  (Measured on the 512 clouds
// of the batch workload: a wave per query for all of them took 1.5 times as
// long, a lane per query for the deeper shells as well 1.2 to 2 times.)
template <class LanesK, class WavesK>
void far_passes(LanesK lanes, WavesK waves, const GridJob* d_jobs, int n_clouds, int* d_fq, int k, hipStream_t st) {
  const dim3 gl(2048), gw(1024), bt(GQ_BT);
  hipLaunchKernelGGL(far_scan_batch_kernel, dim3(1), dim3(1024), 0, st, d_jobs, n_clouds, d_fq, 0);
  hipLaunchKernelGGL(lanes, gl, bt, 0, st, d_jobs, n_clouds, (const int*)d_fq, k, KNN_RCAP + 1);
  hipLaunchKernelGGL(far_scan_batch_kernel, dim3(1), dim3(1024), 0, st, d_jobs, n_clouds, d_fq, 1);
  hipLaunchKernelGGL(waves, gw, bt, 0, st, d_jobs, n_clouds, (const int*)d_fq, k, KNN_RCAP + 2);
}

size_t grid_knn_batch_workspace(const int* n, int n_clouds, int k) {
  size_t b = 0;
  int64_t blocks = 0;
  for (int c = 0; c < n_clouds; ++c) {
    b += grid_knn_workspace(n[c], k);
    blocks += (n[c] + 255) / 256;
  }
  b += ((sizeof(GridJob) * (size_t)n_clouds + 255) & ~size_t(255)) + ((sizeof(int2) * (size_t)blocks + 255) & ~size_t(255));
  b += (sizeof(int) * ((size_t)n_clouds + 3) + 255) & ~size_t(255);  // far list offsets (at + 2)
  return b;
}

hipError_t launch_grid_knn_batch(const float* const* x, const float* const* y, const float* const* z, const int* n,
                                 float* const* a_out, int32_t* const* idx_out, int n_clouds, int k, void* ws,
                                 hipStream_t st) {
  if (n_clouds < 1) return hipSuccess;
  std::vector<GridJob> jobs(n_clouds);
  std::vector<int2> bmap;
  char* p = (char*)ws;
  for (int c = 0; c < n_clouds; ++c) {
    const GridBufs B = carve_grid(p, n[c], k);
    p += grid_knn_workspace(n[c], k);
    int32_t* lists = (idx_out && idx_out[c]) ? idx_out[c] : B.nbr;
    jobs[c] = GridJob{x[c], y[c], z[c], a_out ? a_out[c] : nullptr, n[c], grid_max_cells(n[c]), B.gi, B.cell_of,
                      B.counts, B.cursor, B.starts, B.spts, B.p4, lists, B.far, B.far2};
    for (int b = 0; b < (n[c] + 255) / 256; ++b) bmap.push_back(make_int2(c, b));
  }
  GridJob* d_jobs = (GridJob*)p;
  p += (sizeof(GridJob) * (size_t)n_clouds + 255) & ~size_t(255);
  int2* d_bmap = (int2*)p;
  p += (sizeof(int2) * bmap.size() + 255) & ~size_t(255);
  int* d_fq = (int*)p;
  hipError_t e = hipMemcpyAsync(d_jobs, jobs.data(), sizeof(GridJob) * jobs.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(d_bmap, bmap.data(), sizeof(int2) * bmap.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  // the copies read host vectors that go out of scope below
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  const dim3 gc((unsigned)n_clouds), gcs((unsigned)n_clouds, 16), gb((unsigned)bmap.size());
  hipLaunchKernelGGL(grid_setup_batch_kernel, gc, dim3(1024), 0, st, d_jobs);
  hipLaunchKernelGGL(grid_clear_batch_kernel, gcs, dim3(1024), 0, st, d_jobs, 0);
  hipLaunchKernelGGL(grid_count_batch_kernel, gb, dim3(256), 0, st, d_jobs, d_bmap);
  hipLaunchKernelGGL(grid_refine_batch_kernel, gc, dim3(1024), 0, st, d_jobs);
  hipLaunchKernelGGL(grid_clear_batch_kernel, gcs, dim3(1024), 0, st, d_jobs, 1);
  hipLaunchKernelGGL(grid_count_batch_kernel, gb, dim3(256), 0, st, d_jobs, d_bmap);
  hipLaunchKernelGGL(grid_scan_batch_kernel, gc, dim3(1024), 0, st, d_jobs);
  hipLaunchKernelGGL(grid_scatter_batch_kernel, gb, dim3(256), 0, st, d_jobs, d_bmap);

  if (k <= 8) {
    hipLaunchKernelGGL(grid_knn_batch_kernel<8>, gb, dim3(GQ_BT), 0, st, d_jobs, d_bmap, k);
    far_passes(grid_knn_far_lanes_kernel<8>, grid_knn_far_waves_batch_kernel<8>, d_jobs, n_clouds, d_fq, k, st);
  } else if (k <= 16) {
    hipLaunchKernelGGL(grid_knn_batch_kernel<16>, gb, dim3(GQ_BT), 0, st, d_jobs, d_bmap, k);
    far_passes(grid_knn_far_lanes_kernel<16>, grid_knn_far_waves_batch_kernel<16>, d_jobs, n_clouds, d_fq, k, st);
  } else if (k <= 24) {
    hipLaunchKernelGGL(grid_knn_batch_kernel<24>, gb, dim3(GQ_BT), 0, st, d_jobs, d_bmap, k);
    far_passes(grid_knn_far_lanes_kernel<24>, grid_knn_far_waves_batch_kernel<24>, d_jobs, n_clouds, d_fq, k, st);
  } else {
    hipLaunchKernelGGL(grid_knn_batch_kernel<32>, gb, dim3(GQ_BT), 0, st, d_jobs, d_bmap, k);
    far_passes(grid_knn_far_lanes_kernel<32>, grid_knn_far_waves_batch_kernel<32>, d_jobs, n_clouds, d_fq, k, st);
  }
  hipLaunchKernelGGL(curvature_batch_kernel, gb, dim3(CURV_BT), curv_lds_bytes(k), st, d_jobs, d_bmap, k);
  return hipGetLastError();
}

hipError_t launch_grid_nn(const float* x, const float* y, const float* z, int n, const float* qx, const float* qy,
                          const float* qz, int nq, float max_key, int32_t* nn, float* key, void* ws, hipStream_t st) {
  const GridBufs B = carve_grid(ws, n, 1);
  if (hipError_t e = build_grid(x, y, z, n, B, st)) return e;
  hipLaunchKernelGGL(grid_nn_kernel, dim3((nq + GQ_BT - 1) / GQ_BT), dim3(GQ_BT), 0, st, B.spts, B.starts, B.gi, qx,
                     qy, qz, nq, max_key, nn, key);
  return hipGetLastError();
}

}  // namespace sgr
