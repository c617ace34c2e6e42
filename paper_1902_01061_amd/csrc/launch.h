// Host-side launchers shared between the kernel translation units and the
// C-ABI layer (internal; not part of the public interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace sgr {

struct PrepParams {
  double p;
  double sigma;
  double eps;
  double G1;
  double dt2;
  int32_t E;
  int32_t g_mode;
  int32_t cold_svd = 0;  // 1: the update's SVD starts cold (a deterministic function of C)
  double sigma_scale = 1.0;  // multiplies sigma (explicit or the std of the reference curvatures)
  double momentum = 0.0;     // share of the previous translation carried by the update
};

struct ForceArgs {
  const float* y0x;
  const float* y0y;
  const float* y0z;
  const float* aY;
  const float* mY;      // template masses or nullptr
  const float4* ref4;   // packed reference (x - xbar, b)
  const float* reflw;   // log2 weights
  const double* pose;   // 13 doubles
  const Derived* dv;
  int M, N;
  int chunk_len;        // reference points per block (multiple of the LDS tile), or 0: n_chunks
                        // balanced chunks cut at multiples of 64 points (force kernel only)
  int n_chunks;
  int t;                // iteration index (G from eq. 12 when G <= 0)
  double G;             // explicit force constant, or <= 0
  double* wpart;        // [n_blocks][WR_STRIDE]
  double* fpart;        // [n_chunks][M][3] or nullptr
  const int* perm = nullptr;  // template visiting order (see launch_sort_perm) or nullptr
  // Template packed in visiting order (launch_pack_tmpl), or nullptr: position
  // ip holds (x0, y0, z0, b) and (a, m) of the point perm[ip].
  const float4* tm4 = nullptr;
  const float2* tmx = nullptr;
};

// A cloud for the batched moments kernel.
struct CloudDesc {
  const float* x;
  const float* y;
  const float* z;
  float* a_out;
  int n;
  int pad;
};

// One registration's inputs for the batched prepare / pack kernels.
struct PrepDesc {
  const float* xx;
  const float* xy;
  const float* xz;
  const float* aX;
  const float* wX;
  const float* aY;
  const float* mY;
  const double* mom_t;
  const double* mom_r;
  int64_t ref_off;  // offset of the padded packed reference
  int N, M;
  int blk0;         // first pack block of this registration
  int pad;
};

// One registration of a batch (device-resident table).
struct RegDesc {
  const float* y0x;
  const float* y0y;
  const float* y0z;
  const float* aY;
  const float* mY;
  int64_t ref_off;      // offset of its packed reference in the batch arrays
  int M, N;
  int wslot0;           // first wrench slot of its items
  int n_items;
  int* perm;            // template visiting order [M]
  float4* tm4;          // template packed in that order [M]
  float2* tmx;          // [M]
};

// A batch descriptor read on the device, with its pointers marked as
// global memory (gptr).
__device__ inline PrepDesc prep_at(const PrepDesc* d, int r) {
  PrepDesc g = d[r];
  g.xx = gptr(g.xx), g.xy = gptr(g.xy), g.xz = gptr(g.xz), g.aX = gptr(g.aX), g.wX = gptr(g.wX);
  g.aY = gptr(g.aY), g.mY = gptr(g.mY), g.mom_t = gptr(g.mom_t), g.mom_r = gptr(g.mom_r);
  return g;
}

__device__ inline RegDesc reg_at(const RegDesc* d, int r) {
  RegDesc g = d[r];
  g.y0x = gptr(g.y0x), g.y0y = gptr(g.y0y), g.y0z = gptr(g.y0z), g.aY = gptr(g.aY), g.mY = gptr(g.mY);
  g.perm = gptr(g.perm), g.tm4 = gptr(g.tm4), g.tmx = gptr(g.tmx);
  return g;
}

struct BatchArgs {
  const RegDesc* regs;
  const int4* items;    // (registration, template block, chunk, wrench slot)
  int n_items;
  const float4* ref4;
  const float* reflw;
  const double* poses;  // [B][13]
  const Derived* dvs;   // [B]
  int chunk_len;
  int t;
  double* wpart;
};

struct AdjArgs {
  const float* y0x;
  const float* y0y;
  const float* y0z;
  const float* aY;
  const float* mY;
  const float4* ref4;
  const float* reflw;
  const Derived* dv;
  int M, N;
  int chunk_len, n_chunks, nblk;  // chunk_len 0: n_chunks balanced chunks
  bool p1;              // p == 1: no distance-law derivative terms
  double G;             // force constant
  const float* f;       // forces of the forward pass [M][3]
  const float* gf;      // upstream gradient of f [M][3]
  const double* gw;     // upstream gradient of the wrench (F[3], K[9])
  float* lam;           // [M][3] workspace
  double* ypart;        // [n_chunks][M][4] workspace
  double* spart;        // [nblk][2] workspace
  float* grad_y;        // [M][3]
  float* grad_m;        // [M] or nullptr
  double* grad_se;      // [2] (sigma, eps) or nullptr
};

hipError_t launch_adjoint(const AdjArgs& A, int R, double* fsum_tmp, hipStream_t st);
// Resident blocks per CU of the adjoint pair kernel; granularity of its
// balanced reference chunks (AdjArgs.chunk_len = 0).
int adj_blocks_per_cu(int R, bool p1);
int adj_chunk_gran();
// Adjoint of one rigid update: gpose_in[13] and gW[16] from gpose_out[13]
// (pose_in the pose the update started from, W its wrench).
hipError_t launch_update_bwd(const double* pose_in, const double* W, const double* gpose_out, const Derived* dv,
                             double* gpose_in, double* gW, hipStream_t st);
// o = s R p + t for the template points (FP32 out).
hipError_t launch_pose_points(const float* x, const float* y, const float* z, int M, const double* pose, float* ox,
                              float* oy, float* oz, hipStream_t st);
// gpose += pose cotangent of the per-point gradient gy [M][3] of y = s R p + t;
// part needs pose_grad_blocks(M) * 12 doubles.
int pose_grad_blocks(int M);
hipError_t launch_pose_grad(const float* gy, const float* x, const float* y, const float* z, int M, const double* pose,
                            double* part, double* gpose, hipStream_t st);
hipError_t launch_axpy(const double* x, int n, double* y, hipStream_t st);
hipError_t launch_fill(double* p, int n, double v, hipStream_t st);
hipError_t launch_fill_f(float* p, int64_t n, float v, hipStream_t st);
hipError_t launch_identity_pose(double* pose, hipStream_t st);
hipError_t launch_fill_i(int* p, int n, hipStream_t st);
int grid_max_cells(int n);
size_t grid_knn_workspace(int n, int k);
// The grid search (launch_grid_knn) for many clouds at once: cloud c has
// n[c] points at x[c], y[c], z[c] and receives its curvatures in a_out[c]
// (a_out nullable) and, when idx_out and idx_out[c] are given, its
// neighbour lists there.  One launch per phase for all clouds; neighbour
// lists and curvatures equal those of launch_grid_knn on each cloud.
// Synchronises the stream once (the job table is copied from host memory).
size_t grid_knn_batch_workspace(const int* n, int n_clouds, int k);
hipError_t launch_grid_knn_batch(const float* const* x, const float* const* y, const float* const* z, const int* n,
                                 float* const* a_out, int32_t* const* idx_out, int n_clouds, int k, void* ws,
                                 hipStream_t st);
hipError_t launch_grid_knn(const float* x, const float* y, const float* z, int n, int k, float* a_out,
                           int32_t* idx_out, void* ws, hipStream_t st);
// Nearest point of the cloud (x, y, z, n) to each query among those with
// key <= max_key (-1 / +inf if none), same order as the grid kNN (FP32 key,
// ties by index); ws: grid_knn_workspace(n, 1) bytes.
hipError_t launch_grid_nn(const float* x, const float* y, const float* z, int n, const float* qx, const float* qy,
                          const float* qz, int nq, float max_key, int32_t* nn, float* key, void* ws, hipStream_t st);
// Change flags of the posed template against the reference (see change.hip);
// ws: change_workspace(M, N) bytes.
size_t change_workspace(int M, int N);
hipError_t launch_change(const float* yx, const float* yy, const float* yz, const float* aY, int M, const float* xx,
                         const float* xy, const float* xz, const float* aX, int N, const double* pose, float tau2,
                         double shape_thr, uint8_t* flags, int32_t* nn, float* key, void* ws, hipStream_t st);

hipError_t launch_moments(const float* x, const float* y, const float* z, int64_t n, double* out, hipStream_t st);
// Force with vector descriptors (p = 1, g = s) on the matrix cores.
struct VForceArgs {
  const void* At;       // template augmented rows [Mpad]: K floats, or K halves (split f16)
  const void* Bt;       // reference augmented rows [Npad], same form
  const float4* ref4;   // reference x, y, z (centred at xbar), |x|^2 [Npad]
  const float* y0x;
  const float* y0y;
  const float* y0z;
  const float* mY;      // template masses or nullptr
  const double* pose;
  const Derived* dv;
  int M, N, K, n_chunks, t;
  bool half;            // split-f16 rows and instructions (K = vforce_half_K(D))
  double G;             // > 0 overrides eq. 12
  double* wpart;        // [n_iblk * n_chunks][WR_STRIDE]
  double* fpart;        // [n_chunks][M][3] (WF only)
  double* spart = nullptr;  // with WU: [n_chunks][M][5] pair sums instead of forces and wrench
};
// Far template rows (standardised descriptor more than 8 spreads from the
// mean, within reach of a reference descriptor), listed in increasing order
// into far_idx[0..n), n in far_idx[M] (far_idx holds M + 1 ints).  Their
// evaluation after the contraction reads reference records built once per
// registration (launch_vfar_ref: vfar_pad_refs(N) records of vfar_stride(D)
// doubles) and leaves per-segment sums in part (vfar_part_doubles(M)
// doubles); one wrench slot per far row from slot0.
__host__ __device__ inline int vfar_db(int D) { return 4 * ((D + 3) / 4); }
__host__ __device__ inline int vfar_stride(int D) { return vfar_db(D) + 6; }
size_t vfar_part_doubles(int M);
int vfar_pad_refs(int N);
void vfar_prepare(int D);  // host queries of the far-row launch, outside stream capture
hipError_t launch_vfar_list(const float* aY, int M, int D, const double* vd, const Derived* dv, int* far_idx,
                            hipStream_t st);
hipError_t launch_vfar_ref(const float* aX, const float* wX, int N, int D, const double* vd, const float4* ref4,
                           double* refd, hipStream_t st);
hipError_t launch_vfar(const VForceArgs& A, const float* aY, int D, const double* vd, const double* refd,
                       const int* far_idx, int n_far, double* part, int slot0, bool wu, bool wf, int n_cu,
                       hipStream_t st);
int vforce_K(int D);
// Halves per split-f16 row: the contraction [h, h, l] . [h, l, h] of length
// 3 (D + 2), padded to whole 16x16x32 instructions.
int vforce_half_K(int D);
int vforce_pad_rows(int M);
int vforce_pad_refs(int N);
int vforce_n_iblk(int M);
int vforce_chunks(int M, int N, int n_cu);
// vd: [36] doubles: reference mean (32), sigma, log2(e) / sigma^2, the
// largest |a - abar|^2 / sigma^2 over the reference and the template rows
// that enter the contraction (for vforce_half_ok), and over the reference
hipError_t launch_vprep(const float* aX, int64_t N, const float* aY, int64_t M, int D, double sigma, Derived* dv,
                        double* vd, hipStream_t st);
bool vforce_half_ok(double cmax);
// Rows: vforce_K(D) floats each (half = false) or vforce_half_K(D) halves
// each (half = true).
hipError_t launch_vpack(const float* X, const float* Y, const float* Z, const float* aX, const float* wX, int N,
                        const float* aY, int M, int D, bool half, const Derived* dv, const double* vd, void* Bt,
                        float4* ref4, void* At, hipStream_t st);
hipError_t launch_vforce(const VForceArgs& A, bool wu, bool wf, hipStream_t st);
// Local polynomial descriptor: out[n][3] = (mu1, mu2, residual) of a quadric
// fitted to the k nearest neighbours (k >= 6).
size_t poly_workspace(int n, int k);
hipError_t launch_poly(const float* x, const float* y, const float* z, int n, int k, float* out, void* ws,
                       hipStream_t st);
// Soft histogram of normals: h_out[n][D] from the k nearest neighbours.
size_t normal_hist_workspace(int n, int k);
hipError_t launch_normal_hist(const float* x, const float* y, const float* z, int n, int k, int D, float* h_out,
                              void* ws, hipStream_t st);

// Pose-independent pair sums of the p = 1 law: S[ip] = (sum_j c, sum_j c x_j
// (3), sum_j c |x_j|^2) per template point in visiting order, c the pair
// weight exp2(lw_j - (b_i - b_j)^2), from the packed template and reference;
// part holds pinv_chunks(M, N, n_cu) * M * 5 doubles.  launch_pinv is the
// per-iteration force from them: pinv_blocks(M) wrench partials in wpart
// (the layout of the force kernel, for launch_update).
int pinv_chunks(int M, int N, int n_cu);
int pinv_blocks(int M);
hipError_t launch_psum(const float4* tm4, int M, const float4* ref4, const float* lw, int N, int n_chunks,
                       double* part, double* S, hipStream_t st);
hipError_t launch_pinv(const float4* tm4, const float2* tmx, const double* S, int M, const double* pose,
                       const Derived* dv, int t, bool wu, double* wpart, hipStream_t st);
// S[i] = sum over n_chunks of part[chunk][i] (5 values per point, fixed order).
hipError_t launch_psum_reduce(const double* part, int M, int n_chunks, double* S, hipStream_t st);
// Template in its own order for launch_pinv: (x0, y0, z0, 0) and (0, m).
hipError_t launch_pack_plain(const float* x, const float* y, const float* z, const float* mY, int M, float4* tm4,
                             float2* tmx, hipStream_t st);
// Batched forms: tblk lists (registration, block of 256 template points);
// registration r's sums sit at template offset poff[r] of S.  regs_p is
// regs with wslot0 / n_items describing one wrench slot per listed block.
hipError_t launch_psum_batch(const RegDesc* regs, const int2* tblk, int n_tblk, const int* poff, const float4* ref4,
                             const float* lw, double* S, hipStream_t st);
hipError_t launch_pinv_batch(const RegDesc* regs_p, const int2* tblk, int n_tblk, const int* poff, const double* S,
                             const double* poses, const Derived* dvs, int t, bool wu, double* wpart, hipStream_t st);

// Curvature of the radius neighbourhood of every point: members have float32
// key <= r2, where r2 = (float)(scale2 * mom[9]) when mom is given (mom[9] =
// largest covariance eigenvalue, as launch_moments writes it), else r2_in.
// a_out and cnt_out (member counts) may each be nullptr.  ws: at least
// radius_desc_workspace(n) bytes (Morton-ordered copy, tile boxes, sort).
size_t radius_desc_workspace(int n);
hipError_t launch_radius_desc(const float* x, const float* y, const float* z, int n, const double* mom, double scale2,
                              float r2_in, float* a_out, int32_t* cnt_out, void* ws, hipStream_t st);
hipError_t launch_prepare(const float* aX, const float* wX, int64_t N, const float* aY, const float* mY, int64_t M,
                          const double* mom_t, const double* mom_r, const PrepParams& P, Derived* out, hipStream_t st);
hipError_t launch_pack_ref(const float* x, const float* y, const float* z, const float* aX, const float* wX, int64_t N,
                           const Derived* dv, float4* ref4, float* lw, hipStream_t st);
hipError_t launch_force(const ForceArgs& A, int R, int pm, bool want_u, bool want_f, hipStream_t st, bool sm);
// Resident blocks per CU of the force kernel without energy or per-point
// output (R points per lane, p mode, scalar-load variant).
int force_blocks_per_cu(int R, int pm, bool sm);
hipError_t launch_moments_batch(const CloudDesc* clouds, int n_clouds, double* out, hipStream_t st);
hipError_t launch_prepare_batch(const PrepDesc* d, int B, const PrepParams& P, Derived* outs, hipStream_t st);
hipError_t launch_pack_batch(const PrepDesc* d, const int* blk2reg, int n_blocks, const Derived* dvs, float4* ref4,
                             float* lw, hipStream_t st);
hipError_t launch_update_batch(const double* wpart, const RegDesc* regs, int B, double* poses, Derived* dvs, int t,
                               int do_update, double* energy_out, double* stats, int E, hipStream_t st);
hipError_t launch_init_multistart(const double* R0, int S, const double* mom_t, double* poses, hipStream_t st);
hipError_t launch_argmin(const double* v, int n, int32_t* out, hipStream_t st);
hipError_t launch_force_batch(const BatchArgs& B, int R, int pm, bool want_u, int grid, hipStream_t st);
// Template visiting order: perm = indices of aY in ascending order (stable).
// ws must hold sort_perm_workspace(n, nseg) bytes (n points, nseg registrations).
size_t sort_perm_workspace(int64_t n, int nseg);
// Template copied into visiting order (x0, y0, z0, b) / (a, m), b from dv.
hipError_t launch_pack_tmpl(const float* x, const float* y, const float* z, const float* aY, const float* mY, int M,
                            const int* perm, const Derived* dv, float4* tm4, float2* tmx, hipStream_t st);
hipError_t launch_pack_tmpl_batch(const RegDesc* regs, int B, int max_M, const Derived* dvs, hipStream_t st);
hipError_t launch_sort_perm(const float* aY, int M, int* perm, void* ws, hipStream_t st);
// Batch form: registration r sorts regs[r].aY into perm[off[r] .. off[r+1]) (off on the device, B + 1 entries).
hipError_t launch_sort_perm_batch(const RegDesc* regs, int B, const int* off, int64_t total, int max_M, int* perm,
                                  void* ws, hipStream_t st);
hipError_t launch_force_mixed(const ForceArgs& A, bool want_f, hipStream_t st);
int mixed_points_per_block();
// f_out[perm[ip]] (perm nullable) = sum over chunks of fpart[chunk][ip] (visiting order).
hipError_t launch_reduce_f(const double* fpart, int n_chunks, int M, const int* perm, float* f_out, hipStream_t st);
int force_points_per_block(int R);
int force_chunk_gran();
int force_tile_j();
hipError_t launch_update(const double* wpart, int nblk, const double* pose_in, double* pose_out, Derived* dv, int t,
                         double G_fixed, int do_update, double* wrench_out, double* stats_row, hipStream_t st);
hipError_t launch_residual(const float* yx, const float* yy, const float* yz, int M, const float* xx, const float* xy,
                           const float* xz, int N, const double* pose, const int32_t* corr, double* part, int nblk,
                           double* rmse_out, hipStream_t st);
int residual_blocks(int M);

}  // namespace sgr
