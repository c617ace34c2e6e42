// C-ABI layer: argument checks, workspace, tile selection, graph capture of
// the iteration loop.  Every numeric step is a HIP kernel; this file only
// sequences launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sgreg.h"
#include "launch.h"
#include "tiles.h"

using namespace sgr;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return fail(SGR_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct GraphCache {
  std::vector<uint8_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct sgr_ctx {
  int device = 0;
  int n_cu = 256;
  hipStream_t cap = nullptr;
  char* ws = nullptr;
  size_t ws_size = 0;
  GraphCache gc;
  TileTable tiles;
};

namespace {

struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

int ensure_ws(sgr_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->ws_size) return SGR_OK;
  HIPCHK(hipDeviceSynchronize());
  if (ctx->ws) HIPCHK(hipFree(ctx->ws));
  ctx->ws = nullptr;
  ctx->ws_size = 0;
  size_t sz = bytes + bytes / 4 + (1 << 20);
  if (hipMalloc(&ctx->ws, sz) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return fail(SGR_ENOMEM, "workspace allocation of " + std::to_string(sz) + " bytes failed");
  }
  ctx->ws_size = sz;
  return SGR_OK;
}

int check_cloud(const sgr_cloud* c, const char* what) {
  if (!c) return fail(SGR_EINVAL, std::string(what) + ": NULL cloud");
  if (!c->x || !c->y || !c->z) return fail(SGR_EINVAL, std::string(what) + ": NULL coordinate array");
  if (c->n < 1) return fail(SGR_EINVAL, std::string(what) + ": empty cloud");
  if (c->n > (int64_t)1 << 30) return fail(SGR_EINVAL, std::string(what) + ": more than 2^30 points");
  return SGR_OK;
}

int check_params(const sgr_params* p) {
  if (!p) return fail(SGR_EINVAL, "NULL params");
  if (!std::isfinite(p->p)) return fail(SGR_EINVAL, "p must be finite");
  if (p->p < 1.0 && !(p->eps > 0)) return fail(SGR_EINVAL, "p < 1 needs eps > 0 (the force would diverge at r = 0)");
  if (p->g_mode != 0 && p->g_mode != 1) return fail(SGR_EINVAL, "g_mode must be 0 (g = s) or 1 (g = a a s)");
  if (!(p->G1 > 0) || !std::isfinite(p->G1)) return fail(SGR_EINVAL, "G1 must be positive");
  if (!std::isfinite(p->sigma) || !std::isfinite(p->eps) || p->eps < 0) return fail(SGR_EINVAL, "bad sigma/eps");
  if (!std::isfinite(p->dt2)) return fail(SGR_EINVAL, "bad dt2");
  return SGR_OK;
}

PrepParams prep_of(const sgr_params* p) {
  PrepParams P;
  P.p = p->p;
  P.sigma = p->sigma;
  P.eps = p->eps;
  P.G1 = p->G1;
  P.dt2 = p->dt2;
  P.E = p->E;
  P.g_mode = p->g_mode;
  return P;
}

int pmode_of(double p) { return p == 1.0 ? 1 : (p == 3.0 ? 3 : 0); }

// The packed reference is padded to whole tiles with zero-weight points.
size_t pad_n(int64_t N) { return (size_t)((N + 255) / 256) * 256; }

}  // namespace

extern "C" {

const char* sgr_last_error(void) { return g_err.c_str(); }

int sgr_create(sgr_ctx** out, int device) {
  if (!out) return fail(SGR_EINVAL, "NULL ctx pointer");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(SGR_EINVAL, "no such device");
  HIPCHK(hipSetDevice(device));
  sgr_ctx* c = new sgr_ctx();
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(SGR_EHIP, "stream creation failed");
  }
  c->tiles.init(c->n_cu);
  *out = c;
  return SGR_OK;
}

int sgr_destroy(sgr_ctx* ctx) {
  if (!ctx) return SGR_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->gc.exec) (void)hipGraphExecDestroy(ctx->gc.exec);
  if (ctx->gc.graph) (void)hipGraphDestroy(ctx->gc.graph);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  delete ctx;
  return SGR_OK;
}

int sgr_descriptors(sgr_ctx* ctx, const sgr_cloud* c, int k, float* a_out, double* moments_out, sgr_stream_t stream) {
  if (!ctx) return fail(SGR_EINVAL, "NULL ctx");
  if (int e = check_cloud(c, "cloud")) return e;
  if (k < 1 || k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  if (c->n < k) return fail(SGR_EINVAL, "cloud has fewer points than k");
  if (!a_out && !moments_out) return fail(SGR_EINVAL, "nothing to compute");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  if (a_out) HIPCHK(launch_knn_desc(c->x, c->y, c->z, (int)c->n, k, a_out, nullptr, st));
  if (moments_out) HIPCHK(launch_moments(c->x, c->y, c->z, c->n, moments_out, st));
  return SGR_OK;
}

int sgr_knn(sgr_ctx* ctx, const sgr_cloud* c, int k, int32_t* idx_out, sgr_stream_t stream) {
  if (!ctx || !idx_out) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(c, "cloud")) return e;
  if (k < 1 || k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  if (c->n < k) return fail(SGR_EINVAL, "cloud has fewer points than k");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(launch_knn_desc(c->x, c->y, c->z, (int)c->n, k, nullptr, idx_out, (hipStream_t)stream));
  return SGR_OK;
}

int sgr_step(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
             const double* mom_t, const double* mom_r, const sgr_params* prm, int t, const sgr_pose* in,
             sgr_pose* out, double* wrench_out, float* f_out, sgr_stream_t stream) {
  if (!ctx) return fail(SGR_EINVAL, "NULL ctx");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  if (!a_t || !a_r || !mom_t || !mom_r || !in || !out) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  const Tiles T = ctx->tiles.pick(M, N, pmode_of(prm->p));
  Carve cv{nullptr};
  cv.take<Derived>(1);
  cv.take<float4>(pad_n(N));
  cv.take<float>(pad_n(N));
  cv.take<double>((size_t)T.nblk * WR_STRIDE);
  if (f_out) cv.take<double>((size_t)T.n_chunks * M * 3);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  Derived* dv = w.take<Derived>(1);
  float4* ref4 = w.take<float4>(pad_n(N));
  float* lw = w.take<float>(pad_n(N));
  double* wpart = w.take<double>((size_t)T.nblk * WR_STRIDE);
  double* fpart = f_out ? w.take<double>((size_t)T.n_chunks * M * 3) : nullptr;

  HIPCHK(launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_t, mom_r, prep_of(prm), dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, N, dv, ref4, lw, st));
  ForceArgs A{tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, ref4, lw, (const double*)in, dv, M, N,
              T.chunk_len, T.n_chunks, t, 0.0, wpart, fpart};
  HIPCHK(launch_force(A, T.R, pmode_of(prm->p), wrench_out != nullptr, f_out != nullptr, st, T.sm));
  if (f_out) HIPCHK(launch_reduce_f(fpart, T.n_chunks, M, f_out, st));
  HIPCHK(launch_update(wpart, T.nblk, (const double*)in, (double*)out, dv, t, 0.0, 1, wrench_out, nullptr, st));
  return SGR_OK;
}

int sgr_register(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_params* prm, sgr_pose* inout,
                 double* stats, sgr_stream_t stream) {
  if (!ctx || !inout) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  if (prm->E < 1) return fail(SGR_EINVAL, "E must be >= 1");
  if (prm->k < 1 || prm->k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  if (tmpl->n < prm->k || ref->n < prm->k) return fail(SGR_EINVAL, "a cloud has fewer points than k");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  const int pm = pmode_of(prm->p);
  const Tiles T = ctx->tiles.pick(M, N, pm);
  Carve cv{nullptr};
  cv.take<float>(N);
  cv.take<float>(M);
  cv.take<double>(20);
  cv.take<Derived>(1);
  cv.take<float4>(pad_n(N));
  cv.take<float>(pad_n(N));
  cv.take<double>((size_t)T.nblk * WR_STRIDE);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  float* aX = w.take<float>(N);
  float* aY = w.take<float>(M);
  double* mom = w.take<double>(20);
  Derived* dv = w.take<Derived>(1);
  float4* ref4 = w.take<float4>(pad_n(N));
  float* lw = w.take<float>(pad_n(N));
  double* wpart = w.take<double>((size_t)T.nblk * WR_STRIDE);

  HIPCHK(launch_knn_desc(ref->x, ref->y, ref->z, N, prm->k, aX, nullptr, st));
  HIPCHK(launch_knn_desc(tmpl->x, tmpl->y, tmpl->z, M, prm->k, aY, nullptr, st));
  HIPCHK(launch_moments(ref->x, ref->y, ref->z, N, mom + 10, st));
  HIPCHK(launch_moments(tmpl->x, tmpl->y, tmpl->z, M, mom, st));
  HIPCHK(launch_prepare(aX, ref->m, N, aY, tmpl->m, M, mom, mom + 10, prep_of(prm), dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, aX, ref->m, N, dv, ref4, lw, st));

  auto loop = [&](hipStream_t s) -> int {
    for (int t = 0; t < prm->E; ++t) {
      const bool wu = stats != nullptr || t == prm->E - 1;
      ForceArgs A{tmpl->x, tmpl->y, tmpl->z, aY, tmpl->m, ref4, lw, (const double*)inout, dv, M, N,
                  T.chunk_len, T.n_chunks, t, 0.0, wpart, nullptr};
      HIPCHK(launch_force(A, T.R, pm, wu, false, s, T.sm));
      HIPCHK(launch_update(wpart, T.nblk, (const double*)inout, (double*)inout, dv, t, 0.0, 1, nullptr,
                           stats ? stats + (size_t)t * STATS_STRIDE : nullptr, s));
    }
    return SGR_OK;
  };

  const bool use_graph = (prm->flags & 1) == 0 && prm->E > 1;
  if (!use_graph) {
    if (int e = loop(st)) return e;
  } else {
    struct Key {
      const void* p[10];
      int64_t n[2];
      sgr_params prm;
      Tiles T;
      void* ws;
    } key;
    std::memset(&key, 0, sizeof(key));
    const void* ptrs[10] = {tmpl->x, tmpl->y, tmpl->z, tmpl->m, ref->x, ref->y, ref->z, ref->m, inout, stats};
    std::memcpy(key.p, ptrs, sizeof(ptrs));
    key.n[0] = M;
    key.n[1] = N;
    key.prm = *prm;
    key.T = T;
    key.ws = ctx->ws;
    std::vector<uint8_t> kb((uint8_t*)&key, (uint8_t*)&key + sizeof(key));
    if (!ctx->gc.exec || kb != ctx->gc.key) {
      if (ctx->gc.exec) (void)hipGraphExecDestroy(ctx->gc.exec);
      if (ctx->gc.graph) (void)hipGraphDestroy(ctx->gc.graph);
      ctx->gc.exec = nullptr;
      ctx->gc.graph = nullptr;
      HIPCHK(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
      int e = loop(ctx->cap);
      hipGraph_t g = nullptr;
      hipError_t ce = hipStreamEndCapture(ctx->cap, &g);
      if (e) {
        if (g) (void)hipGraphDestroy(g);
        return e;
      }
      if (ce != hipSuccess) return fail(SGR_EHIP, std::string("graph capture: ") + hipGetErrorString(ce));
      hipGraphExec_t ex = nullptr;
      hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(SGR_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ie));
      }
      ctx->gc.graph = g;
      ctx->gc.exec = ex;
      ctx->gc.key = kb;
    }
    HIPCHK(hipGraphLaunch(ctx->gc.exec, st));
  }
  int32_t status = 0;
  HIPCHK(hipMemcpyAsync(&status, &dv->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (status & ST_DEGENERATE) return fail(SGR_EDEGENERATE, "degenerate input: zero variance or zero curvature spread");
  if (status) return fail(SGR_ENUMERIC, "numeric failure in the update (status " + std::to_string(status) + ")");
  return SGR_OK;
}

int sgr_residual(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_pose* pose, const int32_t* corr,
                 double* rmse_out, sgr_stream_t stream) {
  if (!ctx || !pose || !rmse_out) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  HIPCHK(hipSetDevice(ctx->device));
  const int M = (int)tmpl->n, N = (int)ref->n;
  const int nblk = residual_blocks(M);
  Carve cv{nullptr};
  cv.take<double>((size_t)nblk * 2);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  double* part = w.take<double>((size_t)nblk * 2);
  HIPCHK(launch_residual(tmpl->x, tmpl->y, tmpl->z, M, ref->x, ref->y, ref->z, N, (const double*)pose, corr, part,
                         nblk, rmse_out, (hipStream_t)stream));
  return SGR_OK;
}

int sgr_set_tiles(sgr_ctx* ctx, int64_t M, int64_t N, double p, int R, int blocks_per_cu, int variant) {
  if (!ctx) return fail(SGR_EINVAL, "NULL ctx");
  if (M < 1 || N < 1) return fail(SGR_EINVAL, "bad sizes");
  const auto key = std::make_tuple(log2_bucket(M), log2_bucket(N), pmode_of(p));
  if (R == 0) {
    ctx->tiles.over.erase(key);
    return SGR_OK;
  }
  if (R != 1 && R != 2 && R != 4 && R != 8) return fail(SGR_EINVAL, "R must be 1, 2, 4 or 8");
  if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(SGR_EINVAL, "blocks_per_cu must be in [1, 64]");
  if (variant != 0 && variant != 1) return fail(SGR_EINVAL, "variant must be 0 (LDS) or 1 (scalar loads)");
  ctx->tiles.over[key] = std::make_tuple(R, blocks_per_cu, variant);
  return SGR_OK;
}

int sgr_force_fwd(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                  const double* mom_r, const sgr_params* prm, double G, float* f_out, double* wrench_out,
                  sgr_stream_t stream) {
  if (!ctx || !a_t || !a_r || !mom_r) return fail(SGR_EINVAL, "NULL argument");
  if (!f_out && !wrench_out) return fail(SGR_EINVAL, "nothing to compute");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  if (!(G > 0)) return fail(SGR_EINVAL, "G must be positive");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  const int pm = pmode_of(prm->p);
  const Tiles T = ctx->tiles.pick(M, N, pm);
  Carve cv{nullptr};
  cv.take<double>(16);
  cv.take<double>(16);
  cv.take<Derived>(1);
  cv.take<float4>(pad_n(N));
  cv.take<float>(pad_n(N));
  cv.take<double>((size_t)T.nblk * WR_STRIDE);
  cv.take<double>((size_t)T.n_chunks * M * 3);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  double* mom_t = w.take<double>(16);
  double* pose = w.take<double>(16);
  Derived* dv = w.take<Derived>(1);
  float4* ref4 = w.take<float4>(pad_n(N));
  float* lw = w.take<float>(pad_n(N));
  double* wpart = w.take<double>((size_t)T.nblk * WR_STRIDE);
  double* fpart = w.take<double>((size_t)T.n_chunks * M * 3);
  HIPCHK(launch_moments(tmpl->x, tmpl->y, tmpl->z, M, mom_t, st));
  HIPCHK(launch_identity_pose(pose, st));
  HIPCHK(launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_t, mom_r, prep_of(prm), dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, N, dv, ref4, lw, st));
  ForceArgs A{tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, ref4, lw, pose, dv, M, N,
              T.chunk_len, T.n_chunks, 0, G, wpart, f_out ? fpart : nullptr};
  HIPCHK(launch_force(A, T.R, pm, wrench_out != nullptr, f_out != nullptr, st, T.sm));
  if (f_out) HIPCHK(launch_reduce_f(fpart, T.n_chunks, M, f_out, st));
  if (wrench_out) HIPCHK(launch_update(wpart, T.nblk, pose, nullptr, dv, 0, G, 0, wrench_out, nullptr, st));
  return SGR_OK;
}

int sgr_force_bwd(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                  const double* mom_r, const sgr_params* prm, double G, const float* f, const float* grad_f,
                  const double* grad_wrench, float* grad_y, float* grad_m, double* grad_se, sgr_stream_t stream) {
  if (!ctx || !a_t || !a_r || !mom_r || !f || !grad_y) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  if (!(G > 0)) return fail(SGR_EINVAL, "G must be positive");
  if (grad_se && !(prm->sigma > 0)) return fail(SGR_EINVAL, "the sigma gradient needs an explicit sigma > 0");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  const int pm = pmode_of(prm->p);
  Tiles T = ctx->tiles.pick(M, N, pm);
  if (T.R > 4) T = TileTable::make(M, N, 4, 8 * ctx->n_cu);
  Carve cv{nullptr};
  cv.take<double>(16);
  cv.take<double>(16);
  cv.take<Derived>(1);
  cv.take<float4>(pad_n(N));
  cv.take<float>(pad_n(N));
  cv.take<float>((size_t)M * 3);
  cv.take<double>((size_t)T.n_chunks * M * 4);
  cv.take<double>((size_t)T.nblk * 2);
  cv.take<float>((size_t)M * 3);
  cv.take<double>(16);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  double* mom_t = w.take<double>(16);
  double* fsum = w.take<double>(16);
  Derived* dv = w.take<Derived>(1);
  float4* ref4 = w.take<float4>(pad_n(N));
  float* lw = w.take<float>(pad_n(N));
  float* lam = w.take<float>((size_t)M * 3);
  double* ypart = w.take<double>((size_t)T.n_chunks * M * 4);
  double* spart = w.take<double>((size_t)T.nblk * 2);
  float* gf0 = w.take<float>((size_t)M * 3);
  double* gw0 = w.take<double>(16);
  if (!grad_f) HIPCHK(launch_fill_f(gf0, (int64_t)M * 3, 0.f, st));
  if (!grad_wrench) HIPCHK(launch_fill(gw0, 16, 0.0, st));
  HIPCHK(launch_moments(tmpl->x, tmpl->y, tmpl->z, M, mom_t, st));
  HIPCHK(launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_t, mom_r, prep_of(prm), dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, N, dv, ref4, lw, st));
  AdjArgs A{tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, ref4, lw, dv, M, N, T.chunk_len, T.n_chunks, T.nblk,
            pm == 1, G, f, grad_f ? grad_f : gf0, grad_wrench ? grad_wrench : gw0, lam, ypart, spart,
            grad_y, grad_m, grad_se};
  HIPCHK(launch_adjoint(A, T.R, fsum, st));
  return SGR_OK;
}

struct sgr_plan {
  sgr_ctx* ctx = nullptr;
  sgr_cloud tmpl{}, ref{};
  const float* a_t = nullptr;
  sgr_params prm{};
  Tiles T{};
  int pm = 1;
  char* mem = nullptr;
  Derived* dv = nullptr;
  float4* ref4 = nullptr;
  float* lw = nullptr;
  double* wpart = nullptr;
  double* fpart = nullptr;
};

int sgr_plan_create(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                    const double* mom_t, const double* mom_r, const sgr_params* prm, sgr_plan** out,
                    sgr_stream_t stream) {
  if (!ctx || !out || !a_t || !a_r || !mom_t || !mom_r) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  HIPCHK(hipSetDevice(ctx->device));
  const int M = (int)tmpl->n, N = (int)ref->n;
  sgr_plan* pl = new sgr_plan();
  pl->ctx = ctx;
  pl->tmpl = *tmpl;
  pl->ref = *ref;
  pl->a_t = a_t;
  pl->prm = *prm;
  pl->pm = pmode_of(prm->p);
  pl->T = ctx->tiles.pick(M, N, pl->pm);
  Carve cv{nullptr};
  cv.take<Derived>(1);
  cv.take<float4>(pad_n(N));
  cv.take<float>(pad_n(N));
  cv.take<double>((size_t)pl->T.nblk * WR_STRIDE);
  cv.take<double>((size_t)pl->T.n_chunks * M * 3);
  if (hipMalloc(&pl->mem, cv.off) != hipSuccess) {
    (void)hipGetLastError();
    delete pl;
    return fail(SGR_ENOMEM, "plan allocation failed");
  }
  Carve w{pl->mem};
  pl->dv = w.take<Derived>(1);
  pl->ref4 = w.take<float4>(pad_n(N));
  pl->lw = w.take<float>(pad_n(N));
  pl->wpart = w.take<double>((size_t)pl->T.nblk * WR_STRIDE);
  pl->fpart = w.take<double>((size_t)pl->T.n_chunks * M * 3);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e1 = launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_t, mom_r, prep_of(prm), pl->dv, st);
  hipError_t e2 = e1 == hipSuccess ? launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, N, pl->dv, pl->ref4, pl->lw, st)
                                   : e1;
  if (e2 != hipSuccess) {
    (void)hipFree(pl->mem);
    delete pl;
    return fail(SGR_EHIP, std::string("plan set-up: ") + hipGetErrorString(e2));
  }
  *out = pl;
  return SGR_OK;
}

int sgr_plan_destroy(sgr_plan* pl) {
  if (!pl) return SGR_OK;
  (void)hipSetDevice(pl->ctx->device);
  (void)hipDeviceSynchronize();
  if (pl->mem) (void)hipFree(pl->mem);
  delete pl;
  return SGR_OK;
}

static ForceArgs plan_args(sgr_plan* pl, int t, double G, const sgr_pose* pose, bool with_f) {
  return ForceArgs{pl->tmpl.x, pl->tmpl.y, pl->tmpl.z, pl->a_t, pl->tmpl.m, pl->ref4, pl->lw,
                   (const double*)pose, pl->dv, (int)pl->tmpl.n, (int)pl->ref.n, pl->T.chunk_len, pl->T.n_chunks,
                   t, G, pl->wpart, with_f ? pl->fpart : nullptr};
}

int sgr_plan_force(sgr_plan* pl, int t, double G, const sgr_pose* pose, double* wrench_out, float* f_out,
                   sgr_stream_t stream) {
  if (!pl || !pose) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(pl->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ForceArgs A = plan_args(pl, t, G, pose, f_out != nullptr);
  HIPCHK(launch_force(A, pl->T.R, pl->pm, wrench_out != nullptr, f_out != nullptr, st, pl->T.sm));
  if (f_out) HIPCHK(launch_reduce_f(pl->fpart, pl->T.n_chunks, (int)pl->tmpl.n, f_out, st));
  if (wrench_out)
    HIPCHK(launch_update(pl->wpart, pl->T.nblk, (const double*)pose, nullptr, pl->dv, t, G, 0, wrench_out, nullptr,
                         st));
  return SGR_OK;
}

int sgr_plan_step(sgr_plan* pl, int t, const sgr_pose* pose_in, sgr_pose* pose_out, double* wrench_out,
                  sgr_stream_t stream) {
  if (!pl || !pose_in || !pose_out) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(pl->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ForceArgs A = plan_args(pl, t, 0.0, pose_in, false);
  HIPCHK(launch_force(A, pl->T.R, pl->pm, wrench_out != nullptr, false, st, pl->T.sm));
  HIPCHK(launch_update(pl->wpart, pl->T.nblk, (const double*)pose_in, (double*)pose_out, pl->dv, t, 0.0, 1,
                       wrench_out, nullptr, st));
  return SGR_OK;
}

}  // extern "C"
