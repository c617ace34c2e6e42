// C-ABI layer: argument checks, workspace, tile selection, graph capture of
// the iteration loop.  Every numeric step is a HIP kernel; this file only
// sequences launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
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
  std::string arch;
  hipStream_t cap = nullptr;
  char* ws = nullptr;
  size_t ws_size = 0;
  GraphCache gc;   // single registration
  GraphCache gcb;  // batch / multi-start
  std::vector<GraphCache> gcp;  // pyramidal schedule, one per level
  GraphCache gcv;  // vector descriptors
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

constexpr int FLAG_PINV = 8;

// allow_pinv: the caller (sgr_register, sgr_register_pyramid,
// sgr_register_batch, sgr_multistart, sgr_register_vec) runs an iteration
// loop: it implements flags bit 3 (the pose-independent pair sums of the
// p = 1 law) and a velocity state (momentum).
int check_params(const sgr_params* p, bool allow_pinv = false) {
  if (!p) return fail(SGR_EINVAL, "NULL params");
  if (!std::isfinite(p->p)) return fail(SGR_EINVAL, "p must be finite");
  if (p->p < 1.0 && !(p->eps > 0)) return fail(SGR_EINVAL, "p < 1 needs eps > 0 (the force would diverge at r = 0)");
  if (p->p == -1.0) return fail(SGR_EINVAL, "p = -1 has a logarithmic potential; the energy U is defined for p != -1");
  if (p->g_mode < 0 || p->g_mode > 2)
    return fail(SGR_EINVAL, "g_mode must be 0 (g = s), 1 (g = a a s) or 2 (g = 1, masses only)");
  if (!(p->G1 > 0) || !std::isfinite(p->G1)) return fail(SGR_EINVAL, "G1 must be positive");
  if (p->flags & ~15) return fail(SGR_EINVAL, "unknown flag bits");
  if (p->flags & FLAG_PINV) {
    if (!allow_pinv)
      return fail(SGR_EINVAL, "flags bit 3 applies to sgr_register, sgr_register_pyramid, sgr_register_batch, "
                              "sgr_multistart and sgr_register_vec only");
    if (p->p != 1.0 || p->g_mode > 1 || (p->flags & 2))
      return fail(SGR_EINVAL, "flags bit 3 needs p = 1, g_mode 0 or 1 and no mixed precision");
  }
  if (!std::isfinite(p->sigma) || !std::isfinite(p->eps) || p->eps < 0) return fail(SGR_EINVAL, "bad sigma/eps");
  if (!std::isfinite(p->dt2)) return fail(SGR_EINVAL, "bad dt2");
  if (!(p->momentum >= 0.0 && p->momentum < 1.0)) return fail(SGR_EINVAL, "momentum must be in [0, 1)");
  if (p->momentum != 0.0 && !allow_pinv)
    return fail(SGR_EINVAL, "a velocity state (momentum != 0) needs an iteration loop: sgr_register, "
                            "sgr_register_pyramid, sgr_register_batch, sgr_multistart or sgr_register_vec");
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
  P.momentum = p->momentum;
  return P;
}

int pmode_of(double p) { return p == 1.0 ? 1 : (p == 3.0 ? 3 : 0); }

constexpr int FLAG_NO_GRAPH = 1;
constexpr int FLAG_MIXED = 2;
constexpr int FLAG_VEC_FP32 = 4;

bool is_mixed(const sgr_params* p) { return (p->flags & FLAG_MIXED) != 0; }

int check_mixed(const sgr_params* p) {
  if (is_mixed(p) && p->p != 1.0) return fail(SGR_EINVAL, "the mixed-precision force is implemented for p = 1 only");
  return SGR_OK;
}

// Tiles for a call: the mixed kernel has a fixed 256-point template block.
// Its launch targets 8 blocks per CU, and up to 24 while every block keeps
// at least 4e6 pairs: more rounds of shorter chunks even out the end of a
// large launch, but on a small pair each block's fixed start and end would
// dominate (the scene, 7.7e10 pairs: 8.08 ms at 24 blocks per CU against
// 8.55 at 8; the scan pair, 1.2e9 pairs: 0.145 ms at 8 against 0.164 at 24).
Tiles tiles_for(const sgr_ctx* ctx, int M, int N, const sgr_params* p) {
  if (is_mixed(p)) {
    const int64_t lo = int64_t(8) * ctx->n_cu, hi = int64_t(24) * ctx->n_cu;
    const int64_t tb = std::min(hi, std::max(lo, (int64_t)M * N / 4000000));
    return TileTable::make(M, N, 1, (int)tb);
  }
  return ctx->tiles.pick(M, N, pmode_of(p->p));
}

// Shape of one FP32 force launch for a single registration: every template
// block gets n_chunks reference chunks cut at multiples of force_chunk_gran()
// points, with n_chunks chosen so that the launch is about T.bpc blocks per
// CU (by default one wave of resident blocks, from the kernel's occupancy).
// Whole-tile chunks would leave the last wave of blocks partly empty
// whenever the work is not a multiple of the resident block count, and a
// small pair (a few thousand points) would occupy a few CUs only.
// `slots` is the number of wrench slots the launch writes.
struct FLaunch {
  int n_chunks = 0, slots = 0;
};

FLaunch force_shape(const sgr_ctx* ctx, int M, int N, const Tiles& T, int pm) {
  const int64_t n_iblk = (M + 256 * T.R - 1) / (256 * T.R);
  const int64_t n_sub = (N + force_chunk_gran() - 1) / force_chunk_gran();  // smallest chunks
  const int bpc = T.bpc > 0 ? T.bpc : force_blocks_per_cu(T.R, pm, T.sm != 0);
  const int64_t nc = std::max<int64_t>(1, std::min<int64_t>(n_sub, (int64_t)bpc * ctx->n_cu / n_iblk));
  FLaunch L;
  L.n_chunks = (int)nc;
  L.slots = (int)(n_iblk * nc);
  return L;
}

// Launch shape of the adjoint pair kernel: R template points per lane from
// the tile choice (at most 4), n_chunks balanced reference chunks for about
// two blocks per CU (fewer for a small pair: chunks of at least 16 points).
// Every chunk writes 32 bytes per template point of partial sums, so more,
// shorter chunks cost traffic as well as per-block overhead.
Tiles adj_shape(const sgr_ctx* ctx, int M, int N, int R, bool p1) {
  (void)p1;
  if (R > 4) R = 4;
  Tiles T{};
  T.R = R;
  T.n_iblk = (M + 256 * R - 1) / (256 * R);
  const int64_t n_sub = (N + adj_chunk_gran() - 1) / adj_chunk_gran();
  const int64_t nc = std::max<int64_t>(1, std::min<int64_t>(n_sub, (int64_t)2 * ctx->n_cu / T.n_iblk));
  T.n_chunks = (int)nc;
  T.chunk_len = 0;
  T.nblk = T.n_iblk * T.n_chunks;
  return T;
}

hipError_t run_force(ForceArgs A, const Tiles& T, const FLaunch& L, int pm, bool wu, bool wf, hipStream_t st) {
  A.chunk_len = 0;
  A.n_chunks = L.n_chunks;
  return launch_force(A, T.R, pm, wu, wf, st, T.sm != 0);
}

// The packed reference is padded to whole tiles with zero-weight points.
size_t pad_n(int64_t N) { return (size_t)((N + 255) / 256) * 256; }

// Capture `loop` (which launches on the given stream) into the cache unless
// the cached graph was made for the same key, then launch it on `st`.
template <class F>
int run_graph(sgr_ctx* ctx, GraphCache& gc, const std::vector<uint8_t>& key, F&& loop, hipStream_t st) {
  if (!gc.exec || key != gc.key) {
    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
    if (gc.graph) (void)hipGraphDestroy(gc.graph);
    gc.exec = nullptr;
    gc.graph = nullptr;
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
    gc.graph = g;
    gc.exec = ex;
    gc.key = key;
  }
  HIPCHK(hipGraphLaunch(gc.exec, st));
  return SGR_OK;
}

template <class T>
void key_add(std::vector<uint8_t>& k, const T* p, size_t n) {
  const uint8_t* b = reinterpret_cast<const uint8_t*>(p);
  k.insert(k.end(), b, b + n * sizeof(T));
}

// Batch of registrations sharing parameters: host tables, device copies,
// descriptors, set-up, then E iterations of (persistent force, update).
struct BatchIn {
  int B;
  std::vector<const sgr_cloud*> tm, rf;  // per registration
  std::vector<int> tm_cloud, rf_cloud;   // index of each registration's clouds in `clouds`
  std::vector<const sgr_cloud*> clouds;  // distinct clouds (descriptors computed once each)
  std::vector<int> pack_of;              // registration whose reference packing it uses (itself, or shared)
};

int run_batch(sgr_ctx* ctx, const BatchIn& in, const sgr_params* prm, double* poses, const double* R0_multistart,
              double* energy_out, double* stats, int32_t* best_out, hipStream_t st) {
  const int B = in.B;
  const int pm = pmode_of(prm->p);
  const int ncl = (int)in.clouds.size();
  // launch shape: R from the tile table at the median registration size
  std::vector<int64_t> Ms(B), Ns(B);
  for (int r = 0; r < B; ++r) {
    Ms[r] = in.tm[r]->n;
    Ns[r] = in.rf[r]->n;
  }
  std::vector<int64_t> sm = Ms, sn = Ns;
  std::nth_element(sm.begin(), sm.begin() + B / 2, sm.end());
  std::nth_element(sn.begin(), sn.begin() + B / 2, sn.end());
  int R = ctx->tiles.pick((int)sm[B / 2], (int)sn[B / 2], pm).R;
  if (R > 4) R = 4;
  const int chunk_len = 2048;
  const int ipb = 256 * R;

  // host tables
  std::vector<CloudDesc> cds(ncl);
  std::vector<int64_t> a_off(ncl + 1, 0);
  std::vector<int2> kblocks;
  for (int c = 0; c < ncl; ++c) {
    a_off[c + 1] = a_off[c] + (int64_t)pad_n(in.clouds[c]->n);
    for (int b = 0; b < (int)((in.clouds[c]->n + 255) / 256); ++b) kblocks.push_back(make_int2(c, b));
  }
  std::vector<int64_t> ref_off(B, 0);
  std::vector<int> blk2reg;
  std::vector<int> blk0(B, 0);
  int64_t ref_total = 0;
  for (int r = 0; r < B; ++r) {
    if (in.pack_of[r] != r) continue;
    ref_off[r] = ref_total;
    blk0[r] = (int)blk2reg.size();
    const int nb = (int)((Ns[r] + 255) / 256);
    for (int b = 0; b < nb; ++b) blk2reg.push_back(r);
    ref_total += (int64_t)nb * 256;
  }
  for (int r = 0; r < B; ++r) ref_off[r] = ref_off[in.pack_of[r]];
  std::vector<RegDesc> regs(B);
  std::vector<int4> items;
  int slot = 0;
  for (int r = 0; r < B; ++r) {
    const int nib = (int)((Ms[r] + ipb - 1) / ipb), nch = (int)((Ns[r] + chunk_len - 1) / chunk_len);
    regs[r].wslot0 = slot;
    regs[r].n_items = nib * nch;
    for (int ib = 0; ib < nib; ++ib)
      for (int ch = 0; ch < nch; ++ch) items.push_back(make_int4(r, ib, ch, slot + ib * nch + ch));
    slot += nib * nch;
  }
  auto cost = [&](const int4& it) {
    const int64_t mi = std::min<int64_t>(ipb, Ms[it.x] - (int64_t)it.y * ipb);
    const int64_t nj = std::min<int64_t>(chunk_len, Ns[it.x] - (int64_t)it.z * chunk_len);
    return mi * nj;
  };
  std::stable_sort(items.begin(), items.end(), [&](const int4& a, const int4& b) { return cost(a) > cost(b); });
  const int n_items = (int)items.size();
  // flags bit 3 (p = 1): pair sums once, then one wrench slot per block of
  // 256 template points in every iteration, described by regs_p
  const bool pinv = (prm->flags & FLAG_PINV) != 0;
  std::vector<int2> tblk;
  std::vector<int> pslot0(B, 0), pslots(B, 0);
  if (pinv)
    for (int r = 0; r < B; ++r) {
      pslot0[r] = (int)tblk.size();
      pslots[r] = pinv_blocks((int)Ms[r]);
      for (int b = 0; b < pslots[r]; ++b) tblk.push_back(make_int2(r, b));
    }
  const int n_tblk = (int)tblk.size();
  const int n_slots = std::max(n_items, n_tblk);

  // workspace
  Carve cv{nullptr};
  cv.take<CloudDesc>(ncl);
  cv.take<int2>(kblocks.size());
  cv.take<PrepDesc>(B);
  cv.take<int>(blk2reg.size());
  cv.take<RegDesc>(B);
  cv.take<int4>(n_items);
  cv.take<float>(a_off[ncl]);
  cv.take<double>((size_t)ncl * 10);
  cv.take<Derived>(B);
  cv.take<float4>(ref_total);
  cv.take<float>(ref_total);
  cv.take<double>((size_t)n_slots * WR_STRIDE);
  cv.take<double>(B);
  int64_t perm_total = 0;
  for (int r = 0; r < B; ++r) perm_total += Ms[r];
  cv.take<int>(perm_total);
  cv.take<float4>(perm_total);
  cv.take<float2>(perm_total);
  cv.take<int>(B + 1);
  cv.take<char>(sort_perm_workspace(perm_total, B));
  if (pinv) {
    cv.take<int2>(n_tblk);
    cv.take<RegDesc>(B);
    cv.take<double>((size_t)perm_total * 5);
  }
  std::vector<int> cl_n(ncl);
  for (int c = 0; c < ncl; ++c) cl_n[c] = (int)in.clouds[c]->n;
  const size_t gws_bytes = grid_knn_batch_workspace(cl_n.data(), ncl, prm->k);
  cv.take<char>(gws_bytes);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  CloudDesc* d_cds = w.take<CloudDesc>(ncl);
  int2* d_kb = w.take<int2>(kblocks.size());
  PrepDesc* d_prep = w.take<PrepDesc>(B);
  int* d_b2r = w.take<int>(blk2reg.size());
  RegDesc* d_regs = w.take<RegDesc>(B);
  int4* d_items = w.take<int4>(n_items);
  float* d_a = w.take<float>(a_off[ncl]);
  double* d_mom = w.take<double>((size_t)ncl * 10);
  Derived* d_dv = w.take<Derived>(B);
  float4* d_ref4 = w.take<float4>(ref_total);
  float* d_lw = w.take<float>(ref_total);
  double* d_wpart = w.take<double>((size_t)n_slots * WR_STRIDE);
  double* d_energy = w.take<double>(B);
  int* d_perm = w.take<int>(perm_total);
  float4* d_tm4 = w.take<float4>(perm_total);
  float2* d_tmx = w.take<float2>(perm_total);
  int* d_poff = w.take<int>(B + 1);
  char* d_sws = w.take<char>(sort_perm_workspace(perm_total, B));
  int2* d_tblk = pinv ? w.take<int2>(n_tblk) : nullptr;
  RegDesc* d_regs_p = pinv ? w.take<RegDesc>(B) : nullptr;
  double* d_S = pinv ? w.take<double>((size_t)perm_total * 5) : nullptr;
  char* d_gws = w.take<char>(gws_bytes);

  for (int c = 0; c < ncl; ++c)
    cds[c] = CloudDesc{in.clouds[c]->x, in.clouds[c]->y, in.clouds[c]->z, d_a + a_off[c], (int)in.clouds[c]->n, 0};
  std::vector<PrepDesc> preps(B);
  for (int r = 0; r < B; ++r) {
    const int ct = in.tm_cloud[r], cr = in.rf_cloud[r];
    preps[r] = PrepDesc{in.rf[r]->x, in.rf[r]->y, in.rf[r]->z, d_a + a_off[cr], in.rf[r]->m, d_a + a_off[ct],
                        in.tm[r]->m, d_mom + 10 * ct, d_mom + 10 * cr, ref_off[r], (int)Ns[r], (int)Ms[r], blk0[r], 0};
    regs[r].y0x = in.tm[r]->x;
    regs[r].y0y = in.tm[r]->y;
    regs[r].y0z = in.tm[r]->z;
    regs[r].aY = d_a + a_off[ct];
    regs[r].mY = in.tm[r]->m;
    regs[r].ref_off = ref_off[r];
    regs[r].M = (int)Ms[r];
    regs[r].N = (int)Ns[r];
  }
  std::vector<int> poff(B + 1, 0);
  for (int r = 0; r < B; ++r) {
    regs[r].perm = d_perm + poff[r];
    regs[r].tm4 = d_tm4 + poff[r];
    regs[r].tmx = d_tmx + poff[r];
    poff[r + 1] = poff[r] + (int)Ms[r];
  }
  HIPCHK(hipMemcpyAsync(d_cds, cds.data(), sizeof(CloudDesc) * ncl, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_kb, kblocks.data(), sizeof(int2) * kblocks.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_prep, preps.data(), sizeof(PrepDesc) * B, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_b2r, blk2reg.data(), sizeof(int) * blk2reg.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_regs, regs.data(), sizeof(RegDesc) * B, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_items, items.data(), sizeof(int4) * n_items, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_poff, poff.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, st));
  std::vector<RegDesc> regs_p;
  if (pinv) {
    regs_p = regs;
    for (int r = 0; r < B; ++r) {
      regs_p[r].wslot0 = pslot0[r];
      regs_p[r].n_items = pslots[r];
    }
    HIPCHK(hipMemcpyAsync(d_tblk, tblk.data(), sizeof(int2) * n_tblk, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_regs_p, regs_p.data(), sizeof(RegDesc) * B, hipMemcpyHostToDevice, st));
  }

  // descriptors of every cloud: the exact grid search for all clouds at
  // once, one launch per phase (a grid search per cloud would be a long
  // chain of small launches, brute force n^2 work per cloud)
  {
    std::vector<const float*> cx(ncl), cy(ncl), cz(ncl);
    std::vector<float*> ca(ncl);
    for (int c = 0; c < ncl; ++c) {
      cx[c] = in.clouds[c]->x;
      cy[c] = in.clouds[c]->y;
      cz[c] = in.clouds[c]->z;
      ca[c] = d_a + a_off[c];
    }
    HIPCHK(launch_grid_knn_batch(cx.data(), cy.data(), cz.data(), cl_n.data(), ca.data(), nullptr, ncl, prm->k,
                                 d_gws, st));
  }
  HIPCHK(launch_moments_batch(d_cds, ncl, d_mom, st));
  HIPCHK(launch_prepare_batch(d_prep, B, prep_of(prm), d_dv, st));
  HIPCHK(launch_pack_batch(d_prep, d_b2r, (int)blk2reg.size(), d_dv, d_ref4, d_lw, st));
  {
    const int max_M = (int)*std::max_element(Ms.begin(), Ms.end());
    HIPCHK(launch_sort_perm_batch(d_regs, B, d_poff, perm_total, max_M, d_perm, d_sws, st));
    HIPCHK(launch_pack_tmpl_batch(d_regs, B, max_M, d_dv, st));
  }
  if (pinv) HIPCHK(launch_psum_batch(d_regs, d_tblk, n_tblk, d_poff, d_ref4, d_lw, d_S, st));
  if (R0_multistart) HIPCHK(launch_init_multistart(R0_multistart, B, d_mom + 10 * in.tm_cloud[0], poses, st));

  // One block per work item: the hardware hands the items out in the list's
  // decreasing-cost order as blocks finish.  A persistent grid of 8 blocks
  // per CU striding over the list was 6 % slower on the 256-registration
  // batch (1.43 s against 1.34 s; 4 blocks per CU, 1.55 s): with more blocks
  // than are resident, the second round starts only as whole item lists end.
  const int grid = n_items;
  auto loop = [&](hipStream_t s) -> int {
    for (int t = 0; t < prm->E; ++t) {
      const bool wu = stats != nullptr || t == prm->E - 1;
      if (pinv) {
        HIPCHK(launch_pinv_batch(d_regs_p, d_tblk, n_tblk, d_poff, d_S, poses, d_dv, t, wu, d_wpart, s));
      } else {
        BatchArgs A{d_regs, d_items, n_items, d_ref4, d_lw, poses, d_dv, chunk_len, t, d_wpart};
        HIPCHK(launch_force_batch(A, R, pm, wu, grid, s));
      }
      HIPCHK(launch_update_batch(d_wpart, pinv ? d_regs_p : d_regs, B, poses, d_dv, t, 1,
                                 t == prm->E - 1 ? d_energy : nullptr, stats, prm->E, s));
    }
    return SGR_OK;
  };
  if ((prm->flags & 1) || prm->E < 2) {
    if (int e = loop(st)) return e;
  } else {
    std::vector<uint8_t> key;
    key_add(key, &B, 1);
    key_add(key, prm, 1);
    key_add(key, items.data(), items.size());
    key_add(key, regs.data(), regs.size());
    const void* ptrs[4] = {ctx->ws, poses, stats, R0_multistart};
    key_add(key, ptrs, 4);
    if (int e = run_graph(ctx, ctx->gcb, key, loop, st)) return e;
  }
  if (energy_out) HIPCHK(hipMemcpyAsync(energy_out, d_energy, sizeof(double) * B, hipMemcpyDeviceToDevice, st));
  if (best_out) HIPCHK(launch_argmin(d_energy, B, best_out, st));
  std::vector<Derived> dh(B);
  HIPCHK(hipMemcpyAsync(dh.data(), d_dv, sizeof(Derived) * B, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int bad = 0, degen = 0;
  for (int r = 0; r < B; ++r) {
    bad += dh[r].status != 0;
    degen += (dh[r].status & ST_DEGENERATE) != 0;
  }
  if (degen) return fail(SGR_EDEGENERATE, std::to_string(degen) + " registration(s) with degenerate input");
  if (bad) return fail(SGR_ENUMERIC, std::to_string(bad) + " registration(s) hit a numeric failure");
  return SGR_OK;
}


// ------------------------------------------------- single registration
// Device buffers of one registration (curvatures, moments of both clouds,
// derived constants, packed reference and template, wrench slots, search and
// sort scratch), carved from the context workspace.
struct SingleWs {
  float* aX;
  float* aY;
  double* mom;  // template [0, 10), reference [10, 20)
  Derived* dv;
  float4* ref4;
  float* lw;
  double* wpart;
  char* gws;
  double* ps_part;  // pose-independent pair sums (flags bit 3): per chunk, then reduced
  double* ps_S;
  int ps_chunks;
  int* perm;
  char* sws;
  float4* tm4;
  float2* tmx;
  Tiles T, TM;  // FP32 kernel; kernel of the mixed-precision iterations
  int nslot;
};

// kmax: largest k of a nearest-neighbour search the call makes (0: none).
int carve_single(sgr_ctx* ctx, int M, int N, const sgr_params* prm, int kmax, SingleWs& w, bool radius) {
  const int pm = pmode_of(prm->p);
  const bool pinv = (prm->flags & FLAG_PINV) != 0;
  w.T = ctx->tiles.pick(M, N, pm);
  w.TM = tiles_for(ctx, M, N, prm);
  w.nslot = std::max(force_shape(ctx, M, N, w.T, pm).slots, w.TM.nblk);
  if (pinv) w.nslot = std::max(w.nslot, pinv_blocks(M));
  w.ps_chunks = pinv ? pinv_chunks(M, N, ctx->n_cu) : 0;
  size_t gbytes = kmax > 0 ? std::max(grid_knn_workspace(N, kmax), grid_knn_workspace(M, kmax)) : 0;
  if (radius) gbytes = std::max({gbytes, radius_desc_workspace(N), radius_desc_workspace(M)});
  for (int pass = 0; pass < 2; ++pass) {
    Carve c{pass ? ctx->ws : nullptr};
    w.aX = c.take<float>(N);
    w.aY = c.take<float>(M);
    w.mom = c.take<double>(20);
    w.dv = c.take<Derived>(1);
    w.ref4 = c.take<float4>(pad_n(N));
    w.lw = c.take<float>(pad_n(N));
    w.wpart = c.take<double>((size_t)w.nslot * WR_STRIDE);
    w.gws = c.take<char>(gbytes);
    w.perm = c.take<int>(M);
    w.sws = c.take<char>(sort_perm_workspace(M, 1));
    w.tm4 = c.take<float4>(M);
    w.tmx = c.take<float2>(M);
    w.ps_part = pinv ? c.take<double>((size_t)w.ps_chunks * M * 5) : nullptr;
    w.ps_S = pinv ? c.take<double>((size_t)M * 5) : nullptr;
    if (!pass)
      if (int e = ensure_ws(ctx, c.off)) return e;
  }
  return SGR_OK;
}

// Derived constants from the curvatures and moments already in w, then the
// packed reference and the curvature-sorted packed template.
int setup_single(const sgr_cloud* tmpl, const sgr_cloud* ref, const PrepParams& P, SingleWs& w, hipStream_t st) {
  const int M = (int)tmpl->n, N = (int)ref->n;
  HIPCHK(launch_prepare(w.aX, ref->m, N, w.aY, tmpl->m, M, w.mom, w.mom + 10, P, w.dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, w.aX, ref->m, N, w.dv, w.ref4, w.lw, st));
  HIPCHK(launch_sort_perm(w.aY, M, w.perm, w.sws, st));
  HIPCHK(launch_pack_tmpl(tmpl->x, tmpl->y, tmpl->z, w.aY, tmpl->m, M, w.perm, w.dv, w.tm4, w.tmx, st));
  if (w.ps_S) HIPCHK(launch_psum(w.tm4, M, w.ref4, w.lw, N, w.ps_chunks, w.ps_part, w.ps_S, st));
  return SGR_OK;
}

// Iterations [t0, t1) of (force, update) on the pose in place, captured in a
// graph cached in gc unless FLAG_NO_GRAPH is set or there is one iteration.
// G follows eq. 12 over prm->E.  The energy U is accumulated only where it is
// read, in the per-iteration stats; with stats, the last of the E
// iterations of a mixed-precision registration uses the FP32 kernel so that
// its energy is the FP32 one.
int run_single_loop(sgr_ctx* ctx, GraphCache& gc, const sgr_cloud* tmpl, const sgr_cloud* ref,
                    const sgr_params* prm, const SingleWs& w, sgr_pose* inout, double* stats, int t0, int t1,
                    hipStream_t st) {
  const int M = (int)tmpl->n, N = (int)ref->n;
  const int pm = pmode_of(prm->p);
  auto loop = [&](hipStream_t s) -> int {
    for (int t = t0; t < t1; ++t) {
      const bool last = t == prm->E - 1;
      const bool mixed = is_mixed(prm) && !(last && stats != nullptr);
      const bool wu = !mixed && stats != nullptr;
      const Tiles& Tt = mixed ? w.TM : w.T;
      ForceArgs A{tmpl->x, tmpl->y, tmpl->z, w.aY, tmpl->m, w.ref4, w.lw, (const double*)inout, w.dv, M, N,
                  Tt.chunk_len, Tt.n_chunks, t, 0.0, w.wpart, nullptr, w.perm, w.tm4, w.tmx};
      int used = Tt.nblk;
      if (w.ps_S) {
        // p = 1 with the pair sums formed once by setup_single: O(M) per iteration
        HIPCHK(launch_pinv(w.tm4, w.tmx, w.ps_S, M, (const double*)inout, w.dv, t, wu, w.wpart, s));
        used = pinv_blocks(M);
      } else if (mixed) {
        HIPCHK(launch_force_mixed(A, false, s));
      } else {
        const FLaunch L = force_shape(ctx, M, N, w.T, pm);
        HIPCHK(run_force(A, w.T, L, pm, wu, false, s));
        used = L.slots;
      }
      HIPCHK(launch_update(w.wpart, used, (const double*)inout, (double*)inout, w.dv, t, 0.0, 1, nullptr,
                           stats ? stats + (size_t)t * STATS_STRIDE : nullptr, s));
    }
    return SGR_OK;
  };
  if ((prm->flags & FLAG_NO_GRAPH) || t1 - t0 < 2) return loop(st);
  // The captured kernels read every buffer below at a fixed address, so the
  // key holds all of them: the workspace layout depends on more than the
  // clouds and parameters (the neighbour search's k, radius levels).
  struct Key {
    const void* p[10];
    const void* wsp[11];
    int64_t n[2];
    int32_t t[2];
    sgr_params prm;
    Tiles T, TM;
  } key;
  std::memset(&key, 0, sizeof(key));
  const void* ptrs[10] = {tmpl->x, tmpl->y, tmpl->z, tmpl->m, ref->x, ref->y, ref->z, ref->m, inout, stats};
  std::memcpy(key.p, ptrs, sizeof(ptrs));
  const void* wptrs[11] = {w.aY, w.dv, w.ref4, w.lw, w.wpart, w.perm, w.tm4, w.tmx, w.ps_S, w.aX, w.mom};
  std::memcpy(key.wsp, wptrs, sizeof(wptrs));
  key.n[0] = M;
  key.n[1] = N;
  key.t[0] = t0;
  key.t[1] = t1;
  key.prm = *prm;
  key.T = w.T;
  key.TM = w.TM;
  std::vector<uint8_t> kb((uint8_t*)&key, (uint8_t*)&key + sizeof(key));
  return run_graph(ctx, gc, kb, loop, st);
}

// ------------------------------------------------- vector descriptors
int check_vec(const sgr_params* p, int D) {
  if (D < 1 || D > 30) return fail(SGR_EINVAL, "vector descriptors need 1 <= D <= 30");
  if (p->p != 1.0) return fail(SGR_EINVAL, "the vector-descriptor force is implemented for p = 1");
  if (p->g_mode != 0) return fail(SGR_EINVAL, "the vector-descriptor force uses g = s (g_mode 0)");
  if (is_mixed(p)) return fail(SGR_EINVAL, "the vector-descriptor force has no mixed-precision form");
  return SGR_OK;
}

// Device buffers of the vector-descriptor force: set-up constants,
// augmented rows, reference coordinates, wrench slots, per-chunk forces.
struct VecWs {
  Derived* dv;
  double* vd;
  float* At;
  float* Bt;
  float4* ref4;
  double* wpart;
  double* fpart;
  double* mom;
  int K, n_chunks, slots;
  int n_cu;   // compute units (the far-row grid is one round of blocks)
  bool half;  // split-f16 products (decided by setup_vec)
  int* far_idx;  // far template rows (M + 1 ints: the list, then its length)
  int n_far;     // number of far rows (read back by setup_vec)
  double* far_ref;   // reference records of the far-row evaluation
  double* far_part;  // its per-segment sums
  // flags bit 3: the template in its own order, the pair sums per chunk, reduced
  float4* tm4 = nullptr;
  float2* tmx = nullptr;
  double* ps_part = nullptr;
  double* ps_S = nullptr;
};

int carve_vec(sgr_ctx* ctx, int M, int N, int D, bool with_f, bool with_mom, VecWs& w, bool pinv = false) {
  w.K = vforce_K(D);
  w.n_cu = ctx->n_cu;
  w.n_chunks = vforce_chunks(M, N, ctx->n_cu);
  w.slots = vforce_n_iblk(M) * w.n_chunks;
  // every template row may be a far row, with a wrench slot of its own
  const int wslots = pinv ? std::max(w.slots + M, pinv_blocks(M)) : w.slots + M;
  for (int pass = 0; pass < 2; ++pass) {
    Carve c{pass ? ctx->ws : nullptr};
    w.dv = c.take<Derived>(1);
    w.vd = c.take<double>(36);
    // rows of K floats (FP32 form) or vforce_half_K(D) halves (split f16)
    const size_t row_words = (size_t)std::max(w.K, vforce_half_K(D) / 2);
    w.At = c.take<float>((size_t)vforce_pad_rows(M) * row_words);
    w.Bt = c.take<float>((size_t)vforce_pad_refs(N) * row_words);
    w.ref4 = c.take<float4>((size_t)vforce_pad_refs(N));
    w.wpart = c.take<double>((size_t)wslots * WR_STRIDE);
    w.fpart = with_f ? c.take<double>((size_t)w.n_chunks * M * 3) : nullptr;
    w.mom = with_mom ? c.take<double>(20) : nullptr;
    w.far_idx = c.take<int>((size_t)M + 1);
    w.far_ref = c.take<double>((size_t)vfar_pad_refs(N) * vfar_stride(D));
    w.far_part = c.take<double>(vfar_part_doubles(M));
    if (pinv) {
      w.tm4 = c.take<float4>(M);
      w.tmx = c.take<float2>(M);
      w.ps_part = c.take<double>((size_t)w.n_chunks * M * 5);
      w.ps_S = c.take<double>((size_t)M * 5);
    }
    if (!pass)
      if (int e = ensure_ws(ctx, c.off)) return e;
  }
  return SGR_OK;
}

// Set-up of the vector-descriptor force.  Reads back the range of the
// standardised descriptors (one synchronisation) to choose the split-f16
// form, unless the caller asks for FP32 products.
int setup_vec(const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r, int D,
              const double* mom_t, const double* mom_r, const sgr_params* prm, VecWs& w, hipStream_t st) {
  const int M = (int)tmpl->n, N = (int)ref->n;
  HIPCHK(launch_prepare(nullptr, ref->m, N, nullptr, tmpl->m, M, mom_t, mom_r, prep_of(prm), w.dv, st));
  HIPCHK(launch_vprep(a_r, N, a_t, M, D, prm->sigma, w.dv, w.vd, st));
  HIPCHK(launch_vfar_list(a_t, M, D, w.vd, w.dv, w.far_idx, st));
  double cmax = 0.0;
  int n_far = 0;
  HIPCHK(hipMemcpyAsync(&cmax, w.vd + 34, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&n_far, w.far_idx + M, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  w.n_far = n_far;
  w.half = !(prm->flags & FLAG_VEC_FP32) && vforce_half_ok(cmax);
  if (w.half) w.K = vforce_half_K(D);
  HIPCHK(launch_vpack(ref->x, ref->y, ref->z, a_r, ref->m, N, a_t, M, D, w.half, w.dv, w.vd, w.Bt, w.ref4, w.At,
                      st));
  if (n_far > 0) {
    HIPCHK(launch_vfar_ref(a_r, ref->m, N, D, w.vd, w.ref4, w.far_ref, st));
    vfar_prepare(D);
  }
  return SGR_OK;
}

// The vector-descriptor force of one iteration: the contraction kernel,
// then the far rows; returns through `used` the wrench slots written.
hipError_t run_vforce(const VForceArgs& A, const float* a_t, int D, const VecWs& w, bool wu, bool wf, int* used,
                      hipStream_t st) {
  hipError_t e = launch_vforce(A, wu, wf, st);
  if (e != hipSuccess) return e;
  if (used) *used = w.slots + w.n_far;
  return launch_vfar(A, a_t, D, w.vd, w.far_ref, w.far_idx, w.n_far, w.far_part, w.slots, wu, wf, w.n_cu, st);
}

VForceArgs vargs(const sgr_cloud* tmpl, const sgr_cloud* ref, const VecWs& w, const double* pose, int t) {
  VForceArgs A;
  A.At = w.At;
  A.Bt = w.Bt;
  A.ref4 = w.ref4;
  A.y0x = tmpl->x;
  A.y0y = tmpl->y;
  A.y0z = tmpl->z;
  A.mY = tmpl->m;
  A.pose = pose;
  A.dv = w.dv;
  A.M = (int)tmpl->n;
  A.N = (int)ref->n;
  A.K = w.K;
  A.half = w.half;
  A.n_chunks = w.n_chunks;
  A.t = t;
  A.G = 0.0;
  A.wpart = w.wpart;
  A.fpart = w.fpart;
  return A;
}

// ------------------------------------------------- unrolled differentiation
// Host copy of G_t (eq. 12), as the force kernel evaluates it.
double G_host(const sgr_params* prm, int t) {
  return 0.1 * prm->G1 + 0.9 * prm->G1 / (1.0 + std::exp(-(((double)t - 1.0) - 0.5 * prm->E)));
}

int check_unrolled(const sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                   const double* mom_t, const double* mom_r, const sgr_params* prm, int K) {
  if (!ctx || !a_t || !a_r || !mom_t || !mom_r) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  if (is_mixed(prm)) return fail(SGR_EINVAL, "the unrolled registration uses the FP32 force");
  if (prm->E < 1) return fail(SGR_EINVAL, "E must be >= 1");
  if (K < 1) return fail(SGR_EINVAL, "the checkpoint interval must be >= 1");
  if (!(prm->sigma > 0)) return fail(SGR_EINVAL, "the unrolled registration needs an explicit sigma > 0");
  return SGR_OK;
}

// State of an unrolled registration in the context workspace: the same
// set-up and force launch as sgr_register's iteration loop.
struct Unrolled {
  int M = 0, N = 0, pm = 1;
  Tiles T{};
  FLaunch L{};
  Derived* dv = nullptr;
  float4* ref4 = nullptr;
  float* lw = nullptr;
  int* perm = nullptr;
  char* sws = nullptr;
  float4* tm4 = nullptr;
  float2* tmx = nullptr;
  double* wpart = nullptr;
  double* fpart = nullptr;  // per-point forces (backward only)
};

void unrolled_shape(const sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_params* prm,
                    Unrolled& U) {
  U.M = (int)tmpl->n;
  U.N = (int)ref->n;
  U.pm = pmode_of(prm->p);
  U.T = ctx->tiles.pick(U.M, U.N, U.pm);
  U.L = force_shape(ctx, U.M, U.N, U.T, U.pm);
}

void carve_unrolled(Carve& c, Unrolled& U, bool with_f) {
  U.dv = c.take<Derived>(1);
  U.ref4 = c.take<float4>(pad_n(U.N));
  U.lw = c.take<float>(pad_n(U.N));
  U.perm = c.take<int>(U.M);
  U.sws = c.take<char>(sort_perm_workspace(U.M, 1));
  U.tm4 = c.take<float4>(U.M);
  U.tmx = c.take<float2>(U.M);
  U.wpart = c.take<double>((size_t)U.L.slots * WR_STRIDE);
  U.fpart = with_f ? c.take<double>((size_t)U.L.n_chunks * U.M * 3) : nullptr;
}

int setup_unrolled(const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                   const double* mom_t, const double* mom_r, const sgr_params* prm, const Unrolled& U,
                   hipStream_t st) {
  // cold-started SVD in the update: a recomputed segment then reproduces the
  // forward poses bit for bit
  PrepParams P = prep_of(prm);
  P.cold_svd = 1;
  HIPCHK(launch_prepare(a_r, ref->m, U.N, a_t, tmpl->m, U.M, mom_t, mom_r, P, U.dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, U.N, U.dv, U.ref4, U.lw, st));
  HIPCHK(launch_sort_perm(a_t, U.M, U.perm, U.sws, st));
  HIPCHK(launch_pack_tmpl(tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, U.M, U.perm, U.dv, U.tm4, U.tmx, st));
  return SGR_OK;
}

// Force of iteration t at pose_in.  With pose_out: the rigid update into
// pose_out.  With W_out: the wrench (no update).  With f_out: per-point forces.
int unrolled_force(const sgr_cloud* tmpl, const float* a_t, const Unrolled& U, int t, const double* pose_in,
                   double* pose_out, double* W_out, float* f_out, hipStream_t st) {
  const bool wf = f_out != nullptr;
  ForceArgs A{tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, U.ref4, U.lw, pose_in, U.dv, U.M, U.N,
              U.T.chunk_len, U.T.n_chunks, t, 0.0, U.wpart, wf ? U.fpart : nullptr, U.perm, U.tm4, U.tmx};
  HIPCHK(run_force(A, U.T, U.L, U.pm, false, wf, st));
  if (wf) HIPCHK(launch_reduce_f(U.fpart, U.L.n_chunks, U.M, U.perm, f_out, st));
  HIPCHK(launch_update(U.wpart, U.L.slots, pose_in, pose_out, U.dv, t, 0.0, pose_out ? 1 : 0, W_out, nullptr, st));
  return SGR_OK;
}

}  // namespace

extern "C" {

// ------------------------------------------------- allocation-free step
// sgr_step_static carves its buffers from this array instead of the
// context workspace.  Each device holds its own copy (at its own address)
// from the loading of the library's code on it until the process ends.  The
// name is a host-side stand-in in host code: its device address is taken
// once per device with hipGetSymbolAddress (in sgr_create) and only that
// address is handed to kernels.
constexpr size_t SGR_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) char scratch[SGR_SCRATCH_BYTES];
constexpr int SGR_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[SGR_MAX_DEVICES];

// Called with `device` current.
static int scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= SGR_MAX_DEVICES) return fail(SGR_EINVAL, "device index beyond 63");
  if (g_scratch_ptr[device]) return SGR_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(SGR_EHIP, std::string("device address of the static scratch: ") + hipGetErrorString(e));
  }
  g_scratch_ptr[device] = static_cast<char*>(p);
  return SGR_OK;
}

static char* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < SGR_MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

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
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->n_cu = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    const size_t colon = c->arch.find(':');
    if (colon != std::string::npos) c->arch.resize(colon);
  }
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(SGR_EHIP, "stream creation failed");
  }
  c->tiles.init(c->n_cu);
  if (int e = scratch_init(device)) {
    (void)hipStreamDestroy(c->cap);
    delete c;
    return e;
  }
  *out = c;
  return SGR_OK;
}

int sgr_destroy(sgr_ctx* ctx) {
  if (!ctx) return SGR_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  std::vector<GraphCache*> caches = {&ctx->gc, &ctx->gcb, &ctx->gcv};
  for (GraphCache& g : ctx->gcp) caches.push_back(&g);
  for (GraphCache* g : caches) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
  }
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
  if (a_out) {
    if (int e = ensure_ws(ctx, grid_knn_workspace((int)c->n, k))) return e;
    HIPCHK(launch_grid_knn(c->x, c->y, c->z, (int)c->n, k, a_out, nullptr, ctx->ws, st));
  }
  if (moments_out) HIPCHK(launch_moments(c->x, c->y, c->z, c->n, moments_out, st));
  return SGR_OK;
}

int sgr_knn(sgr_ctx* ctx, const sgr_cloud* c, int k, int32_t* idx_out, sgr_stream_t stream) {
  if (!ctx || !idx_out) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(c, "cloud")) return e;
  if (k < 1 || k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  if (c->n < k) return fail(SGR_EINVAL, "cloud has fewer points than k");
  HIPCHK(hipSetDevice(ctx->device));
  if (int e = ensure_ws(ctx, grid_knn_workspace((int)c->n, k))) return e;
  HIPCHK(launch_grid_knn(c->x, c->y, c->z, (int)c->n, k, nullptr, idx_out, ctx->ws, (hipStream_t)stream));
  return SGR_OK;
}

// One iteration (sgr_step); the buffers come from the context workspace
// (grown with hipMalloc on demand) or, with use_static, from the device's
// static scratch, with no allocation at all.
static int step_impl(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                     const double* mom_t, const double* mom_r, const sgr_params* prm, int t, const sgr_pose* in,
                     sgr_pose* out, double* wrench_out, float* f_out, sgr_stream_t stream, bool use_static) {
  if (!ctx) return fail(SGR_EINVAL, "NULL ctx");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  if (!a_t || !a_r || !mom_t || !mom_r || !in || !out) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  if (int e = check_mixed(prm)) return e;
  const Tiles T = tiles_for(ctx, M, N, prm);
  Carve cv{nullptr};
  cv.take<Derived>(1);
  cv.take<float4>(pad_n(N));
  cv.take<float>(pad_n(N));
  const FLaunch L0 = force_shape(ctx, M, N, T, pmode_of(prm->p));
  const int nslot = is_mixed(prm) ? T.nblk : L0.slots;
  const int nch = is_mixed(prm) ? T.n_chunks : L0.n_chunks;
  cv.take<double>((size_t)nslot * WR_STRIDE);
  if (f_out) cv.take<double>((size_t)nch * M * 3);
  cv.take<int>(M);
  cv.take<char>(sort_perm_workspace(M, 1));
  cv.take<float4>(M);
  cv.take<float2>(M);
  char* base = nullptr;
  if (use_static) {
    base = scratch_of(ctx->device);
    if (!base) return fail(SGR_EHIP, "the static scratch of this device has no device address");
    if (cv.off > SGR_SCRATCH_BYTES)
      return fail(SGR_EINVAL, "this step needs " + std::to_string(cv.off) + " bytes of scratch, more than the " +
                                  std::to_string(SGR_SCRATCH_BYTES) + " bytes of the static scratch");
  } else {
    if (int e = ensure_ws(ctx, cv.off)) return e;
    base = ctx->ws;
  }
  Carve w{base};
  Derived* dv = w.take<Derived>(1);
  float4* ref4 = w.take<float4>(pad_n(N));
  float* lw = w.take<float>(pad_n(N));
  double* wpart = w.take<double>((size_t)nslot * WR_STRIDE);
  double* fpart = f_out ? w.take<double>((size_t)nch * M * 3) : nullptr;
  int* perm = w.take<int>(M);
  char* sws = w.take<char>(sort_perm_workspace(M, 1));
  float4* tm4 = w.take<float4>(M);
  float2* tmx = w.take<float2>(M);

  HIPCHK(launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_t, mom_r, prep_of(prm), dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, N, dv, ref4, lw, st));
  HIPCHK(launch_sort_perm(a_t, M, perm, sws, st));
  HIPCHK(launch_pack_tmpl(tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, M, perm, dv, tm4, tmx, st));
  ForceArgs A{tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, ref4, lw, (const double*)in, dv, M, N,
              T.chunk_len, T.n_chunks, t, 0.0, wpart, fpart, perm, tm4, tmx};
  int used = T.nblk;
  if (is_mixed(prm)) {
    HIPCHK(launch_force_mixed(A, f_out != nullptr, st));
  } else {
    const FLaunch L = force_shape(ctx, M, N, T, pmode_of(prm->p));
    HIPCHK(run_force(A, T, L, pmode_of(prm->p), wrench_out != nullptr, f_out != nullptr, st));
    used = L.slots;
  }
  if (f_out) HIPCHK(launch_reduce_f(fpart, nch, M, perm, f_out, st));
  HIPCHK(launch_update(wpart, used, (const double*)in, (double*)out, dv, t, 0.0, 1, wrench_out, nullptr, st));
  return SGR_OK;
}

int sgr_descriptors_batch(sgr_ctx* ctx, int n_clouds, const sgr_cloud* clouds, int k, float* const* a_out,
                          int32_t* const* idx_out, sgr_stream_t stream) {
  if (!ctx || !clouds || (!a_out && !idx_out)) return fail(SGR_EINVAL, "NULL argument");
  if (n_clouds < 1) return fail(SGR_EINVAL, "n_clouds must be >= 1");
  if (k < 1 || k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  std::vector<const float*> cx(n_clouds), cy(n_clouds), cz(n_clouds);
  std::vector<int> cn(n_clouds);
  for (int c = 0; c < n_clouds; ++c) {
    if (int e = check_cloud(&clouds[c], "cloud")) return e;
    if (clouds[c].n < k) return fail(SGR_EINVAL, "a cloud has fewer points than k");
    if ((a_out && !a_out[c]) || (!a_out && !idx_out[c])) return fail(SGR_EINVAL, "NULL output array");
    cx[c] = clouds[c].x;
    cy[c] = clouds[c].y;
    cz[c] = clouds[c].z;
    cn[c] = (int)clouds[c].n;
  }
  HIPCHK(hipSetDevice(ctx->device));
  if (int e = ensure_ws(ctx, grid_knn_batch_workspace(cn.data(), n_clouds, k))) return e;
  HIPCHK(launch_grid_knn_batch(cx.data(), cy.data(), cz.data(), cn.data(), a_out, idx_out, n_clouds, k, ctx->ws,
                               (hipStream_t)stream));
  return SGR_OK;
}

int sgr_step(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
             const double* mom_t, const double* mom_r, const sgr_params* prm, int t, const sgr_pose* in,
             sgr_pose* out, double* wrench_out, float* f_out, sgr_stream_t stream) {
  return step_impl(ctx, tmpl, a_t, ref, a_r, mom_t, mom_r, prm, t, in, out, wrench_out, f_out, stream, false);
}

int sgr_step_static(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                    const double* mom_t, const double* mom_r, const sgr_params* prm, int t, const sgr_pose* in,
                    sgr_pose* out, double* wrench_out, float* f_out, sgr_stream_t stream) {
  return step_impl(ctx, tmpl, a_t, ref, a_r, mom_t, mom_r, prm, t, in, out, wrench_out, f_out, stream, true);
}

int sgr_register(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_params* prm, sgr_pose* inout,
                 double* stats, sgr_stream_t stream) {
  if (!ctx || !inout) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm, true)) return e;
  if (prm->E < 1) return fail(SGR_EINVAL, "E must be >= 1");
  if (prm->k < 1 || prm->k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  if (tmpl->n < prm->k || ref->n < prm->k) return fail(SGR_EINVAL, "a cloud has fewer points than k");
  if (int e = check_mixed(prm)) return e;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  SingleWs w;
  if (int e = carve_single(ctx, M, N, prm, prm->k, w, false)) return e;
  HIPCHK(launch_grid_knn(ref->x, ref->y, ref->z, N, prm->k, w.aX, nullptr, w.gws, st));
  HIPCHK(launch_grid_knn(tmpl->x, tmpl->y, tmpl->z, M, prm->k, w.aY, nullptr, w.gws, st));
  HIPCHK(launch_moments(ref->x, ref->y, ref->z, N, w.mom + 10, st));
  HIPCHK(launch_moments(tmpl->x, tmpl->y, tmpl->z, M, w.mom, st));
  if (int e = setup_single(tmpl, ref, prep_of(prm), w, st)) return e;
  if (int e = run_single_loop(ctx, ctx->gc, tmpl, ref, prm, w, inout, stats, 0, prm->E, st)) return e;
  int32_t status = 0;
  HIPCHK(hipMemcpyAsync(&status, &w.dv->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (status & ST_DEGENERATE) return fail(SGR_EDEGENERATE, "degenerate input: zero variance or zero curvature spread");
  if (status) return fail(SGR_ENUMERIC, "numeric failure in the update (status " + std::to_string(status) + ")");
  return SGR_OK;
}

int sgr_descriptors_radius(sgr_ctx* ctx, const sgr_cloud* c, float r2, float* a_out, int32_t* count_out,
                           sgr_stream_t stream) {
  if (!ctx) return fail(SGR_EINVAL, "NULL ctx");
  if (int e = check_cloud(c, "cloud")) return e;
  if (!(r2 >= 0.0f) || !std::isfinite(r2)) return fail(SGR_EINVAL, "r2 must be finite and >= 0");
  if (!a_out && !count_out) return fail(SGR_EINVAL, "nothing to compute");
  HIPCHK(hipSetDevice(ctx->device));
  if (int e = ensure_ws(ctx, radius_desc_workspace((int)c->n))) return e;
  HIPCHK(launch_radius_desc(c->x, c->y, c->z, (int)c->n, nullptr, 0.0, r2, a_out, count_out, ctx->ws,
                            (hipStream_t)stream));
  return SGR_OK;
}

int sgr_register_pyramid(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_params* prm,
                         const sgr_level* levels, int n_levels, sgr_pose* inout, double* stats, sgr_stream_t stream) {
  if (!ctx || !inout || !levels) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm, true)) return e;
  if (int e = check_mixed(prm)) return e;
  if (n_levels < 1 || n_levels > 64) return fail(SGR_EINVAL, "n_levels must be in [1, 64]");
  int64_t total = 0;
  int kmax = 0;
  bool radius = false;
  for (int l = 0; l < n_levels; ++l) {
    const sgr_level& v = levels[l];
    if (v.iters < 1) return fail(SGR_EINVAL, "every level needs iters >= 1");
    if (!std::isfinite(v.radius_scale) || v.radius_scale < 0) return fail(SGR_EINVAL, "radius_scale must be >= 0");
    if (!std::isfinite(v.sigma_scale) || !(v.sigma_scale > 0)) return fail(SGR_EINVAL, "sigma_scale must be > 0");
    radius |= v.radius_scale > 0;
    if (v.radius_scale == 0) {
      if (v.k < 1 || v.k > 32) return fail(SGR_EINVAL, "a kNN level needs k in [1, 32]");
      if (tmpl->n < v.k || ref->n < v.k) return fail(SGR_EINVAL, "a cloud has fewer points than a level's k");
      kmax = std::max(kmax, (int)v.k);
    }
    total += v.iters;
  }
  if (total != prm->E) return fail(SGR_EINVAL, "the levels' iterations must add up to E");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  SingleWs w;
  if (int e = carve_single(ctx, M, N, prm, kmax, w, radius)) return e;
  if ((int)ctx->gcp.size() < n_levels) ctx->gcp.resize(n_levels);
  HIPCHK(launch_moments(ref->x, ref->y, ref->z, N, w.mom + 10, st));
  HIPCHK(launch_moments(tmpl->x, tmpl->y, tmpl->z, M, w.mom, st));
  std::vector<int32_t> status(n_levels, 0);
  int t0 = 0;
  for (int l = 0; l < n_levels; ++l) {
    const sgr_level& v = levels[l];
    if (v.radius_scale > 0) {
      const double s2 = v.radius_scale * v.radius_scale;
      HIPCHK(launch_radius_desc(ref->x, ref->y, ref->z, N, w.mom + 10, s2, 0.f, w.aX, nullptr, w.gws, st));
      HIPCHK(launch_radius_desc(tmpl->x, tmpl->y, tmpl->z, M, w.mom, s2, 0.f, w.aY, nullptr, w.gws, st));
    } else {
      HIPCHK(launch_grid_knn(ref->x, ref->y, ref->z, N, v.k, w.aX, nullptr, w.gws, st));
      HIPCHK(launch_grid_knn(tmpl->x, tmpl->y, tmpl->z, M, v.k, w.aY, nullptr, w.gws, st));
    }
    PrepParams P = prep_of(prm);
    P.sigma_scale = v.sigma_scale;
    if (int e = setup_single(tmpl, ref, P, w, st)) return e;
    if (int e = run_single_loop(ctx, ctx->gcp[l], tmpl, ref, prm, w, inout, stats, t0, t0 + v.iters, st)) return e;
    HIPCHK(hipMemcpyAsync(&status[l], &w.dv->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    t0 += v.iters;
  }
  HIPCHK(hipStreamSynchronize(st));
  for (int l = 0; l < n_levels; ++l) {
    if (status[l] & ST_DEGENERATE)
      return fail(SGR_EDEGENERATE, "degenerate input at level " + std::to_string(l) +
                                       ": zero variance or zero curvature spread");
    if (status[l])
      return fail(SGR_ENUMERIC, "numeric failure in the update at level " + std::to_string(l) + " (status " +
                                    std::to_string(status[l]) + ")");
  }
  return SGR_OK;
}

int sgr_descriptors_hn(sgr_ctx* ctx, const sgr_cloud* c, int k, int D, float* h_out, sgr_stream_t stream) {
  if (!ctx || !h_out) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(c, "cloud")) return e;
  if (k < 1 || k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  if (c->n < k) return fail(SGR_EINVAL, "cloud has fewer points than k");
  if (D < 2 || D > 30) return fail(SGR_EINVAL, "D must be in [2, 30]");
  HIPCHK(hipSetDevice(ctx->device));
  if (int e = ensure_ws(ctx, normal_hist_workspace((int)c->n, k))) return e;
  HIPCHK(launch_normal_hist(c->x, c->y, c->z, (int)c->n, k, D, h_out, ctx->ws, (hipStream_t)stream));
  return SGR_OK;
}

int sgr_descriptors_poly(sgr_ctx* ctx, const sgr_cloud* c, int k, float* out, sgr_stream_t stream) {
  if (!ctx || !out) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(c, "cloud")) return e;
  if (k < 6 || k > 32) return fail(SGR_EINVAL, "k must be in [6, 32] (six fitted coefficients)");
  if (c->n < k) return fail(SGR_EINVAL, "cloud has fewer points than k");
  HIPCHK(hipSetDevice(ctx->device));
  if (int e = ensure_ws(ctx, poly_workspace((int)c->n, k))) return e;
  HIPCHK(launch_poly(c->x, c->y, c->z, (int)c->n, k, out, ctx->ws, (hipStream_t)stream));
  return SGR_OK;
}

int sgr_step_vec(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r, int D,
                 const double* mom_t, const double* mom_r, const sgr_params* prm, int t, const sgr_pose* in,
                 sgr_pose* out, double* wrench_out, float* f_out, sgr_stream_t stream) {
  if (!ctx) return fail(SGR_EINVAL, "NULL ctx");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  if (int e = check_vec(prm, D)) return e;
  if (!a_t || !a_r || !mom_t || !mom_r || !in || !out) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n;
  VecWs w;
  if (int e = carve_vec(ctx, M, (int)ref->n, D, f_out != nullptr, false, w)) return e;
  if (int e = setup_vec(tmpl, a_t, ref, a_r, D, mom_t, mom_r, prm, w, st)) return e;
  int used = w.slots;
  HIPCHK(run_vforce(vargs(tmpl, ref, w, (const double*)in, t), a_t, D, w, wrench_out != nullptr,
                    f_out != nullptr, &used, st));
  if (f_out) HIPCHK(launch_reduce_f(w.fpart, w.n_chunks, M, nullptr, f_out, st));
  HIPCHK(launch_update(w.wpart, used, (const double*)in, (double*)out, w.dv, t, 0.0, 1, wrench_out, nullptr, st));
  return SGR_OK;
}

int sgr_register_vec(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                     int D, const sgr_params* prm, sgr_pose* inout, double* stats, sgr_stream_t stream) {
  if (!ctx || !inout || !a_t || !a_r) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm, true)) return e;
  if (int e = check_vec(prm, D)) return e;
  if (prm->E < 1) return fail(SGR_EINVAL, "E must be >= 1");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  const bool pinv = (prm->flags & FLAG_PINV) != 0;
  VecWs w;
  if (int e = carve_vec(ctx, M, N, D, false, true, w, pinv)) return e;
  HIPCHK(launch_moments(ref->x, ref->y, ref->z, N, w.mom + 10, st));
  HIPCHK(launch_moments(tmpl->x, tmpl->y, tmpl->z, M, w.mom, st));
  if (int e = setup_vec(tmpl, a_t, ref, a_r, D, w.mom, w.mom + 10, prm, w, st)) return e;
  if (pinv) {
    // the pair sums once: one pass of the vector kernel writing them per chunk
    VForceArgs A = vargs(tmpl, ref, w, (const double*)inout, 0);
    A.spart = w.ps_part;
    HIPCHK(run_vforce(A, a_t, D, w, true, false, nullptr, st));
    HIPCHK(launch_psum_reduce(w.ps_part, M, w.n_chunks, w.ps_S, st));
    HIPCHK(launch_pack_plain(tmpl->x, tmpl->y, tmpl->z, tmpl->m, M, w.tm4, w.tmx, st));
  }
  auto loop = [&](hipStream_t s) -> int {
    for (int t = 0; t < prm->E; ++t) {
      const bool wu = stats != nullptr;  // U is read only from the stats
      int used = w.slots;
      if (pinv) {
        HIPCHK(launch_pinv(w.tm4, w.tmx, w.ps_S, M, (const double*)inout, w.dv, t, wu, w.wpart, s));
        used = pinv_blocks(M);
      } else {
        HIPCHK(run_vforce(vargs(tmpl, ref, w, (const double*)inout, t), a_t, D, w, wu, false, &used, s));
      }
      HIPCHK(launch_update(w.wpart, used, (const double*)inout, (double*)inout, w.dv, t, 0.0, 1, nullptr,
                           stats ? stats + (size_t)t * STATS_STRIDE : nullptr, s));
    }
    return SGR_OK;
  };
  if ((prm->flags & FLAG_NO_GRAPH) || prm->E < 2) {
    if (int e = loop(st)) return e;
  } else {
    std::vector<uint8_t> key;
    const void* ptrs[12] = {tmpl->x, tmpl->y, tmpl->z, tmpl->m, ref->x, ref->y, ref->z, ref->m, inout, stats, a_t, a_r};
    key_add(key, ptrs, 12);
    const int64_t dims[5] = {M, N, D, w.half ? 1 : 0, w.n_far};
    key_add(key, dims, 5);
    key_add(key, prm, 1);
    const void* wsp = ctx->ws;
    key_add(key, &wsp, 1);
    if (int e = run_graph(ctx, ctx->gcv, key, loop, st)) return e;
  }
  int32_t status = 0;
  HIPCHK(hipMemcpyAsync(&status, &w.dv->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (status & ST_DEGENERATE) return fail(SGR_EDEGENERATE, "degenerate input: zero variance or zero descriptor spread");
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

int sgr_autotune(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                 const double* mom_t, const double* mom_r, const sgr_params* prm, int reps, int* best,
                 double* best_ms, sgr_stream_t stream) {
  if (!ctx || !a_t || !a_r || !mom_t || !mom_r) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm)) return e;
  if (reps < 1) reps = 5;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  const int pm = pmode_of(prm->p);
  const auto key = std::make_tuple(log2_bucket(M), log2_bucket(N), pm);
  // Candidates: template points per lane, the reference load variant, and
  // the blocks per CU of the launch: 1 to 4 (long reference chunks, a few
  // resident blocks), and 1 to 8 waves of resident blocks (from the kernel's
  // occupancy, at most 64 blocks per CU).  Several waves of shorter chunks
  // even out the end of a large launch: the SIMDs serve the oldest wave
  // first, so the blocks of a CU do not finish together, and a block's fixed
  // start and end cost little beside a long pair loop.
  const int cand_R[4] = {1, 2, 4, 8};
  constexpr int kMaxWaves = 8;
  // size the workspace for the largest candidate
  size_t need = 0;
  for (int R : cand_R)
    for (int v : {0, 1}) {
      Tiles T = TileTable::make(M, N, R, 8 * ctx->n_cu, v);
      T.bpc = std::min(64, kMaxWaves * force_blocks_per_cu(R, pm, v != 0));
      Carve cv{nullptr};
      cv.take<double>(16);
      cv.take<Derived>(1);
      cv.take<float4>(pad_n(N));
      cv.take<float>(pad_n(N));
      cv.take<int>(M);
      cv.take<char>(sort_perm_workspace(M, 1));
      cv.take<float4>(M);
      cv.take<float2>(M);
      cv.take<double>((size_t)force_shape(ctx, M, N, T, pm).slots * WR_STRIDE);
      need = std::max(need, cv.off);
    }
  if (int e = ensure_ws(ctx, need)) return e;
  Carve w{ctx->ws};
  double* pose = w.take<double>(16);
  Derived* dv = w.take<Derived>(1);
  float4* ref4 = w.take<float4>(pad_n(N));
  float* lw = w.take<float>(pad_n(N));
  int* perm = w.take<int>(M);
  char* sws = w.take<char>(sort_perm_workspace(M, 1));
  float4* tm4 = w.take<float4>(M);
  float2* tmx = w.take<float2>(M);
  const size_t wp_off = w.off;
  HIPCHK(launch_identity_pose(pose, st));
  HIPCHK(launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_t, mom_r, prep_of(prm), dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, N, dv, ref4, lw, st));
  HIPCHK(launch_sort_perm(a_t, M, perm, sws, st));
  HIPCHK(launch_pack_tmpl(tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, M, perm, dv, tm4, tmx, st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best_t = 1e300;
  int bR = 4, bB = 8, bV = 0;
  for (int v : {0, 1})
    for (int R : cand_R)
      for (int c = 0; c < 4 + kMaxWaves; ++c) {
        const int occ = force_blocks_per_cu(R, pm, v != 0);
        const int bpc = c < 4 ? c + 1 : (c - 3) * occ;
        if (c < 4 && bpc >= occ) continue;  // covered by the occupancy targets
        if (bpc > 64) continue;
        Tiles T = TileTable::make(M, N, R, 8 * ctx->n_cu, v);
        T.bpc = bpc;
        const FLaunch L = force_shape(ctx, M, N, T, pm);
        Carve wc{ctx->ws, wp_off};
        double* wpart = wc.take<double>((size_t)L.slots * WR_STRIDE);
        ForceArgs A{tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, ref4, lw, pose, dv, M, N,
                    T.chunk_len, T.n_chunks, prm->E - 1, 0.0, wpart, nullptr, perm, tm4, tmx};
        HIPCHK(run_force(A, T, L, pm, false, false, st));
        HIPCHK(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) HIPCHK(run_force(A, T, L, pm, false, false, st));
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        const double per = ms / reps;
        if (per < best_t) {
          best_t = per;
          bR = R;
          bB = T.bpc;
          bV = v;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->tiles.over[key] = std::make_tuple(bR, bB, bV);
  if (best) {
    best[0] = bR;
    best[1] = bB;
    best[2] = bV;
  }
  if (best_ms) *best_ms = best_t;
  return SGR_OK;
}

int sgr_tiles_save(sgr_ctx* ctx, const char* path) {
  if (!ctx || !path) return fail(SGR_EINVAL, "NULL argument");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(SGR_EINVAL, std::string("cannot write ") + path);
  std::fprintf(f, "{\"arch\": \"%s\", \"entries\": [", ctx->arch.c_str());
  bool first = true;
  for (const auto& kv : ctx->tiles.over) {
    std::fprintf(f, "%s\n  {\"m_bucket\": %d, \"n_bucket\": %d, \"p_mode\": %d, \"R\": %d, \"blocks_per_cu\": %d, "
                 "\"variant\": %d}", first ? "" : ",", std::get<0>(kv.first), std::get<1>(kv.first),
                 std::get<2>(kv.first), std::get<0>(kv.second), std::get<1>(kv.second), std::get<2>(kv.second));
    first = false;
  }
  std::fprintf(f, "\n]}\n");
  std::fclose(f);
  return SGR_OK;
}

int sgr_tiles_load(sgr_ctx* ctx, const char* path) {
  if (!ctx || !path) return fail(SGR_EINVAL, "NULL argument");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(SGR_EINVAL, std::string("cannot read ") + path);
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
  std::fclose(f);
  const size_t a = txt.find("\"arch\": \"");
  if (a == std::string::npos) return fail(SGR_EINVAL, "not a tile table");
  const size_t a0 = a + 9, a1 = txt.find('"', a0);
  if (txt.compare(a0, a1 - a0, ctx->arch) != 0) return fail(SGR_EINVAL, "tile table is for another architecture");
  size_t pos = 0;
  int loaded = 0;
  while ((pos = txt.find("{\"m_bucket\":", pos)) != std::string::npos) {
    int mb, nb, pmv, R, bpc, v;
    if (std::sscanf(txt.c_str() + pos,
                    "{\"m_bucket\": %d, \"n_bucket\": %d, \"p_mode\": %d, \"R\": %d, \"blocks_per_cu\": %d, "
                    "\"variant\": %d}", &mb, &nb, &pmv, &R, &bpc, &v) != 6)
      return fail(SGR_EINVAL, "malformed tile table entry");
    if ((R != 1 && R != 2 && R != 4 && R != 8) || bpc < 1 || bpc > 64 || (v != 0 && v != 1))
      return fail(SGR_EINVAL, "tile table entry out of range");
    ctx->tiles.over[std::make_tuple(mb, nb, pmv)] = std::make_tuple(R, bpc, v);
    ++loaded;
    ++pos;
  }
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
  if (int e = check_mixed(prm)) return e;
  const Tiles T = tiles_for(ctx, M, N, prm);
  Carve cv{nullptr};
  cv.take<double>(16);
  cv.take<double>(16);
  cv.take<Derived>(1);
  cv.take<float4>(pad_n(N));
  cv.take<float>(pad_n(N));
  const FLaunch L0 = force_shape(ctx, M, N, T, pm);
  const int nslot = is_mixed(prm) ? T.nblk : L0.slots;
  const int nch = is_mixed(prm) ? T.n_chunks : L0.n_chunks;
  cv.take<double>((size_t)nslot * WR_STRIDE);
  cv.take<double>((size_t)nch * M * 3);
  cv.take<int>(M);
  cv.take<char>(sort_perm_workspace(M, 1));
  cv.take<float4>(M);
  cv.take<float2>(M);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  double* mom_t = w.take<double>(16);
  double* pose = w.take<double>(16);
  Derived* dv = w.take<Derived>(1);
  float4* ref4 = w.take<float4>(pad_n(N));
  float* lw = w.take<float>(pad_n(N));
  double* wpart = w.take<double>((size_t)nslot * WR_STRIDE);
  double* fpart = w.take<double>((size_t)nch * M * 3);
  int* perm = w.take<int>(M);
  char* sws = w.take<char>(sort_perm_workspace(M, 1));
  float4* tm4 = w.take<float4>(M);
  float2* tmx = w.take<float2>(M);
  HIPCHK(launch_moments(tmpl->x, tmpl->y, tmpl->z, M, mom_t, st));
  HIPCHK(launch_identity_pose(pose, st));
  HIPCHK(launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_t, mom_r, prep_of(prm), dv, st));
  HIPCHK(launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, N, dv, ref4, lw, st));
  HIPCHK(launch_sort_perm(a_t, M, perm, sws, st));
  HIPCHK(launch_pack_tmpl(tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, M, perm, dv, tm4, tmx, st));
  ForceArgs A{tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, ref4, lw, pose, dv, M, N,
              T.chunk_len, T.n_chunks, 0, G, wpart, f_out ? fpart : nullptr, perm, tm4, tmx};
  int used = T.nblk;
  if (is_mixed(prm)) {
    HIPCHK(launch_force_mixed(A, f_out != nullptr, st));
  } else {
    const FLaunch L = force_shape(ctx, M, N, T, pm);
    HIPCHK(run_force(A, T, L, pm, wrench_out != nullptr, f_out != nullptr, st));
    used = L.slots;
  }
  if (f_out) HIPCHK(launch_reduce_f(fpart, nch, M, perm, f_out, st));
  if (wrench_out) HIPCHK(launch_update(wpart, used, pose, nullptr, dv, 0, G, 0, wrench_out, nullptr, st));
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
  const Tiles T = adj_shape(ctx, M, N, ctx->tiles.pick(M, N, pm).R, pm == 1);
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
  int* perm = nullptr;
  float4* tm4 = nullptr;
  float2* tmx = nullptr;
  int nslot = 0;  // wrench slots allocated
  int nch = 0;    // reference chunks of a launch with per-point output
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
  if (int e = check_mixed(prm)) {
    delete pl;
    return e;
  }
  pl->T = tiles_for(ctx, M, N, prm);
  Carve cv{nullptr};
  cv.take<Derived>(1);
  cv.take<float4>(pad_n(N));
  cv.take<float>(pad_n(N));
  {
    const FLaunch L0 = force_shape(ctx, M, N, pl->T, pl->pm);
    pl->nslot = is_mixed(prm) ? pl->T.nblk : L0.slots;
    pl->nch = is_mixed(prm) ? pl->T.n_chunks : L0.n_chunks;
  }
  cv.take<double>((size_t)pl->nslot * WR_STRIDE);
  cv.take<double>((size_t)pl->nch * M * 3);
  cv.take<int>(M);
  cv.take<char>(sort_perm_workspace(M, 1));
  cv.take<float4>(M);
  cv.take<float2>(M);
  if (hipMalloc(&pl->mem, cv.off) != hipSuccess) {
    (void)hipGetLastError();
    delete pl;
    return fail(SGR_ENOMEM, "plan allocation failed");
  }
  Carve w{pl->mem};
  pl->dv = w.take<Derived>(1);
  pl->ref4 = w.take<float4>(pad_n(N));
  pl->lw = w.take<float>(pad_n(N));
  pl->wpart = w.take<double>((size_t)pl->nslot * WR_STRIDE);
  pl->fpart = w.take<double>((size_t)pl->nch * M * 3);
  pl->perm = w.take<int>(M);
  char* sws = w.take<char>(sort_perm_workspace(M, 1));
  pl->tm4 = w.take<float4>(M);
  pl->tmx = w.take<float2>(M);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e1 = launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_t, mom_r, prep_of(prm), pl->dv, st);
  hipError_t e2 = e1 == hipSuccess ? launch_pack_ref(ref->x, ref->y, ref->z, a_r, ref->m, N, pl->dv, pl->ref4, pl->lw, st)
                                   : e1;
  if (e2 == hipSuccess) e2 = launch_sort_perm(a_t, M, pl->perm, sws, st);
  if (e2 == hipSuccess)
    e2 = launch_pack_tmpl(tmpl->x, tmpl->y, tmpl->z, a_t, tmpl->m, M, pl->perm, pl->dv, pl->tm4, pl->tmx, st);
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
                   t, G, pl->wpart, with_f ? pl->fpart : nullptr, pl->perm, pl->tm4, pl->tmx};
}

int sgr_plan_force(sgr_plan* pl, int t, double G, const sgr_pose* pose, double* wrench_out, float* f_out,
                   sgr_stream_t stream) {
  if (!pl || !pose) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(pl->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ForceArgs A = plan_args(pl, t, G, pose, f_out != nullptr);
  int used = pl->T.nblk;
  if (is_mixed(&pl->prm)) {
    HIPCHK(launch_force_mixed(A, f_out != nullptr, st));
  } else {
    const FLaunch L = force_shape(pl->ctx, (int)pl->tmpl.n, (int)pl->ref.n, pl->T, pl->pm);
    HIPCHK(run_force(A, pl->T, L, pl->pm, wrench_out != nullptr, f_out != nullptr, st));
    used = L.slots;
  }
  if (f_out) HIPCHK(launch_reduce_f(pl->fpart, pl->nch, (int)pl->tmpl.n, pl->perm, f_out, st));
  if (wrench_out)
    HIPCHK(launch_update(pl->wpart, used, (const double*)pose, nullptr, pl->dv, t, G, 0, wrench_out, nullptr, st));
  return SGR_OK;
}

int sgr_plan_step(sgr_plan* pl, int t, const sgr_pose* pose_in, sgr_pose* pose_out, double* wrench_out,
                  sgr_stream_t stream) {
  if (!pl || !pose_in || !pose_out) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(pl->ctx->device));
  hipStream_t st = (hipStream_t)stream;
  ForceArgs A = plan_args(pl, t, 0.0, pose_in, false);
  int used = pl->T.nblk;
  if (is_mixed(&pl->prm)) {
    HIPCHK(launch_force_mixed(A, false, st));
  } else {
    const FLaunch L = force_shape(pl->ctx, (int)pl->tmpl.n, (int)pl->ref.n, pl->T, pl->pm);
    HIPCHK(run_force(A, pl->T, L, pl->pm, wrench_out != nullptr, false, st));
    used = L.slots;
  }
  HIPCHK(launch_update(pl->wpart, used, (const double*)pose_in, (double*)pose_out, pl->dv, t, 0.0, 1, wrench_out,
                       nullptr, st));
  return SGR_OK;
}

int sgr_register_batch(sgr_ctx* ctx, int B, const sgr_cloud* tmpls, const sgr_cloud* refs, const sgr_params* prm,
                       sgr_pose* poses, double* energy_out, double* stats, sgr_stream_t stream) {
  if (!ctx || !tmpls || !refs || !poses) return fail(SGR_EINVAL, "NULL argument");
  if (B < 1) return fail(SGR_EINVAL, "empty batch");
  if (int e = check_params(prm, true)) return e;
  if (is_mixed(prm)) return fail(SGR_EINVAL, "the batched form runs the FP32 force only");
  if (prm->E < 1) return fail(SGR_EINVAL, "E must be >= 1");
  if (prm->k < 1 || prm->k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  BatchIn in;
  in.B = B;
  for (int r = 0; r < B; ++r) {
    if (int e = check_cloud(&tmpls[r], "template")) return e;
    if (int e = check_cloud(&refs[r], "reference")) return e;
    if (tmpls[r].n < prm->k || refs[r].n < prm->k) return fail(SGR_EINVAL, "a cloud has fewer points than k");
    in.tm.push_back(&tmpls[r]);
    in.rf.push_back(&refs[r]);
    in.tm_cloud.push_back((int)in.clouds.size());
    in.clouds.push_back(&tmpls[r]);
    in.rf_cloud.push_back((int)in.clouds.size());
    in.clouds.push_back(&refs[r]);
    in.pack_of.push_back(r);
  }
  HIPCHK(hipSetDevice(ctx->device));
  return run_batch(ctx, in, prm, (double*)poses, nullptr, energy_out, stats, nullptr, (hipStream_t)stream);
}

int sgr_multistart(sgr_ctx* ctx, const sgr_cloud* tmpl, const sgr_cloud* ref, const sgr_params* prm, int S,
                   const double* R0, sgr_pose* poses, double* energy_out, int32_t* best_out, sgr_stream_t stream) {
  if (!ctx || !R0 || !poses) return fail(SGR_EINVAL, "NULL argument");
  if (S < 1) return fail(SGR_EINVAL, "no starts");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (int e = check_params(prm, true)) return e;
  if (is_mixed(prm)) return fail(SGR_EINVAL, "the batched form runs the FP32 force only");
  if (prm->E < 1) return fail(SGR_EINVAL, "E must be >= 1");
  if (prm->k < 1 || prm->k > 32) return fail(SGR_EINVAL, "k must be in [1, 32]");
  if (tmpl->n < prm->k || ref->n < prm->k) return fail(SGR_EINVAL, "a cloud has fewer points than k");
  BatchIn in;
  in.B = S;
  in.clouds = {tmpl, ref};
  for (int s = 0; s < S; ++s) {
    in.tm.push_back(tmpl);
    in.rf.push_back(ref);
    in.tm_cloud.push_back(0);
    in.rf_cloud.push_back(1);
    in.pack_of.push_back(0);
  }
  HIPCHK(hipSetDevice(ctx->device));
  return run_batch(ctx, in, prm, (double*)poses, R0, energy_out, nullptr, best_out, (hipStream_t)stream);
}


int sgr_unrolled_fwd(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                     const double* mom_t, const double* mom_r, const sgr_params* prm, int K, sgr_pose* pose,
                     double* ckpt, sgr_stream_t stream) {
  if (int e = check_unrolled(ctx, tmpl, a_t, ref, a_r, mom_t, mom_r, prm, K)) return e;
  if (!pose || !ckpt) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  Unrolled U;
  unrolled_shape(ctx, tmpl, ref, prm, U);
  Carve cv{nullptr};
  carve_unrolled(cv, U, false);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  carve_unrolled(w, U, false);
  if (int e = setup_unrolled(tmpl, a_t, ref, a_r, mom_t, mom_r, prm, U, st)) return e;
  double* P = (double*)pose;
  for (int t = 0; t < prm->E; ++t) {
    if (t % K == 0)
      HIPCHK(hipMemcpyAsync(ckpt + (size_t)(t / K) * 13, P, 13 * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (int e = unrolled_force(tmpl, a_t, U, t, P, P, nullptr, nullptr, st)) return e;
  }
  return SGR_OK;
}

int sgr_unrolled_bwd(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                     const double* mom_t, const double* mom_r, const sgr_params* prm, int K, const double* ckpt,
                     const double* grad_final, double* grad_pose0, double* grad_se, sgr_stream_t stream) {
  if (int e = check_unrolled(ctx, tmpl, a_t, ref, a_r, mom_t, mom_r, prm, K)) return e;
  if (!ckpt || !grad_final || !grad_pose0 || !grad_se) return fail(SGR_EINVAL, "NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  Unrolled U;
  unrolled_shape(ctx, tmpl, ref, prm, U);
  const int M = U.M, N = U.N, E = prm->E;
  // the adjoint kernels use tile-multiple chunks (at most 4 points per lane)
  const Tiles TA = adj_shape(ctx, M, N, U.T.R, U.pm == 1);
  const int nseg = (E + K - 1) / K;
  const int npg = pose_grad_blocks(M);
  auto carve_rest = [&](Carve& c, double** seg, double** W, double** g0, double** g1, double** gW, double** gse_t,
                        double** mom_y, Derived** dva, double** fsum, double** pg, float** Y, float** f, float** gf0,
                        float** gy, float** lam, double** ypart, double** spart) {
    carve_unrolled(c, U, true);
    *seg = c.take<double>((size_t)(K + 1) * 13);
    *W = c.take<double>(16);
    *g0 = c.take<double>(16);
    *g1 = c.take<double>(16);
    *gW = c.take<double>(16);
    *gse_t = c.take<double>(2);
    *mom_y = c.take<double>(16);
    *dva = c.take<Derived>(1);
    *fsum = c.take<double>(16);
    *pg = c.take<double>((size_t)npg * 12);
    *Y = c.take<float>((size_t)M * 3);
    *f = c.take<float>((size_t)M * 3);
    *gf0 = c.take<float>((size_t)M * 3);
    *gy = c.take<float>((size_t)M * 3);
    *lam = c.take<float>((size_t)M * 3);
    *ypart = c.take<double>((size_t)TA.n_chunks * M * 4);
    *spart = c.take<double>((size_t)TA.nblk * 2);
  };
  double *seg, *W, *g0, *g1, *gW, *gse_t, *mom_y, *fsum, *pg, *ypart, *spart;
  Derived* dva;
  float *Y, *f, *gf0, *gy, *lam;
  {
    Carve cv{nullptr};
    carve_rest(cv, &seg, &W, &g0, &g1, &gW, &gse_t, &mom_y, &dva, &fsum, &pg, &Y, &f, &gf0, &gy, &lam, &ypart, &spart);
    if (int e = ensure_ws(ctx, cv.off)) return e;
  }
  Carve w{ctx->ws};
  carve_rest(w, &seg, &W, &g0, &g1, &gW, &gse_t, &mom_y, &dva, &fsum, &pg, &Y, &f, &gf0, &gy, &lam, &ypart, &spart);
  if (int e = setup_unrolled(tmpl, a_t, ref, a_r, mom_t, mom_r, prm, U, st)) return e;
  HIPCHK(launch_fill_f(gf0, (int64_t)M * 3, 0.f, st));
  HIPCHK(launch_fill(grad_se, 2, 0.0, st));
  HIPCHK(hipMemcpyAsync(g0, grad_final, 13 * sizeof(double), hipMemcpyDeviceToDevice, st));
  float* Yx = Y;
  float* Yy = Y + M;
  float* Yz = Y + 2 * (size_t)M;
  for (int sgi = nseg - 1; sgi >= 0; --sgi) {
    const int t0 = sgi * K, t1 = std::min(E, t0 + K);
    // poses of this segment, recomputed from its checkpoint
    HIPCHK(hipMemcpyAsync(seg, ckpt + (size_t)sgi * 13, 13 * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int t = t0; t < t1 - 1; ++t)
      if (int e = unrolled_force(tmpl, a_t, U, t, seg + (size_t)(t - t0) * 13, seg + (size_t)(t - t0 + 1) * 13,
                                 nullptr, nullptr, st))
        return e;
    for (int t = t1 - 1; t >= t0; --t) {
      const double* Pt = seg + (size_t)(t - t0) * 13;
      // forward quantities of iteration t: per-point forces and the wrench
      if (int e = unrolled_force(tmpl, a_t, U, t, Pt, nullptr, W, f, st)) return e;
      // update: cotangent of the pose it starts from and of (F, K)
      HIPCHK(launch_update_bwd(Pt, W, g0, U.dv, g1, gW, st));
      // force field at the posed template: per-point gradient and (sigma, eps)
      HIPCHK(launch_pose_points(tmpl->x, tmpl->y, tmpl->z, M, Pt, Yx, Yy, Yz, st));
      HIPCHK(launch_moments(Yx, Yy, Yz, M, mom_y, st));
      HIPCHK(launch_prepare(a_r, ref->m, N, a_t, tmpl->m, M, mom_y, mom_r, prep_of(prm), dva, st));
      AdjArgs AA{Yx, Yy, Yz, a_t, tmpl->m, U.ref4, U.lw, dva, M, N, TA.chunk_len, TA.n_chunks, TA.nblk,
                 U.pm == 1, G_host(prm, t), f, gf0, gW, lam, ypart, spart, gy, nullptr, gse_t};
      HIPCHK(launch_adjoint(AA, TA.R, fsum, st));
      HIPCHK(launch_axpy(gse_t, 2, grad_se, st));
      // y_i = s R y0_i + t: per-point gradient onto the pose
      HIPCHK(launch_pose_grad(gy, tmpl->x, tmpl->y, tmpl->z, M, Pt, pg, g1, st));
      std::swap(g0, g1);
    }
  }
  HIPCHK(hipMemcpyAsync(grad_pose0, g0, 13 * sizeof(double), hipMemcpyDeviceToDevice, st));
  return SGR_OK;
}


int sgr_change_detect(sgr_ctx* ctx, const sgr_cloud* tmpl, const float* a_t, const sgr_cloud* ref, const float* a_r,
                      const sgr_pose* pose, double tau, double sigma, double s_min, uint8_t* flags_out,
                      int32_t* nn_out, float* d2_out, sgr_stream_t stream) {
  if (!ctx || !a_t || !a_r || !pose || !flags_out) return fail(SGR_EINVAL, "NULL argument");
  if (int e = check_cloud(tmpl, "template")) return e;
  if (int e = check_cloud(ref, "reference")) return e;
  if (!(tau > 0)) return fail(SGR_EINVAL, "tau must be > 0 (+inf disables the distance test)");
  if (s_min > 1.0) return fail(SGR_EINVAL, "s_min must be <= 1 (<= 0 disables the shape test)");
  if (s_min > 0 && !(sigma > 0 && std::isfinite(sigma))) return fail(SGR_EINVAL, "the shape test needs sigma > 0");
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = (hipStream_t)stream;
  const int M = (int)tmpl->n, N = (int)ref->n;
  Carve cv{nullptr};
  cv.take<char>(change_workspace(M, N));
  cv.take<int32_t>(M);
  cv.take<float>(M);
  if (int e = ensure_ws(ctx, cv.off)) return e;
  Carve w{ctx->ws};
  char* cws = w.take<char>(change_workspace(M, N));
  int32_t* nn = nn_out ? nn_out : w.take<int32_t>(M);
  float* d2 = d2_out ? d2_out : w.take<float>(M);
  // both thresholds rounded once, as a reader would: tau^2 to float32, and
  // sigma^2 (-ln s_min) in FP64
  const float tau2 = (float)(tau * tau);
  const double thr = s_min > 0 ? sigma * sigma * (-std::log(s_min)) : INFINITY;
  HIPCHK(launch_change(tmpl->x, tmpl->y, tmpl->z, a_t, M, ref->x, ref->y, ref->z, a_r, N, (const double*)pose, tau2,
                       thr, flags_out, nn, d2, cws, st));
  return SGR_OK;
}

}  // extern "C"
