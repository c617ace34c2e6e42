// Launch shape of the pair-force kernel: template points per lane (R),
// template blocks, reference chunks.  The defaults are R = 2 (R = 1 for
// small templates) and, for the FP32 force kernel, one wave of resident
// blocks; the tile-multiple chunking here (8 blocks per CU) serves the
// mixed-precision and adjoint kernels.  The autotuner can override R, the
// blocks per CU and the load variant per (M, N, p-mode) bucket.
#pragma once
#include <stdint.h>

#include <map>
#include <tuple>

namespace sgr {

struct Tiles {
  int R;
  int sm;   // 1: reference read through scalar loads instead of LDS
  int bpc;  // FP32 force kernel: blocks per CU (0: one wave of resident blocks)
  int n_iblk;
  int n_chunks;
  int chunk_len;
  int nblk;
};

inline int log2_bucket(int64_t n) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= n) ++b;
  return b;
}

struct TileTable {
  int n_cu = 256;
  // (M bucket, N bucket, p mode) -> (R, blocks per CU target, variant)
  std::map<std::tuple<int, int, int>, std::tuple<int, int, int>> over;

  void init(int cus) { n_cu = cus; }

  static Tiles make(int M, int N, int R, int target_blocks, int sm = 0) {
    const int bt = 256, tj = 256;
    Tiles T;
    T.R = R;
    T.sm = sm;
    T.bpc = 0;
    T.n_iblk = (M + bt * R - 1) / (bt * R);
    int nc = (target_blocks + T.n_iblk - 1) / T.n_iblk;
    const int max_nc = (N + tj - 1) / tj;
    if (nc > max_nc) nc = max_nc;
    if (nc < 1) nc = 1;
    int cl = (N + nc - 1) / nc;
    cl = ((cl + tj - 1) / tj) * tj;
    T.chunk_len = cl;
    T.n_chunks = (N + cl - 1) / cl;
    T.nblk = T.n_iblk * T.n_chunks;
    return T;
  }

  Tiles pick(int M, int N, int pm) const {
    auto it = over.find(std::make_tuple(log2_bucket(M), log2_bucket(N), pm));
    if (it != over.end()) {
      Tiles T = make(M, N, std::get<0>(it->second), std::get<1>(it->second) * n_cu, std::get<2>(it->second));
      T.bpc = std::get<1>(it->second);
      return T;
    }
    const int R = M <= 256 * 2 * 4 ? 1 : 2;
    return make(M, N, R, 8 * n_cu);
  }
};

}  // namespace sgr
