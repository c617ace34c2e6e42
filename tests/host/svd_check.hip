// Host harness for the 3x3 FP64 routines the rigid update runs on the GPU
// (svd3, kabsch_rot, eig_psd3): reads matrices from stdin, prints results.
// Input per case: warm flag, A (9, row-major), V0 (9, row-major; read only
// when warm is 1).  Output per case: sv (3), u (9, u[k][r]), v (9), the
// Kabsch rotation R (9, row-major), its status (1/0), then the
// eigenvalues of (A + A^T) / 2 taken as a PSD matrix's (3).
#include <cstdio>

#include "../../paper_1902_01061_amd/csrc/common.h"

int main() {
  int warm;
  while (std::scanf("%d", &warm) == 1) {
    double A[9], V0[9], Vw[9];
    for (double& x : A) std::scanf("%lf", &x);
    for (double& x : V0) std::scanf("%lf", &x);
    double sv[3], u[3][3], v[3][3], R[9];
    sgr::svd3(A, sv, u, v, warm ? V0 : nullptr);
    for (int e = 0; e < 9; ++e) Vw[e] = V0[e];
    const bool ok = sgr::kabsch_rot(A, R, warm ? Vw : nullptr);
    const double S6[6] = {A[0], A[4], A[8], 0.5 * (A[1] + A[3]), 0.5 * (A[2] + A[6]), 0.5 * (A[5] + A[7])};
    double lam[3];
    sgr::eig_psd3(S6, lam);
    for (double x : sv) std::printf("%.17g ", x);
    for (auto& r : u) for (double x : r) std::printf("%.17g ", x);
    for (auto& r : v) for (double x : r) std::printf("%.17g ", x);
    for (double x : R) std::printf("%.17g ", x);
    std::printf("%d ", ok ? 1 : 0);
    for (double x : lam) std::printf("%.17g ", x);
    std::printf("\n");
  }
  return 0;
}
