// Two-level preconditioning: a Nystrom coarse space joined to the per-leaf
// local part by the Woodbury identity (project addition for the
// Gaussian-process solves; see coarse.hip).
#ifndef FKT_COARSE_H
#define FKT_COARSE_H

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fkt_device.h"

namespace fkt {

// One entry of a batched FP64 product C = alpha op(A) diag(w) op(B) + beta C
// (element offsets into the shared A, B, w and C arrays; w is indexed by the
// contraction index and only read when the launch passes a w array).
struct Gemm64 {
    int M, N, K;
    int lda, ldb, ldc;
    int64_t a_off, b_off, c_off, w_off;
};

// Every descriptor of desc (device, nbatch entries) as one launch;
// max_m / max_n bound the entries' M and N (they size the grid).
hipError_t gemm64_batched(bool ta, bool tb, const Gemm64* desc, int nbatch, int max_m, int max_n, const double* A,
                          const double* B, const double* w, double* C, double alpha, double beta, hipStream_t s);

// out[i][j] = K(|x_i - x_{cols[j]}|) for tree positions i < n and landmark
// tree positions cols[j], j < k (row-major n x k).
hipError_t kernel_columns(const DevPlan& a, const int* cols, int k, double* out, hipStream_t s);

// u = G^T (h .* s) for G [n][k] row-major: per-chunk partial sums of
// nchunk row chunks (part: k x nchunk doubles, column-major by chunk), then
// their sum, one wave per entry of u.
hipError_t gemv_t_weighted(int64_t n, int k, const double* G, const double* h, const double* sv, double* part,
                           int nchunk, double* u, hipStream_t s);
// w = Cinv u (k x k, row-major)
hipError_t gemv_small(int k, const double* Cinv, const double* u, double* w, hipStream_t s);
// y = sv - G w
hipError_t gemv_sub(int64_t n, int k, const double* G, const double* w, const double* sv, double* y, hipStream_t s);
// out[z][i] summed over z < nz into C, plus the identity when add_eye (k x k)
hipError_t sum_partials64(int nz, int64_t len, const double* part, double* out, int add_eye_k, hipStream_t s);

constexpr int kCoarseChunks = 1024;  // row chunks of gemv_t_weighted (4 waves each)
constexpr int kCoarseMaxRank = 4096;

// Host dense SPD helpers (row-major k x k, threads over rows/columns).
// chol_lower: in place, lower triangle of a = L (upper part left untouched);
// false if a is not positive definite.
bool chol_lower(int k, double* a);
// a <- a^{-1} for SPD a; false if a is not positive definite.
bool spd_inverse(int k, double* a);
// w <- L^{-T} (upper triangular, row-major) for a = L L^T; false if a is not
// positive definite.
bool chol_inv_t(int k, const double* a, double* w);

}  // namespace fkt

#endif
