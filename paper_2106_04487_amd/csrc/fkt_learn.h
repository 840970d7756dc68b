// Learned per-leaf spectral preconditioner (device state and operations);
// see learn.hip for the method.
#ifndef FKT_LEARN_H
#define FKT_LEARN_H

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "fkt_host.h"

namespace fkt {

constexpr int kLearnHidden = 256;
constexpr int kLearnFeatures = kLearnFeat;
constexpr int kLearnParams = kLearnFeatures * kLearnHidden + kLearnHidden + kLearnHidden * kLearnHidden + kLearnHidden +
                             kLearnHidden + 1;
constexpr int kLearnMaxLeaf = 2048;  // LDS of the apply kernel: 2 x leaf doubles

struct LearnState;
LearnState* learn_create(int device, hipStream_t s, const LeafSpectra& S, const int64_t* perm, int64_t n, uint64_t seed,
                         std::string& err);
void learn_destroy(LearnState* L);
hipError_t learn_update_spectra(LearnState* L, const LeafSpectra& S);
hipError_t learn_params(LearnState* L, float* host, bool set);
hipError_t learn_grad(LearnState* L, float* host);
// x (device, n, FP32 or FP64) <- N(0, 1) draws keyed by key; synchronises
hipError_t learn_randn(LearnState* L, void* x, int64_t n, bool f32, uint64_t key);
// h = exp(o) / lam from the current weights (and, two-level, C^-1 for it)
hipError_t learn_prepare_filter(LearnState* L);
// z[:, col] = M r[:, col]: the learned filter, or with bj its block-Jacobi
// state h = 1 / lam; two-level when a coarse part is set
hipError_t learn_apply(LearnState* L, const double* r, double* z, int nrhs, int col, hipStream_t s, bool bj = false);
// Coarse part from the Nystrom factor Lmat (device, n x k, tree-order rows);
// k = 0 (or Lmat NULL) drops it. The spectra must be those of the residual
// blocks K_ll + sigma2 I - L_l L_l^T. Synchronises.
hipError_t learn_set_coarse(LearnState* L, const double* Lmat, int k);
int learn_coarse_rank(const LearnState* L);
fkt_status learn_loss_grad(fkt_plan_t P, LearnState* L, int prec, double sigma2, const double* v, int B, double* loss);
fkt_status learn_train(fkt_plan_t P, LearnState* L, int prec, double sigma2, int steps, int B, double lr, uint64_t seed,
                       double* loss_first, double* loss_last);
// Condition-number objective (learn.hip): log kappa(P A) from T PCG / Lanczos
// iterations on b (device, n; overwritten), gradient into the state's
// gradient buffer; and `steps` Adam steps of it on fresh Gaussian b.
fkt_status learn_cond_grad(fkt_plan_t P, LearnState* L, int prec, double sigma2, double* b, int T, double* cond);
fkt_status learn_train_cond(fkt_plan_t P, LearnState* L, int prec, double sigma2, int steps, int T, double lr,
                            uint64_t seed, double* cond_first, double* cond_last);

}  // namespace fkt

#endif
