// Launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/fkt.h"

namespace fkt {

// Read-only plan data on the device (all pointers are device memory).
struct DevPlan {
    int n, d, p, rank, nblocks, nslots, nunits, nred, nnear_units;
    int kind;
    double ell, alpha, var;       // kernel parameters
    const double* pts64;          // [n][d] tree-ordered coordinates
    const float* pts32;           // [n][d] FP32 copy (FP32 plans only)
    const int64_t* perm;          // tree position -> original index
    const int* blk_begin;         // per 64-target block: first tree position
    const int* blk_count;         //   and number of targets (<= 64)
    const int* near_tgt;          // near sets N_l: target positions grouped by leaf
    const int* nu_beg;            // near units: source leaf point range
    const int* nu_end;
    const int* nu_toff;           //   and their targets near_tgt[toff, toff + tcnt)
    const int* nu_tcnt;
    const int* job_off;           // [nblocks + 1] far-field jobs of each block
    const int* job_noff;          // [njobs + 1] into job_nodes
    const int* job_nodes;         // far-node slots of each job
    const uint16_t* job_pairs;    // [njobs][64] target lane | job node index << 6
    int job_seg, job_nseg;        // block-major jobs per work unit, units per block (grid nblocks x job_nseg)
    int nnjobs;                   // node-major far field (0: block-major jobs above)
    const int* nj_slot;           // [nnjobs] far-node slot of each job
    const int* nj_tgt;            // [nnjobs][64] target tree positions (-1: empty lane)
    const double* slot_ctr;       // [nslots][d] expansion centres
    const double* slot_scale;     // [nslots] node radius (1 when zero)
    const int* unit_slot;         // s2m units: node slot
    const int* unit_begin;        //   point range
    const int* unit_end;
    const int* unit_dst;          //   >= 0: moment slot; < 0: partial -1-dst
    const int* red_slot;          // slots summed from partials
    const int* red_off;           // [nred + 1] partial ranges
    const double* tbar;           // [(k*(p+1)+j)*(p+1)+m]
    const double* hn64;           // squared harmonic normalisation (x Z_k), FP64
    const float* hn32;            //   and FP32 copy
    const double* exp2tab;        // [256] 2^(j/256), FP64 exponential table
    // radial compression (Appendix A.4): comp_keep > 0 keeps the first
    // min(comp_keep, nj) radial rows of every degree; the moments are
    // combined into them with comp_coef (see radial_keep, k_compress)
    int fused;                    // near and far field in one persistent launch (k_fused)
    // batched plans: instance of every far-node slot and near unit, and (set
    // only for the operator applications of a solve) one flag per instance:
    // work of an instance whose flag is 0 is skipped (its output rows are
    // then not computed)
    const int* slot_inst;
    const int* nu_inst;
    const unsigned char* inst_active;
    int comp_keep;
    int comp_rank;                // moments per node after compression
    double comp_invlen;           // 1 / l of the scaled distance (1 for 1/r)
    const double* comp_coef;      // [(p+1)][p/2+1][p/2+1]
};

// Right-hand-side columns of one multi-column MVM pass: every stage runs the
// columns together (shared kernel values, harmonics and radial functions)
// on plans with the node-major far field; others run column by column.
constexpr int kMvmCols = 4;
constexpr int kFarSegJobs = 32;  // block-major far jobs per work unit

// Rows kept per degree by the compressed kernels built for (kind, d), 0 for
// none: 1/r and e^(-r/l) in d = 3 (the paper's Table "ranks": R_k = 1 and 2).
constexpr int radial_keep(int kind, int d)
{
    if (d != 3) return 0;
    return kind == FKT_LAPLACE ? 1 : (kind == FKT_EXPONENTIAL ? 2 : 0);
}

// Per-call work buffers (device) for one right-hand-side column.
struct DevWork {
    void* src;    // [n][4 or 6] tree-ordered packed (coordinates, weight) records
    void* zacc;   // [n] per-target sum (far field stored, near field added), tree order
    void* mom;    // [nslots][rank]
    void* part;   // [npartials][rank]
    void* momc;   // [nslots][comp_rank] compressed moments (comp_keep > 0)
    // src and zacc hold ncmax columns ([point][column]); mom, part and momc
    // ncmax blocks ([column][slot or partial][entry]) of these sizes:
    int ncmax;
    size_t mom_cols, part_cols, momc_cols;  // elements per column block
    unsigned* qctr;  // work-queue counter of the persistent launch (fused plans)
    hipStream_t side;    // second stream: the near field runs beside the far field
    hipEvent_t fork, join;
};

// Far nodes per 64-lane far-field job: as many node moment sets as fit in
// 8 KB of LDS (two such buffers per wave), between 1 and 8.
constexpr int m2t_max_job_nodes(int d, int p, int elem_bytes)
{
    long long r = 1;
    for (int i = 1; i <= d; ++i) r = r * (p + i) / i;  // C(p+d, d)
    const long long n = 8192 / (r * elem_bytes);
    return n < 1 ? 1 : (n > 8 ? 8 : (int)n);
}

// Whether kernels for (d, p) are compiled into the library, and the highest
// order built for d (-1 for none).
bool far_supported(int d, int p);
int far_max_order(int d);

// One column of y = K~ x: gather, s2m, m2t, near (+ far) and scatter.
// x, y: n x nrhs row-major in the plan's precision; col selects the column.
// prec: 0 FP64, 1 FP32.
// ev: NULL, or 5 events recorded before the gather and after the gather,
// s2m, m2t and near stages.
// What CG needs of a plan (set by the C-ABI layer).
struct LearnState;
struct CgPlanView {
    int64_t n;
    int prec;
    int device;
    hipStream_t stream;
    const int64_t* perm;     // device: tree position -> original index
    int nleaf, maxleaf;      // block-Jacobi blocks (precond = 1)
    const int* bj_begin;
    const int* bj_count;
    const int64_t* bj_off;
    const double* bj_inv;
    LearnState* learn;       // learned spectral filter (precond = 2)
    int nseg;                // independent systems per column: instances of a batched plan
    const int64_t* seg_off;  // device [nseg + 1]: instance rows [seg_off[i], seg_off[i + 1]) (user order)
    const int32_t* row_seg;  // device [n]: instance of each row (NULL when nseg = 1)
    int coarse = 0;          // two-level: precond 1 and 2 run through learn_apply with the coarse part
    unsigned char* active = nullptr;  // device [nseg] instance flags for masked MVMs (batched plans)
};

// fkt_mvm that skips the work of instances whose flag in the plan's
// instance-flag buffer is 0 (set by the caller on the plan's stream first);
// without such a buffer (one instance) it is fkt_mvm.
fkt_status mvm_masked(fkt_plan_t P, const void* x, void* y, int nrhs);

// Columns col .. col + ncols - 1 of y = K~ x in one pass of nc columns (1 or
// kMvmCols, ncols <= nc; nc > 1 needs the node-major far field or no far
// field, and work buffers sized for nc columns).
hipError_t launch_mvm_column(const DevPlan& a, const DevWork& wk, const void* x, void* y, int nrhs, int col,
                             int ncols, int nc, int prec, hipStream_t s, bool overlap, hipEvent_t* ev);

}  // namespace fkt
