// Launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fkt {

// Read-only plan data on the device (all pointers are device memory).
struct DevPlan {
    int n, d, p, rank, nblocks, nslots, nunits, nred;
    int kind;
    double ell, alpha, var;       // kernel parameters
    const double* pts64;          // [n][d] tree-ordered coordinates
    const float* pts32;           // [n][d] FP32 copy (FP32 plans only)
    const int64_t* perm;          // tree position -> original index
    const int* blk_begin;         // per 64-target block: first tree position
    const int* blk_count;         //   and number of targets (<= 64)
    const int* near_off;          // [nblocks + 1] into near_*
    const int* near_beg;          // source leaf point range
    const int* near_end;
    const uint64_t* near_mask;    // lanes whose target has this leaf in N_l
    const int* far_off;           // [nblocks + 1] into far_*
    const int* far_slot;          // far node (compact slot id)
    const uint64_t* far_mask;     // lanes whose target is in F_b
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
};

// Per-call work buffers (device) for one right-hand-side column.
struct DevWork {
    void* src;    // [n][4 or 6] tree-ordered packed (coordinates, weight) records
    void* zfar;   // [n] far-field result, tree order
    void* mom;    // [nslots][rank]
    void* part;   // [npartials][rank]
};

// Whether kernels for (d, p) are compiled into the library.
bool far_supported(int d, int p);

// One column of y = K~ x: gather, s2m, m2t, near (+ far) and scatter.
// x, y: n x nrhs row-major in the plan's precision; col selects the column.
// prec: 0 FP64, 1 FP32.
// ev: NULL, or 5 events recorded before the gather and after the gather,
// s2m, m2t and near stages.
hipError_t launch_mvm_column(const DevPlan& a, const DevWork& wk, const void* x, void* y, int nrhs, int col,
                             int prec, hipStream_t s, hipEvent_t* ev);

}  // namespace fkt
