// Many-right-hand-side MVM (groups of 32 columns, FP32 plans): padded leaf
// layout for the matrix-core near field, and the launchers (mrhs.hip, mvm.hip).
#ifndef FKT_MRHS_H
#define FKT_MRHS_H

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fkt_device.h"

namespace fkt {

constexpr int kMrCols = 32;      // columns per group
constexpr int kMrJobNodes = 4;   // far nodes per 64-lane job of the matrix-core far field
constexpr int kMrSegJobs = 64;   // far jobs per work unit of the matrix-core far field
constexpr int kMrSegNear = 32;   // near leaves per work unit of the matrix-core near field
constexpr int kMrGroupBlocks = 64;  // target blocks whose far pairs are packed together (at most 64)

struct DevMrhs {
    int npad = 0;                     // leaves padded to multiples of 32 points
    const float* pts = nullptr;       // [d][npad] SoA coordinates (pad: leaf's first point)
    const int* src = nullptr;         // [npad] tree position, -1 on padding
    const int* near_off = nullptr;    // [nblocks + 1] target-major near lists of the 64-target blocks
    const int* near_pbeg = nullptr;   //   padded first point of the leaf (multiple of 32)
    const int* near_pcnt = nullptr;   //   padded point count (multiple of 32)
    const uint64_t* near_mask = nullptr;  // targets of the block that have the leaf in their near set
    // a block's near leaves are cut into units of near_seg leaves, one wave
    // each (grid nblocks x near_nseg); units add into zf, which is then
    // written to the output
    int near_seg = kMrSegNear;
    int near_nseg = 1;
    void* xt = nullptr;               // [32][npad] weights of the group (bf16 or FP32)
    void* zf = nullptr;               // [n][32] far field of the group, FP32, tree order
    bool bf16 = false;
    // far field of the group on the matrix cores
    void* mom = nullptr;              // [32][nslots][rank] FP32 moments
    void* x32 = nullptr;              // [n][32] FP32 weights of the group in tree order
    void* part32 = nullptr;           // [32][npart][rank] partial moments of split nodes
    int64_t npart = 0;
    void* bhi = nullptr;              // [nslots][ks][2][64] bf16 x 8 MFMA B fragments, high part
    void* blo = nullptr;              //   and low part (m - hi)
    int ks = 0;                       // 32-entry k-steps per node (rank padded to a multiple of 64)
    const int* job_off = nullptr;     // far jobs per group of job_group blocks, up to kMrJobNodes nodes each
    const int* job_noff = nullptr;
    const int* job_nodes = nullptr;
    const uint16_t* job_pairs = nullptr;
    int job_group = 1;                // blocks per group (pair word: lane | block in group << 6 | node << 12)
    int ngroups = 0;
    // the far jobs of a group are cut into units of job_seg consecutive jobs,
    // one wave each (grid ngroups x job_nseg), so the waves of heavy groups
    // spread over the machine; every job adds its rows into zf atomically
    int job_seg = kMrSegJobs;
    int job_nseg = 1;
};

// far field of one column (gather clearing wk.zacc, s2m, m2t into wk.zacc)
hipError_t launch_far_column(const DevPlan& a, const DevWork& wk, const void* x, int nrhs, int col, int prec,
                             hipStream_t s);
// FP32 near-kernel constants (log2(e) folded where an exponential follows)
void near_consts_f32(const DevPlan& a, float& c0, float& c1);
#define FKT_DECLARE_M2T_MRHS(K) bool launch_m2t_mrhs_kind##K(const DevPlan& a, const DevMrhs& mr, hipStream_t s);
FKT_DECLARE_M2T_MRHS(0)
FKT_DECLARE_M2T_MRHS(1)
FKT_DECLARE_M2T_MRHS(2)
FKT_DECLARE_M2T_MRHS(3)
FKT_DECLARE_M2T_MRHS(4)
FKT_DECLARE_M2T_MRHS(5)
FKT_DECLARE_M2T_MRHS(6)
#undef FKT_DECLARE_M2T_MRHS
// moments of the 32 columns of the group (x32 gathered) into mom, per dimension
bool launch_s2m_mrhs_d3(const DevPlan& a, const DevMrhs& mr, hipStream_t s);
bool launch_s2m_mrhs_d4(const DevPlan& a, const DevMrhs& mr, hipStream_t s);
bool launch_s2m_mrhs_d5(const DevPlan& a, const DevMrhs& mr, hipStream_t s);
// s2m of one column into the given moment buffer (gather included)
hipError_t launch_s2m_column(const DevPlan& a, const DevWork& wk, const void* x, int nrhs, int col, int prec,
                             hipStream_t s);
// y = K~ x for nrhs (a multiple of 32) FP32 columns
hipError_t launch_mvm_mrhs(const DevPlan& a, const DevWork& wk, const DevMrhs& mr, const float* x, float* y, int nrhs,
                           hipStream_t s);

}  // namespace fkt

#endif
