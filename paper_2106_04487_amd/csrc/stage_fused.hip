// Persistent near + far field launches (k_fused) for one kernel kind
// (FKT_FUSED_KIND, set when compiling).
#include "fkt_kernels.h"

#ifndef FKT_FUSED_KIND
#error "compile with -DFKT_FUSED_KIND=<fkt_kernel_kind value>"
#endif
#define FKT_CAT2(a, b) a##b
#define FKT_CAT(a, b) FKT_CAT2(a, b)

namespace fkt {
namespace {

// resident blocks per CU assumed for the grid (more are harmless: a block
// that finds the queue empty exits at once)
constexpr int kFusedBlocksPerCU = 8;

template <int D, typename T, int P, int NCOL>
bool fused_dpn(const DevPlan& a, const DevWork& wk, hipStream_t s, T c0, T c1, T scale)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return false;
    const int64_t items = (int64_t)(a.nnjobs + kFusedJobs - 1) / kFusedJobs + a.nnear_units;
    const int64_t want = (items + 3) / 4;  // four waves per block
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)cus * kFusedBlocksPerCU));
    hipLaunchKernelGGL((k_fused<D, P, FKT_FUSED_KIND, T, NCOL>), dim3(grid), dim3(256), 0, s, a, (const T*)wk.src,
                       (const T*)wk.mom, wk.mom_cols, (T*)wk.zacc, wk.qctr, c0, c1, scale);
    return true;
}

template <int D, typename T, int P = 0>
bool fused_d(const DevPlan& a, const DevWork& wk, hipStream_t s, int nc, T c0, T c1, T scale)
{
    if constexpr (P > PMax<D>::value) {
        return false;
    } else {
        if (a.p == P) {
            if (nc == 1) return fused_dpn<D, T, P, 1>(a, wk, s, c0, c1, scale);
            if (nc == kMvmCols) return fused_dpn<D, T, P, kMvmCols>(a, wk, s, c0, c1, scale);
            return false;
        }
        return fused_d<D, T, P + 1>(a, wk, s, nc, c0, c1, scale);
    }
}

// built for d = 3 only (the persistent launch measured slower than the two
// separate launches; plan time rejects it for d = 4, 5)
template <typename T>
bool fused_t(const DevPlan& a, const DevWork& wk, hipStream_t s, int nc, T c0, T c1, T scale)
{
    return a.d == 3 ? fused_d<3, T>(a, wk, s, nc, c0, c1, scale) : false;
}

}  // namespace

bool FKT_CAT(launch_fused_kind, FKT_FUSED_KIND)(const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc,
                                                double c0, double c1, double scale)
{
    if (nc != 1 && (nc != kMvmCols || nc > wk.ncmax)) return false;
    if (a.comp_keep > 0 || (a.nslots > 0 && a.nnjobs <= 0) || !wk.qctr) return false;
    return prec == 1 ? fused_t<float>(a, wk, s, nc, (float)c0, (float)c1, (float)scale)
                     : fused_t<double>(a, wk, s, nc, c0, c1, scale);
}

}  // namespace fkt
