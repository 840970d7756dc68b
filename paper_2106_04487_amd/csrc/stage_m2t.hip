// m2t launches for one kernel kind (FKT_M2T_KIND, set when compiling):
// the multipole-to-target kernels are specialised per kernel so that each
// carries only its own radial-derivative code.
#include "fkt_kernels.h"

#ifndef FKT_M2T_KIND
#error "compile with -DFKT_M2T_KIND=<fkt_kernel_kind value>"
#endif
#define FKT_CAT2(a, b) a##b
#define FKT_CAT(a, b) FKT_CAT2(a, b)

namespace fkt {
namespace {

// one pass of NCOL columns at order P
template <int D, typename T, int P, int NCOL>
bool m2t_dpn(const DevPlan& a, const DevWork& wk, hipStream_t s)
{
    constexpr int KEEP = radial_keep(FKT_M2T_KIND, D);
    if constexpr (KEEP > 0) {
        if (a.comp_keep > 0) {
            // compressed: combine the moments, then the node-major far field on them
            if (a.comp_keep != KEEP || a.nnjobs <= 0 || a.comp_rank != crank(D, P, KEEP)) return false;
            for (int c = 0; c < NCOL; ++c)
                hipLaunchKernelGGL((k_compress<D, P, T, KEEP>), dim3((unsigned)((a.nslots + 255) / 256)), dim3(256),
                                   0, s, a, (const T*)wk.mom + c * wk.mom_cols, (T*)wk.momc + c * wk.momc_cols);
            hipLaunchKernelGGL((k_m2t_nodes<D, P, FKT_M2T_KIND, T, KEEP, NCOL>), dim3((unsigned)((a.nnjobs + 3) / 4)),
                               dim3(256), 0, s, a, (const T*)wk.momc, wk.momc_cols, (T*)wk.zacc);
            return true;
        }
    }
    if (a.comp_keep > 0) return false;
    if (a.nnjobs > 0) {
        hipLaunchKernelGGL((k_m2t_nodes<D, P, FKT_M2T_KIND, T, 0, NCOL>), dim3((unsigned)((a.nnjobs + 3) / 4)),
                           dim3(256), 0, s, a, (const T*)wk.mom, wk.mom_cols, (T*)wk.zacc);
        return true;
    }
    if constexpr (NCOL == 1) {
        hipLaunchKernelGGL((k_m2t<D, P, FKT_M2T_KIND, T>), dim3(a.nblocks, a.job_nseg), dim3(kWave), 0, s, a, (const T*)wk.mom,
                           (T*)wk.zacc);
        return true;
    }
    return false;  // several columns need the node-major jobs
}

template <int D, typename T, int P = 0>
bool m2t_d(const DevPlan& a, const DevWork& wk, hipStream_t s, int nc)
{
    if constexpr (P > PMax<D>::value) {
        return false;
    } else {
        if (a.p == P) {
            if (nc == 1) return m2t_dpn<D, T, P, 1>(a, wk, s);
            if (nc == kMvmCols) return m2t_dpn<D, T, P, kMvmCols>(a, wk, s);
            return false;
        }
        return m2t_d<D, T, P + 1>(a, wk, s, nc);
    }
}

template <typename T>
bool m2t_t(const DevPlan& a, const DevWork& wk, hipStream_t s, int nc)
{
    switch (a.d) {
    case 3: return m2t_d<3, T>(a, wk, s, nc);
    case 4: return m2t_d<4, T>(a, wk, s, nc);
    case 5: return m2t_d<5, T>(a, wk, s, nc);
    default: return false;
    }
}

}  // namespace

bool FKT_CAT(launch_m2t_kind, FKT_M2T_KIND)(const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc)
{
    if (nc != 1 && (nc != kMvmCols || nc > wk.ncmax)) return false;
    return prec == 1 ? m2t_t<float>(a, wk, s, nc) : m2t_t<double>(a, wk, s, nc);
}

}  // namespace fkt
