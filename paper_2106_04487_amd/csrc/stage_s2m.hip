// s2m launches (source-to-multipole moments and partial-sum reduction).
#include "fkt_kernels.h"

#if !defined(FKT_S2M_D) || !defined(FKT_S2M_PREC)
#error "compile with -DFKT_S2M_D=<3|4|5> -DFKT_S2M_PREC=<0|1>"
#endif
#define FKT_CAT2(a, b) a##b
#define FKT_CAT(a, b) FKT_CAT2(a, b)

namespace fkt {
namespace {

template <int D, int P, typename T, int C0>
void launch_s2m_chunks(const DevPlan& a, const T* src, int S, int col, T* mom, T* part, hipStream_t s)
{
    constexpr int R = cbinom(P + D, D);
    if constexpr (C0 < R) {
        constexpr int CH = s2m_chunk<T>(R);
        constexpr int C1 = (C0 + CH < R) ? C0 + CH : R;
        hipLaunchKernelGGL((k_s2m<D, P, T, C0, C1>), dim3(a.nunits), dim3(kWave), 0, s, a, src, S, col, mom, part);
        launch_s2m_chunks<D, P, T, C1>(a, src, S, col, mom, part, s);
    }
}

// moments of the nc columns of the pass, one column block after another
template <int D, int P, typename T>
void s2m_dp(const DevPlan& a, const DevWork& wk, hipStream_t s, int nc)
{
    constexpr int R = cbinom(P + D, D);
    const int S = src_stride(D, nc);
    for (int c = 0; c < nc; ++c) {
        T* mom = (T*)wk.mom + c * wk.mom_cols;
        T* part = (T*)wk.part + c * wk.part_cols;
        launch_s2m_chunks<D, P, T, 0>(a, (const T*)wk.src, S, c, mom, part, s);
        if (a.nred > 0) {
            const int64_t tot = (int64_t)a.nred * R;
            hipLaunchKernelGGL((k_s2m_reduce<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a.nred, R,
                               a.red_slot, a.red_off, part, mom);
        }
    }
}

template <int D, typename T, int P = 0>
bool s2m_d(const DevPlan& a, const DevWork& wk, hipStream_t s, int nc)
{
    if constexpr (P > PMax<D>::value) {
        return false;
    } else {
        if (a.p == P) {
            s2m_dp<D, P, T>(a, wk, s, nc);
            return true;
        }
        return s2m_d<D, T, P + 1>(a, wk, s, nc);
    }
}

}  // namespace

// One translation unit per (dimension, precision): FKT_S2M_D and FKT_S2M_PREC
// (0 FP64, 1 FP32) are set when compiling, so the large high-order
// instantiations build in parallel.
bool FKT_CAT(FKT_CAT(launch_s2m_d, FKT_S2M_D), FKT_CAT(_p, FKT_S2M_PREC))(const DevPlan& a, const DevWork& wk,
                                                                         hipStream_t s, int nc)
{
    if (nc != 1 && (nc != kMvmCols || nc > wk.ncmax)) return false;
#if FKT_S2M_PREC == 1
    return s2m_d<FKT_S2M_D, float>(a, wk, s, nc);
#else
    return s2m_d<FKT_S2M_D, double>(a, wk, s, nc);
#endif
}

}  // namespace fkt
