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

template <int D, typename T, int P = 0>
bool m2t_d(const DevPlan& a, const DevWork& wk, hipStream_t s)
{
    if constexpr (P > PMax<D>::value) {
        return false;
    } else {
        if (a.p == P) {
            if (a.nnjobs > 0)
                hipLaunchKernelGGL((k_m2t_nodes<D, P, FKT_M2T_KIND, T>), dim3((unsigned)((a.nnjobs + 3) / 4)), dim3(256),
                                   0, s, a, (const T*)wk.mom, (T*)wk.zacc);
            else
                hipLaunchKernelGGL((k_m2t<D, P, FKT_M2T_KIND, T>), dim3(a.nblocks), dim3(kWave), 0, s, a,
                                   (const T*)wk.mom, (T*)wk.zacc);
            return true;
        }
        return m2t_d<D, T, P + 1>(a, wk, s);
    }
}

template <typename T>
bool m2t_t(const DevPlan& a, const DevWork& wk, hipStream_t s)
{
    switch (a.d) {
    case 3: return m2t_d<3, T>(a, wk, s);
    case 4: return m2t_d<4, T>(a, wk, s);
    case 5: return m2t_d<5, T>(a, wk, s);
    default: return false;
    }
}

}  // namespace

bool FKT_CAT(launch_m2t_kind, FKT_M2T_KIND)(const DevPlan& a, const DevWork& wk, int prec, hipStream_t s)
{
    return prec == 1 ? m2t_t<float>(a, wk, s) : m2t_t<double>(a, wk, s);
}

}  // namespace fkt
