// Orchestration of one MVM pass (gather, s2m, m2t, near field, scatter) over
// one or kMvmCols right-hand-side columns, and the near-field launches.
#include "fkt_kernels.h"
#include "fkt_mrhs.h"

namespace fkt {

bool launch_m2t(int kind, const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc)
{
    switch (kind) {
    case 0: return launch_m2t_kind0(a, wk, prec, s, nc);
    case 1: return launch_m2t_kind1(a, wk, prec, s, nc);
    case 2: return launch_m2t_kind2(a, wk, prec, s, nc);
    case 3: return launch_m2t_kind3(a, wk, prec, s, nc);
    case 4: return launch_m2t_kind4(a, wk, prec, s, nc);
    case 5: return launch_m2t_kind5(a, wk, prec, s, nc);
    case 6: return launch_m2t_kind6(a, wk, prec, s, nc);
    default: return false;
    }
}

namespace {

// near-field kernel constants (FP32 variants fold log2(e) into c0)
template <typename T>
void near_consts(const DevPlan& a, T& c0, T& c1)
{
    const bool f32 = std::is_same<T, float>::value;
    const double log2e = 1.4426950408889634074;
    double k0 = 0.0, k1 = 0.0;
    switch (a.kind) {
    case FKT_GAUSSIAN: k0 = -0.5 / (a.ell * a.ell) * (f32 ? log2e : 1.0); break;
    case FKT_EXPONENTIAL: k0 = -1.0 / a.ell * (f32 ? log2e : 1.0); break;
    case FKT_MATERN32:
    case FKT_MATERN52: {
        const double c = (a.kind == FKT_MATERN32 ? 1.7320508075688772935 : 2.2360679774997896964) / a.ell;
        if (f32) { k0 = -c * log2e; k1 = c; if (a.kind == FKT_MATERN52) k0 = -log2e; }
        else k0 = c;
        break;
    }
    case FKT_RATQUAD: k0 = 0.5 / (a.alpha * a.ell * a.ell); k1 = -a.alpha; break;
    case FKT_CAUCHY: k0 = 1.0 / (a.ell * a.ell); break;
    default: break;
    }
    c0 = (T)k0;
    c1 = (T)k1;
}

template <int D, typename T, int NCOL>
bool run_near_d(const DevPlan& a, const T* src, T* zacc, hipStream_t s)
{
    if (a.nnear_units == 0) return true;
    T c0, c1;
    near_consts<T>(a, c0, c1);
    const T scale = (T)a.var;
    dim3 g(a.nnear_units), b(kWave);
    switch (a.kind) {
#define FKT_NEAR_CASE(K) \
    case K: hipLaunchKernelGGL((k_near<D, K, T, NCOL>), g, b, 0, s, a, src, zacc, c0, c1, scale); return true;
        FKT_NEAR_CASE(FKT_GAUSSIAN)
        FKT_NEAR_CASE(FKT_EXPONENTIAL)
        FKT_NEAR_CASE(FKT_MATERN32)
        FKT_NEAR_CASE(FKT_MATERN52)
        FKT_NEAR_CASE(FKT_RATQUAD)
        FKT_NEAR_CASE(FKT_CAUCHY)
        FKT_NEAR_CASE(FKT_LAPLACE)
#undef FKT_NEAR_CASE
    default: return false;
    }
}

// Stream layout of one pass (overlap on):
//   s:    gather (+ clear accumulators) -> fork -> s2m -> m2t -> wait join -> scatter
//   side:                        wait fork -> near field -> join
// Far and near fields both add into the accumulators, so they may run
// concurrently. With overlap off every stage runs in order on s. Profiling
// events (7, optional): e0 start, e1 after gather, e2 after s2m, e3 after
// m2t, e4/e5 around the near field on its own stream, e6 after the scatter.
// A pass covers columns col .. col + ncols - 1 with NC accumulators per
// target (NC = 1 or kMvmCols; padded columns carry zero weights).
template <typename T, int NC>
hipError_t mvm_pass(const DevPlan& a, const DevWork& wk, const T* x, T* y, int nrhs, int col, int ncols,
                    hipStream_t s, bool overlap, hipEvent_t* ev)
{
    const T* pts = std::is_same<T, float>::value ? (const T*)a.pts32 : (const T*)a.pts64;
    T* src = (T*)wk.src;
    T* zacc = (T*)wk.zacc;
    unsigned* ctr = a.fused ? wk.qctr : nullptr;
    const dim3 gg((a.n + 255) / 256), gb(256);
    hipError_t e;
    auto mark = [&](int i, hipStream_t q) -> hipError_t { return ev ? hipEventRecord(ev[i], q) : hipSuccess; };
    if ((e = mark(0, s)) != hipSuccess) return e;
    switch (a.d) {
    case 3: hipLaunchKernelGGL((k_gather<3, T, NC>), gg, gb, 0, s, a.n, a.perm, pts, x, nrhs, col, ncols, src, zacc, ctr); break;
    case 4: hipLaunchKernelGGL((k_gather<4, T, NC>), gg, gb, 0, s, a.n, a.perm, pts, x, nrhs, col, ncols, src, zacc, ctr); break;
    case 5: hipLaunchKernelGGL((k_gather<5, T, NC>), gg, gb, 0, s, a.n, a.perm, pts, x, nrhs, col, ncols, src, zacc, ctr); break;
    default: return hipErrorInvalidValue;
    }
    if ((e = mark(1, s)) != hipSuccess) return e;
    const int prec = std::is_same<T, float>::value ? 1 : 0;
    if (a.fused) {
        // s2m, then near and far field in one persistent launch; events e4/e5
        // bracket the persistent launch like e2/e3
        if (a.nslots > 0 && !launch_s2m(a, wk, prec, s, NC)) return hipErrorInvalidValue;
        if ((e = mark(2, s)) != hipSuccess) return e;
        if ((e = mark(4, s)) != hipSuccess) return e;
        T c0, c1;
        near_consts<T>(a, c0, c1);
        if (!launch_fused(a.kind, a, wk, prec, s, NC, (double)c0, (double)c1, a.var)) return hipErrorInvalidValue;
        if ((e = mark(3, s)) != hipSuccess) return e;
        if ((e = mark(5, s)) != hipSuccess) return e;
        hipLaunchKernelGGL((k_scatter<T, NC>), gg, gb, 0, s, a.n, a.perm, (const T*)zacc, y, nrhs, col, ncols);
        if ((e = mark(6, s)) != hipSuccess) return e;
        return hipGetLastError();
    }
    overlap = overlap && wk.side != nullptr;
    const hipStream_t sn = overlap ? wk.side : s;
    auto near = [&]() -> hipError_t {
        hipError_t r;
        if ((r = mark(4, sn)) != hipSuccess) return r;
        bool ok = false;
        switch (a.d) {
        case 3: ok = run_near_d<3, T, NC>(a, src, zacc, sn); break;
        case 4: ok = run_near_d<4, T, NC>(a, src, zacc, sn); break;
        case 5: ok = run_near_d<5, T, NC>(a, src, zacc, sn); break;
        default: break;
        }
        if (!ok) return hipErrorInvalidValue;
        return mark(5, sn);
    };
    if (overlap) {
        if ((e = hipEventRecord(wk.fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(wk.side, wk.fork, 0)) != hipSuccess) return e;
        if ((e = near()) != hipSuccess) return e;
        if ((e = hipEventRecord(wk.join, wk.side)) != hipSuccess) return e;
    }
    if (a.nslots > 0 && !launch_s2m(a, wk, prec, s, NC)) return hipErrorInvalidValue;
    if ((e = mark(2, s)) != hipSuccess) return e;
    if (a.nslots > 0 && !launch_m2t(a.kind, a, wk, prec, s, NC)) return hipErrorInvalidValue;
    if ((e = mark(3, s)) != hipSuccess) return e;
    if (overlap) {
        if ((e = hipStreamWaitEvent(s, wk.join, 0)) != hipSuccess) return e;
    } else if ((e = near()) != hipSuccess) {
        return e;
    }
    hipLaunchKernelGGL((k_scatter<T, NC>), gg, gb, 0, s, a.n, a.perm, (const T*)zacc, y, nrhs, col, ncols);
    if ((e = mark(6, s)) != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace

bool launch_fused(int kind, const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc, double c0,
                  double c1, double scale)
{
    switch (kind) {
    case 0: return launch_fused_kind0(a, wk, prec, s, nc, c0, c1, scale);
    case 1: return launch_fused_kind1(a, wk, prec, s, nc, c0, c1, scale);
    case 2: return launch_fused_kind2(a, wk, prec, s, nc, c0, c1, scale);
    case 3: return launch_fused_kind3(a, wk, prec, s, nc, c0, c1, scale);
    case 4: return launch_fused_kind4(a, wk, prec, s, nc, c0, c1, scale);
    case 5: return launch_fused_kind5(a, wk, prec, s, nc, c0, c1, scale);
    case 6: return launch_fused_kind6(a, wk, prec, s, nc, c0, c1, scale);
    default: return false;
    }
}

bool launch_s2m(const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc)
{
    switch (a.d * 2 + (prec == 1 ? 1 : 0)) {
    case 6: return launch_s2m_d3_p0(a, wk, s, nc);
    case 7: return launch_s2m_d3_p1(a, wk, s, nc);
    case 8: return launch_s2m_d4_p0(a, wk, s, nc);
    case 9: return launch_s2m_d4_p1(a, wk, s, nc);
    case 10: return launch_s2m_d5_p0(a, wk, s, nc);
    case 11: return launch_s2m_d5_p1(a, wk, s, nc);
    default: return false;
    }
}

void near_consts_f32(const DevPlan& a, float& c0, float& c1) { near_consts<float>(a, c0, c1); }

hipError_t launch_s2m_column(const DevPlan& a, const DevWork& wk, const void* xv, int nrhs, int col, int prec,
                             hipStream_t s)
{
    if (prec != 1) return hipErrorInvalidValue;
    const float* x = (const float*)xv;
    float* src = (float*)wk.src;
    float* zacc = (float*)wk.zacc;
    const dim3 gg((a.n + 255) / 256), gb(256);
    switch (a.d) {
    case 3: hipLaunchKernelGGL((k_gather<3, float>), gg, gb, 0, s, a.n, a.perm, a.pts32, x, nrhs, col, 1, src, zacc, nullptr); break;
    case 4: hipLaunchKernelGGL((k_gather<4, float>), gg, gb, 0, s, a.n, a.perm, a.pts32, x, nrhs, col, 1, src, zacc, nullptr); break;
    case 5: hipLaunchKernelGGL((k_gather<5, float>), gg, gb, 0, s, a.n, a.perm, a.pts32, x, nrhs, col, 1, src, zacc, nullptr); break;
    default: return hipErrorInvalidValue;
    }
    if (a.nslots > 0 && !launch_s2m(a, wk, 1, s)) return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_far_column(const DevPlan& a, const DevWork& wk, const void* xv, int nrhs, int col, int prec,
                             hipStream_t s)
{
    if (prec != 1) return hipErrorInvalidValue;
    const float* x = (const float*)xv;
    float* src = (float*)wk.src;
    float* zacc = (float*)wk.zacc;
    const dim3 gg((a.n + 255) / 256), gb(256);
    switch (a.d) {
    case 3: hipLaunchKernelGGL((k_gather<3, float>), gg, gb, 0, s, a.n, a.perm, a.pts32, x, nrhs, col, 1, src, zacc, nullptr); break;
    case 4: hipLaunchKernelGGL((k_gather<4, float>), gg, gb, 0, s, a.n, a.perm, a.pts32, x, nrhs, col, 1, src, zacc, nullptr); break;
    case 5: hipLaunchKernelGGL((k_gather<5, float>), gg, gb, 0, s, a.n, a.perm, a.pts32, x, nrhs, col, 1, src, zacc, nullptr); break;
    default: return hipErrorInvalidValue;
    }
    if (a.nslots > 0) {
        if (!launch_s2m(a, wk, 1, s)) return hipErrorInvalidValue;
        if (!launch_m2t(a.kind, a, wk, 1, s)) return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int far_max_order(int d)
{
    switch (d) {
    case 3: return PMax<3>::value;
    case 4: return PMax<4>::value;
    case 5: return PMax<5>::value;
    default: return -1;
    }
}

bool far_supported(int d, int p) { return p >= 0 && p <= far_max_order(d); }

hipError_t launch_mvm_column(const DevPlan& a, const DevWork& wk, const void* x, void* y, int nrhs, int col,
                             int ncols, int nc, int prec, hipStream_t s, bool overlap, hipEvent_t* ev)
{
    if (ncols < 1 || ncols > nc || nc > wk.ncmax || col < 0 || col + ncols > nrhs) return hipErrorInvalidValue;
    if (nc == 1) {
        if (prec == 1) return mvm_pass<float, 1>(a, wk, (const float*)x, (float*)y, nrhs, col, 1, s, overlap, ev);
        return mvm_pass<double, 1>(a, wk, (const double*)x, (double*)y, nrhs, col, 1, s, overlap, ev);
    }
    if (nc != kMvmCols || (a.nslots > 0 && a.nnjobs <= 0)) return hipErrorInvalidValue;
    if (prec == 1)
        return mvm_pass<float, kMvmCols>(a, wk, (const float*)x, (float*)y, nrhs, col, ncols, s, overlap, ev);
    return mvm_pass<double, kMvmCols>(a, wk, (const double*)x, (double*)y, nrhs, col, ncols, s, overlap, ev);
}

}  // namespace fkt
