// Many right-hand sides (groups of 32 columns, FP32 plans): the near field on
// the matrix cores (this file); the moments (s2m_mrhs.hip) and the far-field
// evaluation (m2t_mrhs.hip) of the 32 columns on the matrix cores too.
//
// Near field (Algorithm 1, near_mat, for 32 columns at once): one wave takes
// a 64-target block and up to 32 leaves of the union of its targets' near
// leaves (a block's leaves are cut into such units so that heavy blocks do
// not leave a tail at the end of the launch). For
// every 32 points of a leaf each lane evaluates 32 kernel values (4 row
// tiles of 16 targets x 8 points; rows whose target does not have the leaf
// in its own near set get 0), and the 64 x 32 block of K times the 32 x 32
// block of weights is accumulated by MFMA: v_mfma_f32_16x16x32_bf16 (kernel
// values and weights rounded to bf16, FP32 accumulation) or
// v_mfma_f32_16x16x4f32 (FP32 throughout). Lane l of a 16 x 16 tile holds
// row l % 16 and points 8 (l / 16) .. + 7 of the 32, for both variants (the
// points are a reduction index, so the order within a step is free). The
// unit's 64 x 32 result is added atomically into the group's far-field
// buffer (target-major, 16 consecutive columns per row and instruction),
// which a last kernel writes to y in the caller's order.
//
// Leaves are laid out padded to multiples of 32 points (pad weight 0,
// coordinates of the leaf's first point), so every step loads aligned runs.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fkt_kernels.h"
#include "fkt_mrhs.h"

namespace fkt {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// XT[c][p] = x[perm[src[p]]][col0 + c] (0 on padding), c < 32
template <typename TC>
__global__ __launch_bounds__(256) void k_mr_gather(int npad, const int* __restrict__ src,
                                                   const int64_t* __restrict__ perm, const float* __restrict__ x,
                                                   int nrhs, int col0, TC* __restrict__ XT)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npad) return;
    const int s = src[p];
    const float* xr = s >= 0 ? x + perm[s] * nrhs + col0 : nullptr;
#pragma unroll 8
    for (int c = 0; c < kMrCols; ++c) XT[(size_t)c * npad + p] = (TC)(xr ? xr[c] : 0.f);
}

// p[0, n) = 0 (a kernel, not a memset node, so the MVM stays capturable)
__global__ __launch_bounds__(256) void k_mr_zero(int64_t n, float* __restrict__ p)
{
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (int64_t)gridDim.x * 256) p[g] = 0.f;
}

// X32[i][c] = x[perm[i]][col0 + c]: the group's weights in tree order
__global__ __launch_bounds__(256) void k_mr_xgather(int n, const int64_t* __restrict__ perm,
                                                    const float* __restrict__ x, int nrhs, int col0,
                                                    float* __restrict__ X32)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)n * kMrCols) return;
    const int64_t i = g / kMrCols;
    const int c = (int)(g % kMrCols);
    X32[g] = x[perm[i] * nrhs + col0 + c];
}

// B fragments of the moments: for node slot s, k-step t (32 entries) and
// column tile ct, lane l holds entries k = 32 t + 8 (l / 16) + q, q < 8, of
// column 16 ct + l % 16, split into bf16 high and low parts (0 past rank)
__global__ __launch_bounds__(256) void k_mom_frag(int nslots, int R, int KS, const float* __restrict__ mom,
                                                  bf8* __restrict__ bhi, bf8* __restrict__ blo)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)nslots * KS * 2 * kWave;
    if (g >= total) return;
    const int lane = (int)(g % kWave);
    const int ct = (int)((g / kWave) % 2);
    const int t = (int)((g / (2 * kWave)) % KS);
    const int64_t sl = g / (2 * (int64_t)kWave * KS);
    const int col = 16 * ct + (lane & 15);
    const float* mc = mom + ((size_t)col * nslots + sl) * R;
    bf8 h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = 32 * t + 8 * (lane >> 4) + q;
        const float v = k < R ? mc[k] : 0.f;
        h[q] = (__bf16)v;
        l[q] = (__bf16)(v - (float)h[q]);
    }
    bhi[g] = h;
    blo[g] = l;
}

bool launch_m2t_mrhs(const DevPlan& a, const DevMrhs& mr, hipStream_t s)
{
    switch (a.kind) {
    case 0: return launch_m2t_mrhs_kind0(a, mr, s);
    case 1: return launch_m2t_mrhs_kind1(a, mr, s);
    case 2: return launch_m2t_mrhs_kind2(a, mr, s);
    case 3: return launch_m2t_mrhs_kind3(a, mr, s);
    case 4: return launch_m2t_mrhs_kind4(a, mr, s);
    case 5: return launch_m2t_mrhs_kind5(a, mr, s);
    case 6: return launch_m2t_mrhs_kind6(a, mr, s);
    default: return false;
    }
}

template <int D, int KIND, typename TC>
__global__ __launch_bounds__(kWave) void k_near_mrhs(const DevPlan a, const DevMrhs mr, const TC* __restrict__ XT,
                                                     float* __restrict__ zf, float c0, float c1, float scale)
{
    using NK = NearKernel<KIND, float>;
    constexpr bool kBf16 = std::is_same<TC, __bf16>::value;
    const int blk = blockIdx.x, lane = threadIdx.x;
    const int r16 = lane & 15, g = lane >> 4;
    // this unit's near leaves of the block
    const int e0 = mr.near_off[blk] + (int)blockIdx.y * mr.near_seg;
    const int e1 = min(mr.near_off[blk + 1], e0 + mr.near_seg);
    if (e0 >= e1) return;  // whole-wave exit
    const int tb = a.blk_begin[blk], cnt = a.blk_count[blk];
    float tx[4][D];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const int row = rt * 16 + r16;
        const int t = tb + (row < cnt ? row : 0);
#pragma unroll
        for (int k = 0; k < D; ++k) tx[rt][k] = a.pts32[(size_t)t * D + k];
    }
    f4 acc[4][2];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};

    for (int e = e0; e < e1; ++e) {
        const uint64_t mask = mr.near_mask[e];
        float flag[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) flag[rt] = (float)((mask >> (rt * 16 + r16)) & 1ull);
        const int pb = mr.near_pbeg[e], pe = pb + mr.near_pcnt[e];
        for (int s0 = pb; s0 < pe; s0 += 32) {
            const int sp = s0 + 8 * g;  // this lane's 8 points
            float sx[D][8];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const f4 u0 = *(const f4*)(mr.pts + (size_t)k * mr.npad + sp);
                const f4 u1 = *(const f4*)(mr.pts + (size_t)k * mr.npad + sp + 4);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sx[k][q] = u0[q];
                    sx[k][q + 4] = u1[q];
                }
            }
            if constexpr (kBf16) {
                bf8 b[2];
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) b[ct] = *(const bf8*)(XT + (size_t)(ct * 16 + r16) * mr.npad + sp);
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    bf8 av;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        float d2 = 0.f;
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const float w = tx[rt][k] - sx[k][q];
                            d2 = fmaf(w, w, d2);
                        }
                        av[q] = (__bf16)(flag[rt] * NK::eval(d2, c0, c1, nullptr));
                    }
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[ct], acc[rt][ct], 0, 0, 0);
                }
            } else {
                float b[2][8];
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    const float* xp = (const float*)XT + (size_t)(ct * 16 + r16) * mr.npad + sp;
                    const f4 u0 = *(const f4*)xp, u1 = *(const f4*)(xp + 4);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        b[ct][q] = u0[q];
                        b[ct][q + 4] = u1[q];
                    }
                }
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        float d2 = 0.f;
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            const float w = tx[rt][k] - sx[k][q];
                            d2 = fmaf(w, w, d2);
                        }
                        const float kv = flag[rt] * NK::eval(d2, c0, c1, nullptr);
#pragma unroll
                        for (int ct = 0; ct < 2; ++ct)
                            acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv, b[ct][q], acc[rt][ct], 0, 0, 0);
                    }
            }
        }
    }
    // C layout of a 16 x 16 tile: lane l, entry r -> row 4 (l / 16) + r, column l % 16
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rt * 16 + 4 * g + r, col = ct * 16 + r16;
                if (row < cnt) unsafeAtomicAdd(zf + (size_t)(tb + row) * kMrCols + col, scale * acc[rt][ct][r]);
            }
}

// y[perm[t]][col0 + c] = zf[t][c]: near plus far field of the group, to the
// caller's order
__global__ __launch_bounds__(256) void k_mr_out(int n, const int64_t* __restrict__ perm, const float* __restrict__ zf,
                                                float* __restrict__ y, int nrhs, int col0)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)n * kMrCols) return;
    const int64_t t = g / kMrCols;
    const int c = (int)(g % kMrCols);
    y[perm[t] * nrhs + col0 + c] = zf[g];
}

template <int D, typename TC>
bool launch_near_mrhs_d(const DevPlan& a, const DevMrhs& mr, const TC* XT, float* zf, hipStream_t s)
{
    float c0, c1;
    near_consts_f32(a, c0, c1);
    const float scale = (float)a.var;
    switch (a.kind) {
#define FKT_MR_CASE(K) \
    case K: hipLaunchKernelGGL((k_near_mrhs<D, K, TC>), dim3(a.nblocks, mr.near_nseg), dim3(kWave), 0, s, a, mr, XT, \
                               zf, c0, c1, scale); return true;
        FKT_MR_CASE(FKT_GAUSSIAN)
        FKT_MR_CASE(FKT_EXPONENTIAL)
        FKT_MR_CASE(FKT_MATERN32)
        FKT_MR_CASE(FKT_MATERN52)
        FKT_MR_CASE(FKT_RATQUAD)
        FKT_MR_CASE(FKT_CAUCHY)
        FKT_MR_CASE(FKT_LAPLACE)
#undef FKT_MR_CASE
    default: return false;
    }
}

template <typename TC>
hipError_t mvm_mrhs_t(const DevPlan& a, const DevWork& wk, const DevMrhs& mr, const float* x, float* y, int nrhs,
                      hipStream_t s)
{
    TC* XT = (TC*)mr.xt;
    float* zf = (float*)mr.zf;
    for (int col0 = 0; col0 < nrhs; col0 += kMrCols) {
        if (mr.mom && a.nslots > 0) {
            // far field of the group on the matrix cores: moments of the 32
            // columns (MFMA s2m), B fragments, then one MFMA multipole-to-
            // target pass that writes zf for all 32 columns
            const int64_t nx = (int64_t)a.n * kMrCols;
            hipLaunchKernelGGL(k_mr_xgather, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, s, a.n, a.perm, x,
                               nrhs, col0, (float*)mr.x32);
            bool ok_s2m = false;
            switch (a.d) {
            case 3: ok_s2m = launch_s2m_mrhs_d3(a, mr, s); break;
            case 4: ok_s2m = launch_s2m_mrhs_d4(a, mr, s); break;
            case 5: ok_s2m = launch_s2m_mrhs_d5(a, mr, s); break;
            default: break;
            }
            if (!ok_s2m) return hipErrorInvalidValue;
            const int64_t nf = (int64_t)a.nslots * mr.ks * 2 * kWave;
            hipLaunchKernelGGL(k_mom_frag, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, a.nslots, a.rank,
                               mr.ks, (const float*)mr.mom, (bf8*)mr.bhi, (bf8*)mr.blo);
            // the far-field units add into zf
            const int64_t nz = (int64_t)a.n * kMrCols;
            hipLaunchKernelGGL(k_mr_zero, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((nz + 255) / 256, 8192))), dim3(256), 0, s,
                               nz, zf);
            if (!launch_m2t_mrhs(a, mr, s)) return hipErrorInvalidValue;
        } else {
            // no far-node slots: no target has a far field
            const int64_t nz = (int64_t)a.n * kMrCols;
            hipLaunchKernelGGL(k_mr_zero, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((nz + 255) / 256, 8192))),
                               dim3(256), 0, s, nz, zf);
        }
        hipLaunchKernelGGL((k_mr_gather<TC>), dim3((mr.npad + 255) / 256), dim3(256), 0, s, mr.npad, mr.src, a.perm, x,
                           nrhs, col0, XT);
        bool ok = false;
        switch (a.d) {
        case 3: ok = launch_near_mrhs_d<3, TC>(a, mr, XT, zf, s); break;
        case 4: ok = launch_near_mrhs_d<4, TC>(a, mr, XT, zf, s); break;
        case 5: ok = launch_near_mrhs_d<5, TC>(a, mr, XT, zf, s); break;
        default: break;
        }
        if (!ok) return hipErrorInvalidValue;
        const int64_t ny = (int64_t)a.n * kMrCols;
        hipLaunchKernelGGL(k_mr_out, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, s, a.n, a.perm, zf, y, nrhs, col0);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mvm_mrhs(const DevPlan& a, const DevWork& wk, const DevMrhs& mr, const float* x, float* y, int nrhs,
                           hipStream_t s)
{
    if (nrhs % kMrCols != 0) return hipErrorInvalidValue;
    return mr.bf16 ? mvm_mrhs_t<__bf16>(a, wk, mr, x, y, nrhs, s) : mvm_mrhs_t<float>(a, wk, mr, x, y, nrhs, s);
}

}  // namespace fkt
