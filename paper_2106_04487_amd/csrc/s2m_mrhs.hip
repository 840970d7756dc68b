// Moments of a group of 32 right-hand sides on the matrix cores (FP32
// plans), one object per dimension (FKT_S2M_D, set when compiling).
//
// The moments of node b (Algorithm 1, source2mult) are M_b[e][c] =
// sum_s B_e(s) x_s[c], with B_e(s) the normalised solid harmonic of entry e
// times the radial power of source s (the same factors as the one-column
// s2m, without the weight). For 32 columns that is an (entries x points) by
// (points x 32) product, so the basis is generated once per source for all
// columns and the contraction runs as FP32 MFMA (v_mfma_f32_16x16x4f32).
//
// Work units are those of the one-column s2m (at most 1024 points of one
// node); one wave per (unit, chunk of at most 128 entries). For every 64
// points each lane generates its point's entries of the chunk and stores them
// into an LDS block of 32 entries x 64 points; every 32 entries the wave
// multiplies the block by the 64 x 32 weights of the points (held in
// registers as MFMA B fragments) into per-chunk accumulators. Units of nodes
// split over several units write partial moments, summed in unit order by
// k_s2m_reduce_mr.
#include <hip/hip_runtime.h>

#include "fkt_kernels.h"
#include "fkt_mrhs.h"

#if !defined(FKT_S2M_D)
#error "compile with -DFKT_S2M_D=<3|4|5>"
#endif
#define FKT_CAT2(a, b) a##b
#define FKT_CAT(a, b) FKT_CAT2(a, b)

namespace fkt {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kMrChunk = 128;  // moment entries per wave and launch
constexpr int kBtStride = 68;  // LDS row stride (floats): 16-byte reads of 16 rows spread over the banks

// Orders this wave's LDS writes before its later LDS reads and back (the
// block is one wave, whose LDS operations complete in issue order; only the
// compiler has to be kept from moving accesses across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fragment layouts of v_mfma_f32_16x16x4f32 (checked on the device): lane l
// holds A[l % 16][l / 16], B[l / 16][l % 16] and D[4 (l / 16) + r][l % 16].
// Here A = basis (16 entries x 4 points), B = weights (4 points x 16 columns).
// Point 4 ks + l / 16 of a 64-point group is k-step ks of lane group l / 16;
// the LDS block keeps point p in column 16 (p % 4) + p / 4, so the 16 k-steps
// a lane needs are 16 consecutive floats of its entry's row.
template <int D, int P, int C0, int C1>
__global__ __launch_bounds__(kWave) void k_s2m_mrhs(const DevPlan a, const float* __restrict__ X32,
                                                    float* __restrict__ mom, float* __restrict__ part32,
                                                    int64_t npart)
{
    constexpr int R = cbinom(P + D, D);
    constexpr int CH = C1 - C0;
    constexpr int ET = (CH + 15) / 16;  // row tiles of 16 entries
    static_assert(CH > 0 && CH <= kMrChunk, "chunk size");
    __shared__ __attribute__((aligned(16))) float Bt[32][kBtStride];
    const int u = blockIdx.x;
    const int lane = threadIdx.x, r16 = lane & 15, g4 = lane >> 4;
    const int slot = a.unit_slot[u];
    const int beg = a.unit_begin[u], end = a.unit_end[u];
    double c[D];
#pragma unroll
    for (int i = 0; i < D; ++i) c[i] = a.slot_ctr[slot * D + i];
    const double is = 1.0 / a.slot_scale[slot];
    const float* __restrict__ hn2 = a.hn32;
    const int pcol = 16 * (lane & 3) + (lane >> 2);  // LDS column of this lane's point
    // rows of a last, partial block that no entry writes must hold finite values
    for (int i = lane; i < 32 * kBtStride; i += kWave) (&Bt[0][0])[i] = 0.f;

    f4 acc[ET][2];
#pragma unroll
    for (int et = 0; et < ET; ++et)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[et][ct] = f4{0.f, 0.f, 0.f, 0.f};

    for (int g0 = beg; g0 < end; g0 += kWave) {
        // B fragments: weights of point g0 + 4 ks + g4, column 16 ct + r16
        float xb[2][16];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int p = g0 + 4 * ks + g4;
            const float* xr = X32 + (size_t)min(p, end - 1) * kMrCols;
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) xb[ct][ks] = p < end ? xr[16 * ct + r16] : 0.f;
        }
        // this lane's point (past the unit's end: its last point, weight 0)
        const int sp = min(g0 + lane, end - 1);
        const float* __restrict__ hnl = opaque(hn2);
        float x[D], rho2[D + 1];
        rho2[0] = 0.f;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            x[i] = (float)((a.pts64[(size_t)sp * D + i] - c[i]) * is);
            rho2[i + 1] = rho2[i] + x[i] * x[i];
        }
        float q[P / 2 + 1];
        q[0] = 1.f;
#pragma unroll
        for (int i = 1; i <= P / 2; ++i) q[i] = q[i - 1] * rho2[D];

        // contract the block of entries [C0 + 32 sub, C0 + 32 sub + 32)
        auto flush = [&](auto subc) {
            constexpr int sub = decltype(subc)::value;
            wave_lds_sync();
#pragma unroll
            for (int et2 = 0; et2 < 2; ++et2) {
                const int et = 2 * sub + et2;
                if (et < ET) {
                    const float* row = &Bt[16 * et2 + r16][16 * g4];
                    f4 av[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) av[v] = *(const f4*)(row + 4 * v);
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                        for (int ks = 0; ks < 16; ++ks)
                            acc[et][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks / 4][ks % 4], xb[ct][ks],
                                                                               acc[et][ct], 0, 0, 0);
                }
            }
            wave_lds_sync();
        };
        int off = 0;
        auto emit = [&](auto kc, float v) {
            constexpr int k = decltype(kc)::value;
            constexpr int nj = nj_of(P, k);
            auto put = [&](auto jc) {
                constexpr int jj = decltype(jc)::value;
                const int idx = off + jj;
                if (idx >= C0 && idx < C1) {
                    const int e = idx - C0;
                    Bt[e % 32][pcol] = v * q[jj];
                    if (e % 32 == 31) {
                        switch (e / 32) {
                        case 0: flush(std::integral_constant<int, 0>{}); break;
                        case 1: flush(std::integral_constant<int, 1>{}); break;
                        case 2: flush(std::integral_constant<int, 2>{}); break;
                        default: flush(std::integral_constant<int, 3>{}); break;
                        }
                    }
                }
            };
            static_for<0, nj>(put);
            off += nj;
        };
        harmonics<D, P, true, float>(x, rho2, hnl, emit);
        if constexpr (CH % 32 != 0) {
            // last, partial block: its rows past the chunk feed only output
            // rows that are not stored
            flush(std::integral_constant<int, CH / 32>{});
        }
    }

    // D rows are entries 16 et + 4 g4 + r, columns 16 ct + r16
    const int dst = a.unit_dst[u];
#pragma unroll
    for (int et = 0; et < ET; ++et)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = 16 * et + 4 * g4 + r;
            if (e < CH) {
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    const int col = 16 * ct + r16;
                    float* out = dst >= 0 ? mom + ((size_t)col * a.nslots + dst) * R
                                          : part32 + ((size_t)col * npart + (-1 - dst)) * R;
                    out[C0 + e] = acc[et][ct][r];
                }
            }
        }
}

// moments of nodes split over several units: ordered sums of the partials,
// for the 32 columns
__global__ __launch_bounds__(256) void k_s2m_reduce_mr(int nred, int R, int nslots, int64_t npart,
                                                       const int* __restrict__ red_slot,
                                                       const int* __restrict__ red_off,
                                                       const float* __restrict__ part32, float* __restrict__ mom)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per = (int64_t)nred * R;
    if (g >= per * kMrCols) return;
    const int col = (int)(g / per);
    const int r = (int)((g % per) / R), i = (int)(g % R);
    float s = 0.f;
    for (int q = red_off[r]; q < red_off[r + 1]; ++q) s += part32[((size_t)col * npart + q) * R + i];
    mom[((size_t)col * nslots + red_slot[r]) * R + i] = s;
}

template <int D, int P, int C0>
void launch_chunks(const DevPlan& a, const DevMrhs& mr, hipStream_t s)
{
    constexpr int R = cbinom(P + D, D);
    if constexpr (C0 < R) {
        constexpr int C1 = (C0 + kMrChunk < R) ? C0 + kMrChunk : R;
        hipLaunchKernelGGL((k_s2m_mrhs<D, P, C0, C1>), dim3(a.nunits), dim3(kWave), 0, s, a,
                           (const float*)mr.x32, (float*)mr.mom, (float*)mr.part32, mr.npart);
        launch_chunks<D, P, C1>(a, mr, s);
    }
}

template <int D, int P = 0>
bool launch_dp(const DevPlan& a, const DevMrhs& mr, hipStream_t s)
{
    if constexpr (P > PMax<D>::value) {
        return false;
    } else {
        if (a.p == P) {
            launch_chunks<D, P, 0>(a, mr, s);
            if (a.nred > 0) {
                const int64_t tot = (int64_t)a.nred * a.rank * kMrCols;
                hipLaunchKernelGGL(k_s2m_reduce_mr, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a.nred,
                                   a.rank, a.nslots, mr.npart, a.red_slot, a.red_off, (const float*)mr.part32,
                                   (float*)mr.mom);
            }
            return true;
        }
        return launch_dp<D, P + 1>(a, mr, s);
    }
}

}  // namespace

bool FKT_CAT(launch_s2m_mrhs_d, FKT_S2M_D)(const DevPlan& a, const DevMrhs& mr, hipStream_t s)
{
    if (a.d != FKT_S2M_D || a.nunits == 0) return a.nunits == 0;
    return launch_dp<FKT_S2M_D>(a, mr, s);
}

}  // namespace fkt
