// Far field of a group of 32 right-hand sides on the matrix cores (FP32
// plans), one object per kernel kind (FKT_M2T_KIND, set when compiling).
//
// For a (target, far node) pair the multipole-to-target step is a dot
// product of the pair's basis vector b (entries Y_kh(r^) (s/|r|)^j F_kj(|r|),
// the same factors as the one-column kernel) with the node's moments, so
// for 32 columns it is a (pairs x rank) by (rank x 32) product. The far
// pairs of a group of consecutive 64-target blocks are packed by node into
// jobs of 64 pairs of up to kMrJobNodes nodes (lanes grouped by node), so a
// node's moment fragments, which dominate the memory traffic, serve as many
// rows as possible. One wave walks a unit of a group's jobs: each lane
// generates its pair's basis entries in emission order and writes them,
// split into bf16 high and low parts, into an LDS chunk laid out as MFMA A
// fragments; every 32 entries the chunk is multiplied by each job node's
// moments (bf16 high/low B fragments prepared once per group of columns)
// with v_mfma_f32_16x16x32_bf16, three products per tile (hi*hi + hi*lo +
// lo*hi: about 16 bits of mantissa), rows of other nodes masked to zero.
// Each job's rows are then added into the far-field buffer (target-major,
// cleared beforehand) by atomic adds, 16 consecutive columns per row and
// instruction. Units hold a fixed number of jobs, so heavy groups spread
// over the machine instead of leaving a tail at the end of the launch.
#include <hip/hip_runtime.h>

#include "fkt_kernels.h"
#include "fkt_mrhs.h"

#ifndef FKT_M2T_KIND
#error "compile with -DFKT_M2T_KIND=<fkt_kernel_kind value>"
#endif
#define FKT_CAT2(a, b) a##b
#define FKT_CAT(a, b) FKT_CAT2(a, b)

namespace fkt {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kKC = 32;         // basis entries per LDS chunk (16 KB of LDS with the sums)
constexpr int kKS = kKC / 32;    // MFMA k-steps of 32 per chunk

// Three waves per SIMD (at most 168 registers): at d = 5, p = 8 this spills
// about 45 registers to scratch and still measured 4 % faster than two waves.
template <int D, int P, int KIND>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_m2t_mrhs(const DevPlan a, const DevMrhs mr, const bf8* __restrict__ Bhi,
                                                    const bf8* __restrict__ Blo, int KS, float* __restrict__ zf)
{
    constexpr int R = cbinom(P + D, D);
    constexpr int RP = (R + kKC - 1) / kKC * kKC;
    constexpr int NF = f_off(P, P + 1);
    __shared__ bf8 Ahi[4][kKS][kWave];  // [row tile][k-step in chunk][fragment lane]
    __shared__ bf8 Alo[4][kKS][kWave];
    const int grp = blockIdx.x, lane = threadIdx.x, r16 = lane & 15;
    const int jb = mr.job_off[grp] + (int)blockIdx.y * mr.job_seg, je = mr.job_off[grp + 1];
    if (jb >= je) return;  // whole-wave exit: this unit has no jobs
    const int q0 = grp * mr.job_group;

    const int j1 = min(je, jb + mr.job_seg);
    for (int j = jb; j < j1; ++j) {
        const int n0 = mr.job_noff[j], nn = mr.job_noff[j + 1] - n0;
        const unsigned pw = mr.job_pairs[(size_t)j * kWave + lane];
        const bool valid = pw != 0xffffu;
        const int ni = valid ? (int)(pw >> 12) : 0;
        const int tgt = valid ? a.blk_begin[q0 + ((pw >> 6) & 63)] + (int)(pw & 63) : -1;
        // lane k < nn holds the slot of job node k, read back with readlane
        const int jslot = mr.job_nodes[n0 + min(lane, nn - 1)];
        const int slot = __shfl(jslot, ni, kWave);
        double txl[D];
#pragma unroll
        for (int i = 0; i < D; ++i) txl[i] = valid ? a.pts64[(size_t)tgt * D + i] : 0.0;

        // geometry and radial factors of this lane's pair (FP64), as in k_m2t
        double r[D], r2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            r[i] = valid ? txl[i] - a.slot_ctr[(size_t)slot * D + i] : (i == 0 ? 1.0 : 0.0);
            r2 = fma(r[i], r[i], r2);
        }
        const double ir = rsqrt_pos(r2);
        const double rr = r2 * ir;
        float x[D], rho2[D + 1];
        rho2[0] = 0.f;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            x[i] = (float)(r[i] * ir);
            rho2[i + 1] = rho2[i] + x[i] * x[i];
        }
        rho2[D] = 1.f;
        float rad[NF];
        {
            double Dm[P + 1];
            radial_derivs<KIND, P>(a, rr, Dm);
            double um[P + 1];
            um[0] = Dm[0];
            double rp = 1.0;
#pragma unroll
            for (int m = 1; m <= P; ++m) {
                rp *= rr;
                um[m] = Dm[m] * rp;
            }
            const double v = a.slot_scale[slot] * ir;
            double vp[P + 1];
            vp[0] = 1.0;
#pragma unroll
            for (int jp = 1; jp <= P; ++jp) vp[jp] = vp[jp - 1] * v;
            auto radial_k = [&](auto kc) {
                constexpr int k = decltype(kc)::value;
                auto radial_j = [&](auto jc) {
                    constexpr int jj = decltype(jc)::value;
                    constexpr int jv = k + 2 * jj;
                    double f = (jv == 0) ? um[0] : 0.0;
                    auto term = [&](auto mc) {
                        constexpr int m = decltype(mc)::value + 1;
                        constexpr double c = cx_tbar(D, k, jv, m);
                        f = fma(um[m], c, f);
                    };
                    static_for<0, jv>(term);
                    rad[f_off(P, k) + jj] = valid ? (float)(vp[jv] * f) : 0.f;
                };
                static_for<0, nj_of(P, k)>(radial_j);
            };
            static_for<0, P + 1>(radial_k);
        }

        f4 acc[4][2];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};
        // contract the chunk holding entries [kbase, kbase + kKC) with every node
        auto flush = [&](int kbase) {
            __syncthreads();
            const int ks0 = kbase / 32;
#pragma unroll 1
            for (int k = 0; k < nn; ++k) {
                const uint64_t nm = __ballot(valid && ni == k);
                const int sl = __builtin_amdgcn_readlane(jslot, k);
#pragma unroll
                for (int ks = 0; ks < kKS; ++ks) {
                    const size_t fb = ((size_t)sl * KS + ks0 + ks) * 2 * kWave;
                    const bf8 bh0 = Bhi[fb + lane], bh1 = Bhi[fb + kWave + lane];
                    const bf8 bl0 = Blo[fb + lane], bl1 = Blo[fb + kWave + lane];
#pragma unroll
                    for (int rt = 0; rt < 4; ++rt) {
                        if (((nm >> (16 * rt)) & 0xffffull) == 0) continue;
                        const bool mine = (nm >> (16 * rt + r16)) & 1ull;
                        const bf8 z = {};
                        const bf8 ah = mine ? Ahi[rt][ks][lane] : z;
                        const bf8 al = mine ? Alo[rt][ks][lane] : z;
                        acc[rt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh0, acc[rt][0], 0, 0, 0);
                        acc[rt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl0, acc[rt][0], 0, 0, 0);
                        acc[rt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh0, acc[rt][0], 0, 0, 0);
                        acc[rt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh1, acc[rt][1], 0, 0, 0);
                        acc[rt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl1, acc[rt][1], 0, 0, 0);
                        acc[rt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh1, acc[rt][1], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        };
        // entry idx of this lane's row goes to fragment lane (lane % 16) + 16 g,
        // element q, of row tile lane / 16, with g = (idx % 32) / 8, q = idx % 8;
        // eight consecutive entries are collected and stored as one vector.
        // Entries are converted two at a time: the high parts of a pair by one
        // packed conversion (round to nearest even), unpacked to FP32 by a
        // shift and a mask, then the low parts (value minus high part) by a
        // second packed conversion.
        typedef float f2 __attribute__((ext_vector_type(2)));
        typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        u4 hw, lw;
        float ev = 0.f;
        auto put = [&](int idx, float bv) {
            const int c = idx % kKC, ks = c / 32, g = (c % 32) / 8, q = c % 8;
            if (q % 2 == 0) {
                ev = bv;
            } else {
                const bf2 hp = __builtin_convertvector(f2{ev, bv}, bf2);
                const unsigned hu = __builtin_bit_cast(unsigned, hp);
                const float h0 = __builtin_bit_cast(float, hu << 16), h1 = __builtin_bit_cast(float, hu & 0xffff0000u);
                const bf2 lp = __builtin_convertvector(f2{ev - h0, bv - h1}, bf2);
                hw[q / 2] = hu;
                lw[q / 2] = __builtin_bit_cast(unsigned, lp);
            }
            if (q == 7) {
                Ahi[lane >> 4][ks][r16 + 16 * g] = __builtin_bit_cast(bf8, hw);
                Alo[lane >> 4][ks][r16 + 16 * g] = __builtin_bit_cast(bf8, lw);
            }
            if (c == kKC - 1) flush(idx - (kKC - 1));
        };
        int off = 0;
        auto emit = [&](auto kc, float yv) {
            constexpr int k = decltype(kc)::value;
            constexpr int nj = nj_of(P, k);
            auto one = [&](auto jc) {
                constexpr int jj = decltype(jc)::value;
                put(off + jj, yv * rad[f_off(P, k) + jj]);
            };
            static_for<0, nj>(one);
            off += nj;
        };
        harmonics<D, P, false, float>(x, rho2, (const float*)nullptr, emit);
        auto pad = [&](auto ic) {
            constexpr int idx = R + decltype(ic)::value;
            put(idx, 0.f);
        };
        static_for<0, RP - R>(pad);

        // pair rows into the far field: C layout of a 16 x 16 tile, lane l,
        // entry q -> row 4 (l / 16) + q, column l % 16
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * rt + 4 * (lane >> 4) + q;
                const int trow = __shfl(tgt, row, kWave);
                if (trow >= 0)
#pragma unroll
                    for (int ct = 0; ct < 2; ++ct)
                        unsafeAtomicAdd(zf + (size_t)trow * kMrCols + 16 * ct + r16, acc[rt][ct][q]);
            }
    }
}

template <int D, int P = 0>
bool launch_d(const DevPlan& a, const DevMrhs& mr, hipStream_t s)
{
    if constexpr (P > PMax<D>::value) {
        return false;
    } else {
        if (a.p == P) {
            hipLaunchKernelGGL((k_m2t_mrhs<D, P, FKT_M2T_KIND>), dim3(mr.ngroups, mr.job_nseg), dim3(kWave), 0, s, a, mr,
                               (const bf8*)mr.bhi, (const bf8*)mr.blo, mr.ks, (float*)mr.zf);
            return true;
        }
        return launch_d<D, P + 1>(a, mr, s);
    }
}

}  // namespace

bool FKT_CAT(launch_m2t_mrhs_kind, FKT_M2T_KIND)(const DevPlan& a, const DevMrhs& mr, hipStream_t s)
{
    switch (a.d) {
    case 3: return launch_d<3>(a, mr, s);
    case 4: return launch_d<4>(a, mr, s);
    case 5: return launch_d<5>(a, mr, s);
    default: return false;
    }
}

}  // namespace fkt
