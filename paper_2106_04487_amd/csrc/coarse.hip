// Two-level preconditioning for CG on (K~ + sigma2 I) x = b (project
// addition; the paper solves its Gaussian-process systems through MVMs,
// Sec. 5.3). Per-leaf preconditioners cannot reach the smooth global modes
// that make long-length-scale kernel systems ill-conditioned, so a coarse
// space is added: with k landmark points J, the Nystrom factor
//     L = K(X, X_J) W,   W = chol(K(X_J, X_J) + sigma2 I)^-T,
// approximates K by L L^T, and the Woodbury identity joins it to the
// per-leaf part D^-1 = blockdiag(V_l^T diag(h_l) V_l) of the residual leaf
// blocks R_l = K_ll + sigma2 I - L_l L_l^T = V_l^T diag(lam_l) V_l:
//     P = (L L^T + D)^-1 = V^T (h .* (s - G C^-1 G^T (h .* s))),  s = V r,
// with G = V L (per leaf) and C = I + G^T diag(h) G (k x k). This file
// holds the dense FP64 pieces: the kernel columns, a batched tiled GEMM,
// the tall-skinny matrix-vector products and the host SPD factorisations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <vector>

#include "../../include/fkt.h"
#include "fkt_coarse.h"
#include "fkt_host.h"

namespace fkt {
namespace {

constexpr int kT = 256;

__device__ __forceinline__ double kernel_value_dev(int kind, double ell, double alpha, double var, double r)
{
    switch (kind) {
    case FKT_GAUSSIAN: return var * exp(-r * r / (2.0 * ell * ell));
    case FKT_EXPONENTIAL: return var * exp(-r / ell);
    case FKT_MATERN32: { const double a = 1.7320508075688772935 * r / ell; return var * (1.0 + a) * exp(-a); }
    case FKT_MATERN52: {
        const double a = 2.2360679774997896964 * r / ell;
        return var * (1.0 + a + a * a / 3.0) * exp(-a);
    }
    case FKT_RATQUAD: return var * pow(1.0 + r * r / (2.0 * alpha * ell * ell), -alpha);
    case FKT_CAUCHY: return var / (1.0 + r * r / (ell * ell));
    case FKT_LAPLACE: return r > 0.0 ? var / r : 0.0;
    }
    return 0.0;
}

__global__ __launch_bounds__(kT) void k_kernel_columns(const DevPlan a, const int* __restrict__ cols, int k,
                                                       double* __restrict__ out)
{
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= (int64_t)a.n * k) return;
    const int64_t i = g / k;
    const int j = (int)(g - i * k);
    const int c = cols[j];
    double s = 0.0;
    for (int q = 0; q < a.d; ++q) {
        const double u = a.pts64[i * a.d + q] - a.pts64[(int64_t)c * a.d + q];
        s = fma(u, u, s);
    }
    out[g] = kernel_value_dev(a.kind, a.ell, a.alpha, a.var, sqrt(s));
}

// C = alpha op(A) diag(w) op(B) + beta C per descriptor (grid.z): 64 x 64
// output tiles of 256 threads, 4 x 4 outputs per thread, the contraction in
// steps of 16 staged through LDS; every index is bounds-checked, so M, N, K
// and the leading dimensions are arbitrary.
template <bool TA, bool TB, bool WT>
__global__ __launch_bounds__(kT) void k_gemm64(const Gemm64* __restrict__ desc, const double* __restrict__ A,
                                               const double* __restrict__ B, const double* __restrict__ w,
                                               double* __restrict__ C, double alpha, double beta)
{
    __shared__ double As[16][65];
    __shared__ double Bs[16][65];
    const Gemm64 dsc = desc[blockIdx.z];
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    if (m0 >= dsc.M || n0 >= dsc.N) return;
    const double* __restrict__ Ab = A + dsc.a_off;
    const double* __restrict__ Bb = B + dsc.b_off;
    const double* __restrict__ wb = WT ? w + dsc.w_off : nullptr;
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    for (int p0 = 0; p0 < dsc.K; p0 += 16) {
        // A tile: 64 rows x 16 contraction entries
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + q * kT;              // 0..1023
            int i, p;
            if (TA) { p = e >> 6; i = e & 63; }    // consecutive rows: A[p][i] contiguous in i
            else { i = e >> 4; p = e & 15; }       // consecutive contraction: A[i][p] contiguous in p
            const int gi = m0 + i, gp = p0 + p;
            double v = 0.0;
            if (gi < dsc.M && gp < dsc.K) {
                v = TA ? Ab[(int64_t)gp * dsc.lda + gi] : Ab[(int64_t)gi * dsc.lda + gp];
                if (WT) v *= wb[gp];
            }
            As[p][i] = v;
        }
        // B tile: 16 contraction entries x 64 columns
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + q * kT;
            int j, p;
            if (TB) { j = e >> 4; p = e & 15; }    // B[j][p] contiguous in p
            else { p = e >> 6; j = e & 63; }       // B[p][j] contiguous in j
            const int gj = n0 + j, gp = p0 + p;
            double v = 0.0;
            if (gj < dsc.N && gp < dsc.K) v = TB ? Bb[(int64_t)gj * dsc.ldb + gp] : Bb[(int64_t)gp * dsc.ldb + gj];
            Bs[p][j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            double av[4], bv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) av[r] = As[p][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = Bs[p][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
        }
        __syncthreads();
    }
    double* __restrict__ Cb = C + dsc.c_off;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int gi = m0 + ty * 4 + r;
        if (gi >= dsc.M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int gj = n0 + tx * 4 + c;
            if (gj >= dsc.N) continue;
            double* o = Cb + (int64_t)gi * dsc.ldc + gj;
            *o = beta == 0.0 ? alpha * acc[r][c] : fma(alpha, acc[r][c], beta * *o);
        }
    }
}

// part[chunk][j] = sum over the chunk's rows i of G[i][j] h[i] s[i]
__global__ __launch_bounds__(kT) void k_gemv_t_part(int64_t n, int k, int64_t rows, const double* __restrict__ G,
                                                    const double* __restrict__ h, const double* __restrict__ sv,
                                                    double* __restrict__ part)
{
    const int64_t i0 = (int64_t)blockIdx.x * rows, i1 = min(n, i0 + rows);
    for (int j = threadIdx.x; j < k; j += kT) {
        // four independent accumulators keep four row loads in flight
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int64_t i = i0;
        for (; i + 3 < i1; i += 4) {
            a0 = fma(G[i * k + j], h[i] * sv[i], a0);
            a1 = fma(G[(i + 1) * k + j], h[i + 1] * sv[i + 1], a1);
            a2 = fma(G[(i + 2) * k + j], h[i + 2] * sv[i + 2], a2);
            a3 = fma(G[(i + 3) * k + j], h[i + 3] * sv[i + 3], a3);
        }
        for (; i < i1; ++i) a0 = fma(G[i * k + j], h[i] * sv[i], a0);
        part[(int64_t)j * gridDim.x + blockIdx.x] = (a0 + a1) + (a2 + a3);
    }
}

// u[j] = sum_z part[j][z]: one wave per j, lanes over the chunks
__global__ __launch_bounds__(kT) void k_sum_chunks(int nz, int k, const double* __restrict__ part,
                                                   double* __restrict__ u)
{
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (j >= k) return;
    double s = 0.0;
    for (int z = lane; z < nz; z += 64) s += part[(int64_t)j * nz + z];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) u[j] = s;
}

// out[i] = sum_z part[z][i] (+1 on the diagonal of a k x k matrix when eye_k > 0)
__global__ __launch_bounds__(kT) void k_sum_part64(int nz, int64_t len, const double* __restrict__ part,
                                                   double* __restrict__ out, int eye_k)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * len + i];
    if (eye_k > 0 && (i / eye_k) == (i % eye_k)) s += 1.0;
    out[i] = s;
}

// w = Cinv u: one wave per row
__global__ __launch_bounds__(kT) void k_gemv_small(int k, const double* __restrict__ Cinv, const double* __restrict__ u,
                                                   double* __restrict__ w)
{
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (row >= k) return;
    double s = 0.0;
    for (int j = lane; j < k; j += 64) s = fma(Cinv[(int64_t)row * k + j], u[j], s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) w[row] = s;
}

// y[i] = sv[i] - G[i] . w: one wave per row, w staged in LDS
__global__ __launch_bounds__(kT) void k_gemv_sub(int64_t n, int k, const double* __restrict__ G,
                                                 const double* __restrict__ w, const double* __restrict__ sv,
                                                 double* __restrict__ y)
{
    extern __shared__ double wl[];
    for (int j = threadIdx.x; j < k; j += kT) wl[j] = w[j];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * (kT / 64)) {
        double s = 0.0;
        for (int j = lane; j < k; j += 64) s = fma(G[i * k + j], wl[j], s);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) y[i] = sv[i] - s;
    }
}

unsigned grid_of(int64_t m) { return (unsigned)((m + kT - 1) / kT); }

}  // namespace

hipError_t gemm64_batched(bool ta, bool tb, const Gemm64* desc, int nbatch, int max_m, int max_n, const double* A,
                          const double* B, const double* w, double* C, double alpha, double beta, hipStream_t s)
{
    if (nbatch <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((max_m + 63) / 64), (unsigned)((max_n + 63) / 64), (unsigned)nbatch);
#define FKT_G(TA_, TB_, W_) \
    hipLaunchKernelGGL((k_gemm64<TA_, TB_, W_>), grid, dim3(kT), 0, s, desc, A, B, w, C, alpha, beta)
    if (w) {
        if (ta && !tb) FKT_G(true, false, true);
        else if (!ta && !tb) FKT_G(false, false, true);
        else if (!ta && tb) FKT_G(false, true, true);
        else FKT_G(true, true, true);
    } else {
        if (ta && !tb) FKT_G(true, false, false);
        else if (!ta && !tb) FKT_G(false, false, false);
        else if (!ta && tb) FKT_G(false, true, false);
        else FKT_G(true, true, false);
    }
#undef FKT_G
    return hipGetLastError();
}

hipError_t kernel_columns(const DevPlan& a, const int* cols, int k, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_kernel_columns, dim3(grid_of((int64_t)a.n * k)), dim3(kT), 0, s, a, cols, k, out);
    return hipGetLastError();
}

hipError_t gemv_t_weighted(int64_t n, int k, const double* G, const double* h, const double* sv, double* part,
                           int nchunk, double* u, hipStream_t s)
{
    const int64_t rows = (n + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_gemv_t_part, dim3((unsigned)nchunk), dim3(kT), 0, s, n, k, rows, G, h, sv, part);
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)((k + 3) / 4)), dim3(kT), 0, s, nchunk, k, part, u);
    return hipGetLastError();
}

hipError_t gemv_small(int k, const double* Cinv, const double* u, double* w, hipStream_t s)
{
    hipLaunchKernelGGL(k_gemv_small, dim3((unsigned)((k + 3) / 4)), dim3(kT), 0, s, k, Cinv, u, w);
    return hipGetLastError();
}

hipError_t gemv_sub(int64_t n, int k, const double* G, const double* w, const double* sv, double* y, hipStream_t s)
{
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 3) / 4, 4096);
    hipLaunchKernelGGL(k_gemv_sub, dim3(blocks), dim3(kT), sizeof(double) * k, s, n, k, G, w, sv, y);
    return hipGetLastError();
}

hipError_t sum_partials64(int nz, int64_t len, const double* part, double* out, int add_eye_k, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_part64, dim3(grid_of(len)), dim3(kT), 0, s, nz, len, part, out, add_eye_k);
    return hipGetLastError();
}

// ------------------------------------------------------------- host SPD

bool chol_lower(int k, double* a)
{
    // left-looking by columns; the entries below the diagonal of column j
    // are independent and spread over threads
    for (int j = 0; j < k; ++j) {
        double* aj = a + (size_t)j * k;
        double dj = aj[j];
        for (int q = 0; q < j; ++q) dj -= aj[q] * aj[q];
        if (!(dj > 0.0) || !std::isfinite(dj)) return false;
        dj = std::sqrt(dj);
        aj[j] = dj;
        const int64_t rem = k - j - 1;
        auto col = [&](int64_t i0, int64_t i1) {
            for (int64_t i = j + 1 + i0; i < j + 1 + i1; ++i) {
                double* ai = a + (size_t)i * k;
                double s = ai[j];
                for (int q = 0; q < j; ++q) s -= ai[q] * aj[q];
                ai[j] = s / dj;
            }
        };
        if (rem * (int64_t)j > 200000) parallel_for(rem, 16, col);
        else col(0, rem);
    }
    return true;
}

// x <- L^-1 (lower triangular, row-major, zeros above) for the lower factor
// in a. Row i of X = L^-1 is (e_i - sum_{q<i} L_iq X_q) / L_ii: each row an
// axpy combination of earlier rows (unit stride); threads take blocks of 32
// columns.
static void lower_inverse(int k, const double* a, std::vector<double>& x)
{
    x.assign((size_t)k * k, 0.0);
    constexpr int64_t cb = 32;
    parallel_for((k + cb - 1) / cb, 1, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t c0 = b * cb, c1 = std::min<int64_t>(k, c0 + cb);
            for (int64_t i = c0; i < k; ++i) {
                double* xi = x.data() + (size_t)i * k;
                const double* ai = a + (size_t)i * k;
                const int64_t ce = std::min<int64_t>(c1, i + 1);
                for (int64_t c = c0; c < ce; ++c) xi[c] = (i == c) ? 1.0 : 0.0;
                for (int64_t q = c0; q < i; ++q) {  // X_qc = 0 for c > q
                    const double f = ai[q];
                    const double* xq = x.data() + (size_t)q * k;
                    const int64_t qe = std::min<int64_t>(ce, q + 1);
                    for (int64_t c = c0; c < qe; ++c) xi[c] -= f * xq[c];
                }
                const double inv = 1.0 / ai[i];
                for (int64_t c = c0; c < ce; ++c) xi[c] *= inv;
            }
        }
    });
}

bool spd_inverse(int k, double* a)
{
    if (!chol_lower(k, a)) return false;
    std::vector<double> x;
    lower_inverse(k, a, x);
    // a^-1 = X^T X = sum_q (row q of X)^T (row q of X): every thread owns 8
    // output rows and adds the rank-one terms row by row (unit stride)
    std::fill(a, a + (size_t)k * k, 0.0);
    constexpr int64_t rb = 8;
    parallel_for((k + rb - 1) / rb, 1, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            const int64_t i0 = b * rb, i1 = std::min<int64_t>(k, i0 + rb);
            for (int64_t q = i0; q < k; ++q) {
                const double* xq = x.data() + (size_t)q * k;
                for (int64_t i = i0; i < std::min<int64_t>(i1, q + 1); ++i) {
                    const double f = xq[i];
                    double* ar = a + (size_t)i * k;
                    for (int64_t j = 0; j <= q; ++j) ar[j] += f * xq[j];
                }
            }
        }
    });
    return true;
}

bool chol_inv_t(int k, const double* a, double* w)
{
    std::vector<double> f(a, a + (size_t)k * k), x;
    if (!chol_lower(k, f.data())) return false;
    lower_inverse(k, f.data(), x);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) w[(size_t)i * k + j] = x[(size_t)j * k + i];
    return true;
}

}  // namespace fkt
