// Learned per-leaf preconditioner for CG on (K~ + sigma2 I) x = b.
//
// Not part of the paper's method (the paper solves Gaussian-process systems
// through MVMs, Sec. 5.3); it is built on the near-field diagonal blocks the
// plan produces. Each leaf block A_l = K(X_l, X_l) + sigma2 I = V_l^T
// diag(lam_l) V_l (host eigendecomposition) gets the filter
//     M_l = V_l^T diag(h_l) V_l,   h_{l,i} = exp(o_{l,i}) / lam_{l,i},
// where o is the output of one MLP (4 features -> 256 tanh -> 256 tanh -> 1,
// FP32) evaluated for every eigenvalue of every leaf. M = blockdiag(M_l) is
// symmetric positive definite for any weights, so plain PCG stays valid;
// with o = 0 it is block-Jacobi exactly (the initial state: the last layer
// starts at zero).
//
// Training minimises L = (1/B) sum_b min_a |a A M v_b - v_b|^2 / |v_b|^2
// over Gaussian v_b, with A the plan's own operator (FKT MVM + sigma2) and
// the optimal a_b = <u_b, v_b> / |u_b|^2, u_b = A M v_b: like PCG, L does not
// see the scale of M. Its gradient holds a_b fixed (it is stationary) and
// takes A as symmetric (the kernel matrix is; the FKT operator is within its
// approximation error):
//   g_b = (2 a_b / (B |v_b|^2)) A (a_b u_b - v_b),
//   dL/dh_{l,i} = sum_b (V_l g_{l,b})_i (V_l v_{l,b})_i,   dL/do = h dL/dh,
// then back through the MLP with this file's kernels (MFMA GEMMs for the
// 256 x 256 layer), and an Adam step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fkt.h"
#include "fkt_coarse.h"
#include "fkt_learn.h"

namespace fkt {
namespace {

constexpr int kH = kLearnHidden;
constexpr int kF = kLearnFeatures;
constexpr int kT = 256;  // threads of the elementwise / per-leaf kernels

// parameter layout (FP32): W1 [F][H], b1 [H], W2 [H][H], b2 [H], w3 [H], b3
constexpr int oW1 = 0, ob1 = oW1 + kF * kH, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, ow3 = ob2 + kH, ob3 = ow3 + kH;
constexpr int kNP = ob3 + 1;
static_assert(kNP == kLearnParams, "parameter count");

unsigned blocks_of(int64_t m, int per = kT) { return (unsigned)((m + per - 1) / per); }

// ------------------------------------------------------------ MFMA GEMM
//
// C[M x N] = op(A) op(B), FP32, v_mfma_f32_16x16x4f32. A workgroup of four
// waves owns a 64 x 64 tile of C (each wave 32 x 32: 2 x 2 MFMA tiles) and
// walks K in steps of 16 staged through LDS. op(A) = A (stored [M][K]) or
// A^T (stored [K][M]); op(B) = B (stored [K][N]) or B^T (stored [N][K]).
// M, N multiples of 64 and K (per split) a multiple of 16, checked by the
// host. Epilogues:
//   kEpiStore      C = acc
//   kEpiTanhBias   C = tanh(acc + bias[n])
//   kEpiDTanh      C = acc * (1 - aux[m][n]^2)
//   kEpiSplit      C[z] = acc over the z-th K range (partial sums)
enum { kEpiStore = 0, kEpiTanhBias = 1, kEpiDTanh = 2, kEpiSplit = 3 };
typedef float f4 __attribute__((ext_vector_type(4)));

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, int kchunk, const float* __restrict__ A,
                                              const float* __restrict__ B, float* __restrict__ C,
                                              const float* __restrict__ aux)
{
    __shared__ float As[64][17];   // [m][k]
    __shared__ float Bs[16][68];   // [k][n]
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += 16) {
        if (!TA) {  // A [M][K]: thread -> row m, 4 consecutive k
            const int m = t >> 2, k4 = (t & 3) * 4;
            const f4 v = *(const f4*)(A + (size_t)(m0 + m) * K + k0 + k4);
            As[m][k4 + 0] = v[0]; As[m][k4 + 1] = v[1]; As[m][k4 + 2] = v[2]; As[m][k4 + 3] = v[3];
        } else {    // A stored [K][M]: thread -> row k, 4 consecutive m
            const int k = t >> 4, m4 = (t & 15) * 4;
            const f4 v = *(const f4*)(A + (size_t)(k0 + k) * M + m0 + m4);
            As[m4 + 0][k] = v[0]; As[m4 + 1][k] = v[1]; As[m4 + 2][k] = v[2]; As[m4 + 3][k] = v[3];
        }
        if (!TB) {  // B [K][N]
            const int k = t >> 4, n4 = (t & 15) * 4;
            const f4 v = *(const f4*)(B + (size_t)(k0 + k) * N + n0 + n4);
            Bs[k][n4 + 0] = v[0]; Bs[k][n4 + 1] = v[1]; Bs[k][n4 + 2] = v[2]; Bs[k][n4 + 3] = v[3];
        } else {    // B stored [N][K]
            const int n = t >> 2, k4 = (t & 3) * 4;
            const f4 v = *(const f4*)(B + (size_t)(n0 + n) * K + k0 + k4);
            Bs[k4 + 0][n] = v[0]; Bs[k4 + 1][n] = v[1]; Bs[k4 + 2][n] = v[2]; Bs[k4 + 3][n] = v[3];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    float* __restrict__ Cz = EPI == kEpiSplit ? C + (size_t)blockIdx.z * M * N : C;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r, n = n0 + wn + j * 16 + (lane & 15);
                float v = acc[i][j][r];
                if constexpr (EPI == kEpiTanhBias) v = tanhf(v + aux[n]);
                if constexpr (EPI == kEpiDTanh) {
                    const float hv = aux[(size_t)m * N + n];
                    v *= 1.f - hv * hv;
                }
                Cz[(size_t)m * N + n] = v;
            }
}

// ------------------------------------------------------------ MLP pieces

// H1 = tanh(X W1 + b1), X [Sp][F]
__global__ __launch_bounds__(kT) void k_layer1(int64_t Sp, const float* __restrict__ X, const float* __restrict__ P,
                                               float* __restrict__ H1)
{
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= Sp * kH) return;
    const int64_t s = g / kH;
    const int c = (int)(g % kH);
    float v = P[ob1 + c];
#pragma unroll
    for (int f = 0; f < kF; ++f) v = fmaf(X[s * kF + f], P[oW1 + f * kH + c], v);
    H1[g] = tanhf(v);
}

// o[s] = H2[s,:] . w3 + b3: one wave per row
__global__ __launch_bounds__(kT) void k_layer3(int64_t Sp, const float* __restrict__ H2, const float* __restrict__ P,
                                               float* __restrict__ o)
{
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (s >= Sp) return;
    float v = 0.f;
#pragma unroll
    for (int j = 0; j < kH / 64; ++j) v = fmaf(H2[s * kH + lane + 64 * j], P[ow3 + lane + 64 * j], v);
#pragma unroll
    for (int w = 32; w > 0; w >>= 1) v += __shfl_xor(v, w, 64);
    if (lane == 0) o[s] = v + P[ob3];
}

// h = exp(o) / lam (FP64)
__global__ __launch_bounds__(kT) void k_filter(int64_t n, const float* __restrict__ o, const double* __restrict__ lam,
                                               double* __restrict__ h)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) h[i] = exp((double)o[i]) / lam[i];
}

// D2 = go (x) w3 * (1 - H2^2)
__global__ __launch_bounds__(kT) void k_dlayer2(int64_t Sp, const float* __restrict__ go, const float* __restrict__ P,
                                                const float* __restrict__ H2, float* __restrict__ D2)
{
    const int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (g >= Sp * kH) return;
    const int64_t s = g / kH;
    const int c = (int)(g % kH);
    const float hv = H2[g];
    D2[g] = go[s] * P[ow3 + c] * (1.f - hv * hv);
}

// partial[chunk][r][c] = sum over rows s of the chunk of w_r(s) A[s][c] for
// c < ncols: rows r < nw take weights W[s][r] (W is [Sp][nw]), and with
// ones a last row of weight 1 follows.
constexpr int kRedRows = 1024;
__global__ __launch_bounds__(kT) void k_colred(int64_t Sp, int ncols, const float* __restrict__ A, int lda, bool ones,
                                               const float* __restrict__ W, int nw, float* __restrict__ partial)
{
    const int c = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * kRedRows, s1 = min(Sp, s0 + kRedRows);
    const int R = nw + (ones ? 1 : 0);
    float accw[kF], acc1 = 0.f;
#pragma unroll
    for (int q = 0; q < kF; ++q) accw[q] = 0.f;
    if (c >= ncols) return;
    for (int64_t s = s0; s < s1; ++s) {
        const float a = A[s * lda + c];
        acc1 += a;
#pragma unroll
        for (int q = 0; q < kF; ++q)
            if (q < nw) accw[q] = fmaf(W[s * nw + q], a, accw[q]);
    }
    float* out = partial + (size_t)blockIdx.x * R * ncols;
#pragma unroll
    for (int q = 0; q < kF; ++q)
        if (q < nw) out[(size_t)q * ncols + c] = accw[q];
    if (ones) out[(size_t)nw * ncols + c] = acc1;
}

// out[i] = sum_z part[z][i], i < len
__global__ __launch_bounds__(kT) void k_sum_partials(int nz, int64_t len, const float* __restrict__ part,
                                                     float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int z = 0; z < nz; ++z) s += part[(size_t)z * len + i];
    out[i] = s;
}

// Adam (beta1 0.9, beta2 0.999, eps 1e-8), step t >= 1
__global__ __launch_bounds__(kT) void k_adam(int np, float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, float lr, float c1,
                                             float c2)
{
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi, vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// ------------------------------------------------------ spectral kernels
//
// One workgroup per leaf; leaf points are tree positions b..b+m-1, the
// caller's rows perm[b + i]. V [m][m] row i = eigenvector i, Vt = V^T.

// out[tree b+i][col] = sum_j V[i][j] x[perm[b+j]][col]   (c = V x)
__global__ __launch_bounds__(kT) void k_spec_proj(const int* __restrict__ begin, const int* __restrict__ count,
                                                  const int64_t* __restrict__ off, const double* __restrict__ Vt,
                                                  const int64_t* __restrict__ perm, int nrhs, int col,
                                                  const double* __restrict__ x, double* __restrict__ out, int ldo)
{
    extern __shared__ double xl[];
    const int l = blockIdx.x, b = begin[l], m = count[l];
    const double* __restrict__ Q = Vt + off[l];
    for (int j = threadIdx.x; j < m; j += kT) xl[j] = x[perm[b + j] * nrhs + col];
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += kT) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s = fma(Q[(size_t)j * m + i], xl[j], s);
        out[(size_t)(b + i) * ldo + col] = s;
    }
}

// y[perm[b+j]][col] = sum_i V[i][j] h[b+i] c[tree b+i][col]   (y = V^T (h c))
__global__ __launch_bounds__(kT) void k_spec_recon(const int* __restrict__ begin, const int* __restrict__ count,
                                                   const int64_t* __restrict__ off, const double* __restrict__ V,
                                                   const int64_t* __restrict__ perm, const double* __restrict__ h,
                                                   const double* __restrict__ c, int ldc, int nrhs, int col,
                                                   double* __restrict__ y)
{
    extern __shared__ double cl[];
    const int l = blockIdx.x, b = begin[l], m = count[l];
    const double* __restrict__ Q = V + off[l];
    for (int i = threadIdx.x; i < m; i += kT) cl[i] = h[b + i] * c[(size_t)(b + i) * ldc + col];
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += kT) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s = fma(Q[(size_t)i * m + j], cl[i], s);
        y[perm[b + j] * nrhs + col] = s;
    }
}

// z = M r for one column (CG): c = V r in LDS, scaled by h, then V^T.
__global__ __launch_bounds__(kT) void k_spec_apply(const int* __restrict__ begin, const int* __restrict__ count,
                                                   const int64_t* __restrict__ off, const double* __restrict__ V,
                                                   const double* __restrict__ Vt, const int64_t* __restrict__ perm,
                                                   const double* __restrict__ h, int nrhs, int col,
                                                   const double* __restrict__ r, double* __restrict__ z)
{
    extern __shared__ double sh[];
    const int l = blockIdx.x, b = begin[l], m = count[l];
    double* rl = sh;
    double* cl = sh + m;
    for (int j = threadIdx.x; j < m; j += kT) rl[j] = r[perm[b + j] * nrhs + col];
    __syncthreads();
    const double* __restrict__ Qt = Vt + off[l];
    for (int i = threadIdx.x; i < m; i += kT) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s = fma(Qt[(size_t)j * m + i], rl[j], s);
        cl[i] = h[b + i] * s;
    }
    __syncthreads();
    const double* __restrict__ Q = V + off[l];
    for (int j = threadIdx.x; j < m; j += kT) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s = fma(Q[(size_t)i * m + j], cl[i], s);
        z[perm[b + j] * nrhs + col] = s;
    }
}

// Two-level pieces (one column): s = V x[:, col] into a tree-order vector,
// and y[:, col] = V^T (h .* c) from a tree-order vector.
__global__ __launch_bounds__(kT) void k_spec_proj1(const int* __restrict__ begin, const int* __restrict__ count,
                                                   const int64_t* __restrict__ off, const double* __restrict__ Vt,
                                                   const int64_t* __restrict__ perm, int nrhs, int col,
                                                   const double* __restrict__ x, double* __restrict__ out)
{
    extern __shared__ double xl[];
    const int l = blockIdx.x, b = begin[l], m = count[l];
    const double* __restrict__ Q = Vt + off[l];
    for (int j = threadIdx.x; j < m; j += kT) xl[j] = x[perm[b + j] * nrhs + col];
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += kT) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s = fma(Q[(size_t)j * m + i], xl[j], s);
        out[b + i] = s;
    }
}
__global__ __launch_bounds__(kT) void k_spec_recon1(const int* __restrict__ begin, const int* __restrict__ count,
                                                    const int64_t* __restrict__ off, const double* __restrict__ V,
                                                    const int64_t* __restrict__ perm, const double* __restrict__ h,
                                                    const double* __restrict__ c, int nrhs, int col,
                                                    double* __restrict__ y)
{
    extern __shared__ double cl[];
    const int l = blockIdx.x, b = begin[l], m = count[l];
    const double* __restrict__ Q = V + off[l];
    for (int i = threadIdx.x; i < m; i += kT) cl[i] = h[b + i] * c[b + i];
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += kT) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s = fma(Q[(size_t)i * m + j], cl[i], s);
        y[perm[b + j] * nrhs + col] = s;
    }
}
// column col of a [n][B] tree-order array <-> a contiguous vector
__global__ __launch_bounds__(kT) void k_put_col(int64_t n, int B, int col, const double* __restrict__ v,
                                                double* __restrict__ a)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) a[i * B + col] = v[i];
}
__global__ __launch_bounds__(kT) void k_get_col(int64_t n, int B, int col, const double* __restrict__ a,
                                                double* __restrict__ v)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) v[i] = a[i * B + col];
}
__global__ __launch_bounds__(kT) void k_recip(int64_t n, const double* __restrict__ lam, double* __restrict__ h)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) h[i] = 1.0 / lam[i];
}

// Condition-number objective: go[i] = (a_i^2 - b_i^2) / h_i (FP32), 0 for
// padding, with a, b the spectral coordinates of the two extreme Ritz vectors.
__global__ __launch_bounds__(kT) void k_dout_cond(int64_t n, int64_t Sp, const double* __restrict__ h,
                                                  const double* __restrict__ a, const double* __restrict__ b,
                                                  float* __restrict__ go)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= Sp) return;
    go[i] = i < n ? (float)((a[i] * a[i] - b[i] * b[i]) / h[i]) : 0.f;
}

// u = sum_j c[j] Z[j][:] (Z: T rows of n)
__global__ __launch_bounds__(kT) void k_combine(int64_t n, int T, const double* __restrict__ c,
                                                const double* __restrict__ Z, double* __restrict__ u)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < T; ++j) s = fma(c[j], Z[(int64_t)j * n + i], s);
    u[i] = s;
}

// y = a x + y, and the scaled copy z = a x
__global__ __launch_bounds__(kT) void k_axpy1(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) y[i] = fma(a, x[i], y[i]);
}
__global__ __launch_bounds__(kT) void k_scale1(int64_t n, double a, const double* __restrict__ x, double* __restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) z[i] = a * x[i];
}
// p = z + beta p
__global__ __launch_bounds__(kT) void k_xpby1(int64_t n, const double* __restrict__ z, double beta, double* __restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = fma(beta, p[i], z[i]);
}

// go[i] = h_i sum_b c[i][b] p[i][b] scale[b]  (FP32 out), 0 for padding
__global__ __launch_bounds__(kT) void k_dout(int64_t n, int64_t Sp, int B, const double* __restrict__ h,
                                             const double* __restrict__ c, const double* __restrict__ p,
                                             const double* __restrict__ scale, float* __restrict__ go)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= Sp) return;
    if (i >= n) {
        go[i] = 0.f;
        return;
    }
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += c[i * B + b] * p[i * B + b] * scale[b];
    go[i] = (float)(h[i] * s);
}

// r[i][b] = a[b] u[i][b] - v[i][b]
__global__ __launch_bounds__(kT) void k_scaled_resid(int64_t m, int B, const double* __restrict__ a,
                                                     const double* __restrict__ u, const double* __restrict__ v,
                                                     double* __restrict__ r)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < m) r[i] = a[i % B] * u[i] - v[i];
}

// ------------------------------------------------------ batch helpers

// per-block partial column dots of a and b ([n][B] row-major)
constexpr int kDotBlocks = 256;
__global__ __launch_bounds__(kT) void k_coldot(int64_t n, int B, const double* __restrict__ a,
                                               const double* __restrict__ b, double* __restrict__ partial)
{
    __shared__ double sh[kT];
    for (int c = 0; c < B; ++c) {
        double s = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
            s += a[i * B + c] * b[i * B + c];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int o = kT / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[blockIdx.x * B + c] = sh[0];
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kT) void k_cvt(int64_t m, const double* __restrict__ a, T* __restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < m) b[i] = (T)a[i];
}

// r = (double)kw + sigma2 w - v ; ([n][B])
template <typename T>
__global__ __launch_bounds__(kT) void k_resid(int64_t m, const T* __restrict__ kw, const double* __restrict__ w,
                                              const double* __restrict__ v, double sigma2, double* __restrict__ r)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < m) r[i] = (double)kw[i] + sigma2 * w[i] - (v ? v[i] : 0.0);
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) as a counter-based hash,
// then Box-Muller: x[i] ~ N(0, 1).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__global__ __launch_bounds__(kT) void k_randn(int64_t m, uint64_t key, double* __restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= m) return;
    const uint64_t a = splitmix64(key ^ (2 * (uint64_t)i)), b = splitmix64(key ^ (2 * (uint64_t)i + 1));
    const double u1 = ((a >> 11) + 1) * 0x1.0p-53;  // (0, 1]
    const double u2 = (b >> 11) * 0x1.0p-53;        // [0, 1)
    x[i] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

}  // namespace

// ------------------------------------------------------------ state

struct LearnState {
    int device = 0;
    hipStream_t s = nullptr;
    int64_t n = 0, Sp = 0;
    int nleaf = 0, maxleaf = 0;
    const int64_t* perm = nullptr;  // plan's, not owned
    int* leaf_begin = nullptr;
    int* leaf_count = nullptr;
    int64_t* off = nullptr;
    double *V = nullptr, *Vt = nullptr, *lam = nullptr, *h = nullptr;
    float *X = nullptr, *P = nullptr, *G = nullptr, *Am = nullptr, *Av = nullptr;
    float *H1 = nullptr, *H2 = nullptr, *D2 = nullptr, *D1 = nullptr, *o = nullptr, *go = nullptr;
    float *part = nullptr;
    int nsplit = 1, nchunks = 1;
    int64_t adam_t = 0;
    std::vector<void*> allocs;
    // host copy of the leaf layout
    std::vector<int32_t> hbegin, hcount;
    std::vector<int64_t> hoff;
    // two-level state (ck > 0): G = V L per leaf [n][ck] (tree-order rows),
    // C^-1 for block-Jacobi (h = 1 / lam) and for the learned filter, and
    // work vectors of the coarse correction
    int ck = 0;
    double *cG = nullptr, *cCinv_bj = nullptr, *cCinv = nullptr, *h_bj = nullptr;
    double *cs = nullptr, *cy = nullptr, *cpart = nullptr, *cu = nullptr, *cw = nullptr, *cgram = nullptr;
    Gemm64* cdesc = nullptr;
    int cnz = 0;
    std::vector<void*> coarse_allocs;
    void drop_coarse()
    {
        (void)hipStreamSynchronize(s);
        for (void* q : coarse_allocs) (void)hipFree(q);
        coarse_allocs.clear();
        ck = 0;
        cG = cCinv_bj = cCinv = h_bj = cs = cy = cpart = cu = cw = cgram = nullptr;
        cdesc = nullptr;
    }
    template <class T>
    hipError_t cget(size_t count, T** out)
    {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, sizeof(T) * (count ? count : 1));
        if (e == hipSuccess) coarse_allocs.push_back(q);
        *out = (T*)q;
        return e;
    }

    template <class T>
    hipError_t get(size_t count, T** out)
    {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, sizeof(T) * (count ? count : 1));
        if (e == hipSuccess) allocs.push_back(q);
        *out = (T*)q;
        return e;
    }
    ~LearnState()
    {
        drop_coarse();
        for (void* q : allocs) (void)hipFree(q);
    }
};

void learn_destroy(LearnState* L) { delete L; }

// deterministic initial weights: W1, W2 ~ N(0, 1/fan_in) from SplitMix64 and
// Box-Muller on the host, biases 0, last layer 0 (so that o = 0: block-Jacobi)
static void init_params(uint64_t seed, std::vector<float>& p)
{
    p.assign(kNP, 0.f);
    auto mix = [](uint64_t z) {
        z += 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto normal = [&](uint64_t i) {
        const double u1 = ((mix(seed ^ (2 * i)) >> 11) + 1) * 0x1.0p-53, u2 = (mix(seed ^ (2 * i + 1)) >> 11) * 0x1.0p-53;
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    for (int i = 0; i < kF * kH; ++i) p[oW1 + i] = (float)(normal(i) / std::sqrt((double)kF));
    for (int i = 0; i < kH * kH; ++i) p[oW2 + i] = (float)(normal(kF * kH + i) / std::sqrt((double)kH));
}

LearnState* learn_create(int device, hipStream_t s, const LeafSpectra& S, const int64_t* perm, int64_t n, uint64_t seed,
                         std::string& err)
{
    LearnState* L = new LearnState();
    L->device = device;
    L->s = s;
    L->n = n;
    L->Sp = (n + 63) / 64 * 64;
    L->nleaf = (int)S.leaf_begin.size();
    L->maxleaf = S.max_leaf;
    L->perm = perm;
    L->nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(64, L->Sp / 2048));
    L->nchunks = (int)((L->Sp + kRedRows - 1) / kRedRows);
    const int64_t Sp = L->Sp;
    std::vector<double> vt(S.vecs.size());
    for (int l = 0; l < L->nleaf; ++l) {
        const int m = S.leaf_count[l];
        const double* a = S.vecs.data() + S.off[l];
        double* b = vt.data() + S.off[l];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) b[(size_t)j * m + i] = a[(size_t)i * m + j];
    }
    L->hbegin = S.leaf_begin;
    L->hcount = S.leaf_count;
    L->hoff = S.off;
    std::vector<float> X((size_t)Sp * kF, 0.f);
    std::copy(S.feat.begin(), S.feat.end(), X.begin());
    std::vector<float> p0;
    init_params(seed, p0);
    auto up = [&](const void* src, size_t bytes, void* dst) { return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice); };
    hipError_t e = hipSuccess;
    const size_t part_n = std::max((size_t)L->nsplit * kH * kH, (size_t)L->nchunks * (1 + kF) * kH);
    if ((e = L->get(L->nleaf, &L->leaf_begin)) || (e = L->get(L->nleaf, &L->leaf_count)) ||
        (e = L->get(L->nleaf + 1, &L->off)) || (e = L->get(S.vecs.size(), &L->V)) || (e = L->get(vt.size(), &L->Vt)) ||
        (e = L->get(n, &L->lam)) || (e = L->get(n, &L->h)) || (e = L->get((size_t)Sp * kF, &L->X)) ||
        (e = L->get(kNP, &L->P)) || (e = L->get(kNP, &L->G)) || (e = L->get(kNP, &L->Am)) || (e = L->get(kNP, &L->Av)) ||
        (e = L->get((size_t)Sp * kH, &L->H1)) || (e = L->get((size_t)Sp * kH, &L->H2)) ||
        (e = L->get((size_t)Sp * kH, &L->D2)) || (e = L->get((size_t)Sp * kH, &L->D1)) || (e = L->get(Sp, &L->o)) ||
        (e = L->get(Sp, &L->go)) || (e = L->get(part_n, &L->part)) ||
        (e = up(S.leaf_begin.data(), sizeof(int) * L->nleaf, L->leaf_begin)) ||
        (e = up(S.leaf_count.data(), sizeof(int) * L->nleaf, L->leaf_count)) ||
        (e = up(S.off.data(), sizeof(int64_t) * (L->nleaf + 1), L->off)) ||
        (e = up(S.vecs.data(), sizeof(double) * S.vecs.size(), L->V)) ||
        (e = up(vt.data(), sizeof(double) * vt.size(), L->Vt)) || (e = up(S.vals.data(), sizeof(double) * n, L->lam)) ||
        (e = up(X.data(), sizeof(float) * X.size(), L->X)) || (e = up(p0.data(), sizeof(float) * kNP, L->P)) ||
        (e = hipMemset(L->Am, 0, sizeof(float) * kNP)) || (e = hipMemset(L->Av, 0, sizeof(float) * kNP))) {
        err = std::string("learned preconditioner allocation/upload: ") + hipGetErrorString(e);
        delete L;
        return nullptr;
    }
    return L;
}

// new spectra and features (another sigma2); weights and Adam state kept
hipError_t learn_update_spectra(LearnState* L, const LeafSpectra& S)
{
    std::vector<double> vt(S.vecs.size());
    for (int l = 0; l < L->nleaf; ++l) {
        const int m = S.leaf_count[l];
        const double* a = S.vecs.data() + S.off[l];
        double* b = vt.data() + S.off[l];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) b[(size_t)j * m + i] = a[(size_t)i * m + j];
    }
    std::vector<float> X((size_t)L->Sp * kF, 0.f);
    std::copy(S.feat.begin(), S.feat.end(), X.begin());
    hipError_t e;
    if ((e = hipStreamSynchronize(L->s)) != hipSuccess) return e;
    L->drop_coarse();  // the coarse part belongs to the previous spectra
    if ((e = hipMemcpy(L->V, S.vecs.data(), sizeof(double) * S.vecs.size(), hipMemcpyHostToDevice))) return e;
    if ((e = hipMemcpy(L->Vt, vt.data(), sizeof(double) * vt.size(), hipMemcpyHostToDevice))) return e;
    if ((e = hipMemcpy(L->lam, S.vals.data(), sizeof(double) * L->n, hipMemcpyHostToDevice))) return e;
    return hipMemcpy(L->X, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice);
}

hipError_t learn_params(LearnState* L, float* host, bool set)
{
    hipError_t e = hipStreamSynchronize(L->s);
    if (e != hipSuccess) return e;
    if (set) return hipMemcpy(L->P, host, sizeof(float) * kNP, hipMemcpyHostToDevice);
    return hipMemcpy(host, L->P, sizeof(float) * kNP, hipMemcpyDeviceToHost);
}

// forward pass over all eigenvalues, then h = exp(o) / lam
static hipError_t forward(LearnState* L)
{
    const int64_t Sp = L->Sp;
    hipStream_t s = L->s;
    hipLaunchKernelGGL(k_layer1, dim3(blocks_of(Sp * kH)), dim3(kT), 0, s, Sp, L->X, L->P, L->H1);
    hipLaunchKernelGGL((k_gemm<false, false, kEpiTanhBias>), dim3(Sp / 64, kH / 64, 1), dim3(256), 0, s, (int)Sp, kH,
                       kH, kH, L->H1, L->P + oW2, L->H2, L->P + ob2);
    hipLaunchKernelGGL(k_layer3, dim3(blocks_of(Sp, kT / 64)), dim3(kT), 0, s, Sp, L->H2, L->P, L->o);
    hipLaunchKernelGGL(k_filter, dim3(blocks_of(L->n)), dim3(kT), 0, s, L->n, L->o, L->lam, L->h);
    return hipGetLastError();
}

// C^-1 with C = I + G^T diag(h) G (k x k): split-row product on the device,
// inverse on the host (FP64, SPD), back to Cinv. Synchronises.
static hipError_t coarse_inverse(LearnState* L, const double* h, double* Cinv)
{
    const int k = L->ck;
    hipStream_t s = L->s;
    hipError_t e = gemm64_batched(true, false, L->cdesc, L->cnz, k, k, L->cG, L->cG, h, L->cgram, 1.0, 0.0, s);
    if (e != hipSuccess) return e;
    if ((e = sum_partials64(L->cnz, (int64_t)k * k, L->cgram, L->cs, k, s)) != hipSuccess) return e;
    std::vector<double> C((size_t)k * k);
    if ((e = hipMemcpyAsync(C.data(), L->cs, sizeof(double) * C.size(), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (!spd_inverse(k, C.data())) return hipErrorInvalidValue;
    return hipMemcpy(Cinv, C.data(), sizeof(double) * C.size(), hipMemcpyHostToDevice);
}

hipError_t learn_set_coarse(LearnState* L, const double* Lmat, int k)
{
    L->drop_coarse();
    if (k <= 0 || !Lmat) return hipSuccess;
    const int64_t n = L->n;
    // the split-row products of C read cgram = cnz k x k partials; cs doubles
    // as the k x k staging buffer, so it holds max(n, k^2)
    L->cnz = (int)std::max<int64_t>(1, std::min<int64_t>(64, n / 4096));
    hipError_t e;
    if ((e = L->cget((size_t)n * k, &L->cG)) || (e = L->cget((size_t)k * k, &L->cCinv_bj)) ||
        (e = L->cget((size_t)k * k, &L->cCinv)) || (e = L->cget(n, &L->h_bj)) ||
        (e = L->cget(std::max<size_t>(n, (size_t)k * k), &L->cs)) || (e = L->cget(n, &L->cy)) ||
        (e = L->cget((size_t)kCoarseChunks * k, &L->cpart)) || (e = L->cget(k, &L->cu)) || (e = L->cget(k, &L->cw)) ||
        (e = L->cget((size_t)L->cnz * k * k, &L->cgram)) || (e = L->cget(L->nleaf + L->cnz, &L->cdesc))) {
        L->drop_coarse();
        return e;
    }
    L->ck = k;
    // descriptors: per leaf G_l = V_l L_l; then the split rows of C
    std::vector<Gemm64> d;
    int maxm = 0;
    for (int l = 0; l < L->nleaf; ++l) {
        const int m = L->hcount[l];
        const int64_t b0 = L->hbegin[l];
        maxm = std::max(maxm, m);
        d.push_back(Gemm64{m, k, m, m, k, k, L->hoff[l], b0 * k, b0 * k, 0});
    }
    const int64_t rows = (n + L->cnz - 1) / L->cnz;
    for (int z = 0; z < L->cnz; ++z) {
        const int64_t r0 = std::min<int64_t>(n, z * rows), r1 = std::min<int64_t>(n, r0 + rows);
        d.push_back(Gemm64{k, k, (int)(r1 - r0), k, k, k, r0 * k, r0 * k, (int64_t)z * k * k, r0});
    }
    if ((e = hipMemcpy(L->cdesc, d.data(), sizeof(Gemm64) * d.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = gemm64_batched(false, false, L->cdesc, L->nleaf, maxm, k, L->V, Lmat, nullptr, L->cG, 1.0, 0.0, L->s)) !=
            hipSuccess) {
        L->drop_coarse();
        return e;
    }
    L->cdesc += L->nleaf;  // the remaining descriptors are the C products
    hipLaunchKernelGGL(k_recip, dim3(blocks_of(n)), dim3(kT), 0, L->s, n, L->lam, L->h_bj);
    if ((e = coarse_inverse(L, L->h_bj, L->cCinv_bj)) != hipSuccess) {
        L->drop_coarse();
        return e;
    }
    return hipSuccess;
}

int learn_coarse_rank(const LearnState* L) { return L ? L->ck : 0; }

hipError_t learn_prepare_filter(LearnState* L)
{
    hipError_t e = forward(L);
    if (e != hipSuccess || L->ck == 0) return e;
    return coarse_inverse(L, L->h, L->cCinv);
}

// psi(y) = y - G C^-1 G^T (h .* y) for tree-order vectors
static hipError_t coarse_psi(LearnState* L, const double* h, const double* Cinv, const double* y, double* out,
                             hipStream_t s)
{
    hipError_t e;
    if ((e = gemv_t_weighted(L->n, L->ck, L->cG, h, y, L->cpart, kCoarseChunks, L->cu, s)) != hipSuccess) return e;
    if ((e = gemv_small(L->ck, Cinv, L->cu, L->cw, s)) != hipSuccess) return e;
    return gemv_sub(L->n, L->ck, L->cG, L->cw, y, out, s);
}

hipError_t learn_apply(LearnState* L, const double* r, double* z, int nrhs, int col, hipStream_t s, bool bj)
{
    const size_t lds = sizeof(double) * L->maxleaf;
    if (L->ck == 0) {
        if (bj) return hipErrorInvalidValue;  // one-level block-Jacobi runs on the Cholesky factors (cg.hip)
        hipLaunchKernelGGL(k_spec_apply, dim3(L->nleaf), dim3(kT), 2 * lds, s, L->leaf_begin, L->leaf_count, L->off,
                           L->V, L->Vt, L->perm, L->h, nrhs, col, r, z);
        return hipGetLastError();
    }
    // two-level: z = V^T (h .* psi(V r))
    const double* h = bj ? L->h_bj : L->h;
    hipLaunchKernelGGL(k_spec_proj1, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off, L->Vt,
                       L->perm, nrhs, col, r, L->cs);
    hipError_t e = coarse_psi(L, h, bj ? L->cCinv_bj : L->cCinv, L->cs, L->cy, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_spec_recon1, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off, L->V,
                       L->perm, h, L->cy, nrhs, col, z);
    return hipGetLastError();
}

// backward from go (set by k_dout) into G
static hipError_t backward(LearnState* L)
{
    const int64_t Sp = L->Sp;
    hipStream_t s = L->s;
    hipLaunchKernelGGL(k_dlayer2, dim3(blocks_of(Sp * kH)), dim3(kT), 0, s, Sp, L->go, L->P, L->H2, L->D2);
    // dW2 = H1^T D2 (split over the rows), into G + oW2
    const int kchunk = (int)((Sp / L->nsplit + 15) / 16 * 16);
    hipLaunchKernelGGL((k_gemm<true, false, kEpiSplit>), dim3(kH / 64, kH / 64, L->nsplit), dim3(256), 0, s, kH, kH,
                       (int)Sp, kchunk, L->H1, L->D2, L->part, (const float*)nullptr);
    hipLaunchKernelGGL(k_sum_partials, dim3(blocks_of((int64_t)kH * kH)), dim3(kT), 0, s, L->nsplit,
                       (int64_t)kH * kH, L->part, L->G + oW2);
    // db2 = colsum D2 (G + ob2); dw3 = H2^T go (G + ow3); db3 = sum go (G + ob3)
    hipLaunchKernelGGL(k_colred, dim3(L->nchunks), dim3(kT), 0, s, Sp, kH, L->D2, kH, true, (const float*)nullptr, 0,
                       L->part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kT), 0, s, L->nchunks, (int64_t)kH, L->part, L->G + ob2);
    hipLaunchKernelGGL(k_colred, dim3(L->nchunks), dim3(kT), 0, s, Sp, kH, L->H2, kH, false, L->go, 1, L->part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kT), 0, s, L->nchunks, (int64_t)kH, L->part, L->G + ow3);
    hipLaunchKernelGGL(k_colred, dim3(L->nchunks), dim3(kT), 0, s, Sp, 1, L->go, 1, true, (const float*)nullptr, 0,
                       L->part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kT), 0, s, L->nchunks, (int64_t)1, L->part, L->G + ob3);
    // D1 = (D2 W2^T) * (1 - H1^2)
    hipLaunchKernelGGL((k_gemm<false, true, kEpiDTanh>), dim3(Sp / 64, kH / 64, 1), dim3(256), 0, s, (int)Sp, kH, kH,
                       kH, L->D2, L->P + oW2, L->D1, L->H1);
    // [dW1; db1] = [X, 1]^T D1: rows W1[0..F-1] then b1, contiguous at G + oW1
    hipLaunchKernelGGL(k_colred, dim3(L->nchunks), dim3(kT), 0, s, Sp, kH, L->D1, kH, true, L->X, kF, L->part);
    hipLaunchKernelGGL(k_sum_partials, dim3(blocks_of((int64_t)(1 + kF) * kH)), dim3(kT), 0, s, L->nchunks,
                       (int64_t)(1 + kF) * kH, L->part, L->G + oW1);
    return hipGetLastError();
}

// loss and gradient for the batch v ([n][B] caller order, FP64, device)
fkt_status learn_loss_grad(fkt_plan_t P, LearnState* L, int prec, double sigma2, const double* v, int B, double* loss)
{
    const int64_t n = L->n, m = n * B;
    hipStream_t s = L->s;
    std::vector<void*> tmp;
    auto get = [&](size_t bytes, void** out) {
        hipError_t e = hipMalloc(out, bytes ? bytes : 256);
        if (e == hipSuccess) tmp.push_back(*out);
        return e;
    };
    struct Free {
        std::vector<void*>& t;
        ~Free()
        {
            for (void* q : t) (void)hipFree(q);
        }
    } fr{tmp};
    double *c, *w, *r, *g, *pp, *part, *vv;
    void *op_in, *op_out;
    const size_t es = prec == 1 ? sizeof(float) : sizeof(double);
    if (get(sizeof(double) * m, (void**)&c) || get(sizeof(double) * m, (void**)&w) || get(sizeof(double) * m, (void**)&r) ||
        get(sizeof(double) * m, (void**)&g) || get(sizeof(double) * m, (void**)&pp) ||
        get(sizeof(double) * kDotBlocks * B, (void**)&part) || get(sizeof(double) * B, (void**)&vv) ||
        get(es * m, &op_in) || get(es * m, &op_out))
        return FKT_ENOMEM;
    std::vector<double> hp((size_t)kDotBlocks * B), nv(B), nr(B);
    auto coldots = [&](const double* a, const double* b, std::vector<double>& out) -> bool {
        hipLaunchKernelGGL(k_coldot, dim3(kDotBlocks), dim3(kT), 0, s, n, B, a, b, part);
        if (hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
        if (hipStreamSynchronize(s) != hipSuccess) return false;
        out.assign(B, 0.0);
        for (int k = 0; k < kDotBlocks; ++k)
            for (int q = 0; q < B; ++q) out[q] += hp[(size_t)k * B + q];
        return true;
    };
    auto op = [&](const double* in, const double* sub, double* out) -> fkt_status {
        // out = A in - sub, A = FKT MVM (plan precision) + sigma2
        if (prec == 1) {
            hipLaunchKernelGGL((k_cvt<float>), dim3(blocks_of(m)), dim3(kT), 0, s, m, in, (float*)op_in);
            fkt_status st = fkt_mvm(P, op_in, op_out, B);
            if (st != FKT_OK) return st;
            hipLaunchKernelGGL((k_resid<float>), dim3(blocks_of(m)), dim3(kT), 0, s, m, (const float*)op_out, in, sub,
                               sigma2, out);
        } else {
            fkt_status st = fkt_mvm(P, in, op_out, B);
            if (st != FKT_OK) return st;
            hipLaunchKernelGGL((k_resid<double>), dim3(blocks_of(m)), dim3(kT), 0, s, m, (const double*)op_out, in, sub,
                               sigma2, out);
        }
        return hipGetLastError() == hipSuccess ? FKT_OK : FKT_EDEVICE;
    };
    if (learn_prepare_filter(L) != hipSuccess) return FKT_EDEVICE;  // h, and C^-1 for it (two-level)
    const size_t lds = sizeof(double) * L->maxleaf;
    // c = V v, or psi(V v) with the coarse part (P = V^T diag(h) psi V);
    // w = P v
    for (int b = 0; b < B; ++b) {
        if (L->ck == 0) {
            hipLaunchKernelGGL(k_spec_proj, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off,
                               L->Vt, L->perm, B, b, v, c, B);
        } else {
            hipLaunchKernelGGL(k_spec_proj1, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off,
                               L->Vt, L->perm, B, b, v, L->cs);
            if (coarse_psi(L, L->h, L->cCinv, L->cs, L->cy, s) != hipSuccess) return FKT_EDEVICE;
            hipLaunchKernelGGL(k_put_col, dim3(blocks_of(n)), dim3(kT), 0, s, n, B, b, L->cy, c);
        }
        hipLaunchKernelGGL(k_spec_recon, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off, L->V,
                           L->perm, L->h, c, B, B, b, w);
    }
    fkt_status st = op(w, nullptr, g);  // u = A M v (in g)
    if (st != FKT_OK) return st;
    std::vector<double> uv, uu, ab(2 * B);
    if (!coldots(v, v, nv) || !coldots(g, v, uv) || !coldots(g, g, uu)) return FKT_EDEVICE;
    for (int b = 0; b < B; ++b) ab[b] = uu[b] > 0.0 ? uv[b] / uu[b] : 0.0;
    if (hipMemcpyAsync(vv, ab.data(), sizeof(double) * B, hipMemcpyHostToDevice, s) != hipSuccess) return FKT_EDEVICE;
    hipLaunchKernelGGL(k_scaled_resid, dim3(blocks_of(m)), dim3(kT), 0, s, m, B, vv, g, v, r);  // r = a u - v
    if (!coldots(r, r, nr)) return FKT_EDEVICE;  // also retires the use of vv
    double lsum = 0.0;
    for (int b = 0; b < B; ++b) lsum += nv[b] > 0.0 ? nr[b] / nv[b] : 0.0;
    *loss = lsum / B;
    st = op(r, nullptr, g);  // g = A r (A taken as symmetric)
    if (st != FKT_OK) return st;
    // dL/dh needs (psi V g) and (psi V v): the derivative of P = V^T diag(h)
    // psi V in h is V^T E diag(dh) E^T V with E^T = psi, C's dependence on h
    // included
    for (int b = 0; b < B; ++b) {
        if (L->ck == 0) {
            hipLaunchKernelGGL(k_spec_proj, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off,
                               L->Vt, L->perm, B, b, g, pp, B);
        } else {
            hipLaunchKernelGGL(k_spec_proj1, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off,
                               L->Vt, L->perm, B, b, g, L->cs);
            if (coarse_psi(L, L->h, L->cCinv, L->cs, L->cy, s) != hipSuccess) return FKT_EDEVICE;
            hipLaunchKernelGGL(k_put_col, dim3(blocks_of(n)), dim3(kT), 0, s, n, B, b, L->cy, pp);
        }
    }
    for (int b = 0; b < B; ++b) ab[B + b] = nv[b] > 0.0 ? 2.0 * ab[b] / (B * nv[b]) : 0.0;
    if (hipMemcpyAsync(vv, ab.data() + B, sizeof(double) * B, hipMemcpyHostToDevice, s) != hipSuccess)
        return FKT_EDEVICE;
    hipLaunchKernelGGL(k_dout, dim3(blocks_of(L->Sp)), dim3(kT), 0, s, n, L->Sp, B, L->h, c, pp, vv, L->go);
    if (backward(L) != hipSuccess) return FKT_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return FKT_EDEVICE;
    return FKT_OK;
}

// Condition-number objective. PCG (the current filter, one- or two-level)
// from x0 = 0 on b runs T iterations; its step lengths define the Lanczos
// tridiagonal of P A (diagonal 1/alpha_j + beta_{j-1}/alpha_{j-1}, off
// diagonal sqrt(beta_j)/alpha_j) and its preconditioned residuals the
// Lanczos vectors (-1)^j z_j / sqrt(r_j . z_j), which are orthonormal in
// the P^-1 inner product. The extreme Ritz pairs (lambda, u) then give
// log kappa = log lambda_max - log lambda_min. Since P^-1 = L L^T + D with D
// = blockdiag(V^T diag(1/h) V) affine in 1/h, d lambda = lambda (V u)_i^2
// dh_i / h_i^2 at u^T P^-1 u = 1, so d log kappa / do_i = (V u_max)_i^2 / h_i
// - (V u_min)_i^2 / h_i. Leaves the gradient in L->G; b is overwritten.
fkt_status learn_cond_grad(fkt_plan_t P, LearnState* L, int prec, double sigma2, double* b, int T, double* cond)
{
    const int64_t n = L->n;
    hipStream_t s = L->s;
    std::vector<void*> tmp;
    auto get = [&](size_t bytes, void** out) {
        hipError_t e = hipMalloc(out, bytes ? bytes : 256);
        if (e == hipSuccess) tmp.push_back(*out);
        return e;
    };
    struct Free {
        std::vector<void*>& t;
        ~Free()
        {
            for (void* q : t) (void)hipFree(q);
        }
    } fr{tmp};
    double *z, *p, *q, *Z, *ua, *ub, *ta, *tb, *part, *cd;
    void *op_in, *op_out;
    const size_t es = prec == 1 ? sizeof(float) : sizeof(double);
    if (get(sizeof(double) * n, (void**)&z) || get(sizeof(double) * n, (void**)&p) || get(sizeof(double) * n, (void**)&q) ||
        get(sizeof(double) * n * T, (void**)&Z) || get(sizeof(double) * n, (void**)&ua) ||
        get(sizeof(double) * n, (void**)&ub) || get(sizeof(double) * n, (void**)&ta) ||
        get(sizeof(double) * n, (void**)&tb) || get(sizeof(double) * kDotBlocks, (void**)&part) ||
        get(sizeof(double) * 2 * T, (void**)&cd) || get(es * n, &op_in) || get(es * n, &op_out))
        return FKT_ENOMEM;
    std::vector<double> hp(kDotBlocks);
    auto dot = [&](const double* a, const double* bb, double* out) -> bool {
        hipLaunchKernelGGL(k_coldot, dim3(kDotBlocks), dim3(kT), 0, s, n, 1, a, bb, part);
        if (hipMemcpyAsync(hp.data(), part, sizeof(double) * kDotBlocks, hipMemcpyDeviceToHost, s) != hipSuccess) return false;
        if (hipStreamSynchronize(s) != hipSuccess) return false;
        double t = 0.0;
        for (double v : hp) t += v;
        *out = t;
        return true;
    };
    auto op = [&](const double* in, double* out) -> fkt_status {  // out = (K~ + sigma2 I) in
        if (prec == 1) {
            hipLaunchKernelGGL((k_cvt<float>), dim3(blocks_of(n)), dim3(kT), 0, s, n, in, (float*)op_in);
            fkt_status st = fkt_mvm(P, op_in, op_out, 1);
            if (st != FKT_OK) return st;
            hipLaunchKernelGGL((k_resid<float>), dim3(blocks_of(n)), dim3(kT), 0, s, n, (const float*)op_out, in,
                               (const double*)nullptr, sigma2, out);
        } else {
            fkt_status st = fkt_mvm(P, in, op_out, 1);
            if (st != FKT_OK) return st;
            hipLaunchKernelGGL((k_resid<double>), dim3(blocks_of(n)), dim3(kT), 0, s, n, (const double*)op_out, in,
                               (const double*)nullptr, sigma2, out);
        }
        return hipGetLastError() == hipSuccess ? FKT_OK : FKT_EDEVICE;
    };
    if (learn_prepare_filter(L) != hipSuccess) return FKT_EDEVICE;
    // PCG on b (the residual r lives in b)
    double* r = b;
    std::vector<double> alpha(T), beta(T);
    if (learn_apply(L, r, z, 1, 0, s) != hipSuccess) return FKT_EDEVICE;
    double rho = 0.0;
    if (!dot(r, z, &rho) || !(rho > 0.0)) return FKT_EDEVICE;
    hipLaunchKernelGGL(k_scale1, dim3(blocks_of(n)), dim3(kT), 0, s, n, 1.0 / std::sqrt(rho), z, Z);
    hipLaunchKernelGGL(k_scale1, dim3(blocks_of(n)), dim3(kT), 0, s, n, 1.0, z, p);
    int Tk = T;
    for (int j = 0; j < T; ++j) {
        fkt_status st = op(p, q);
        if (st != FKT_OK) return st;
        double pq = 0.0;
        if (!dot(p, q, &pq) || !(pq > 0.0)) { Tk = j; break; }
        alpha[j] = rho / pq;
        hipLaunchKernelGGL(k_axpy1, dim3(blocks_of(n)), dim3(kT), 0, s, n, -alpha[j], q, r);
        if (learn_apply(L, r, z, 1, 0, s) != hipSuccess) return FKT_EDEVICE;
        double rn = 0.0;
        if (!dot(r, z, &rn)) return FKT_EDEVICE;
        if (!(rn > 0.0)) { Tk = j + 1; beta[j] = 0.0; break; }
        beta[j] = rn / rho;
        if (j + 1 < T)
            hipLaunchKernelGGL(k_scale1, dim3(blocks_of(n)), dim3(kT), 0, s, n, ((j + 1) & 1 ? -1.0 : 1.0) / std::sqrt(rn),
                               z, Z + (int64_t)(j + 1) * n);
        hipLaunchKernelGGL(k_xpby1, dim3(blocks_of(n)), dim3(kT), 0, s, n, z, beta[j], p);
        rho = rn;
    }
    if (Tk < 2) return FKT_EDEVICE;
    // Lanczos tridiagonal and its extreme eigenpairs (host)
    std::vector<double> Tm((size_t)Tk * Tk, 0.0), w(Tk);
    for (int j = 0; j < Tk; ++j) {
        Tm[(size_t)j * Tk + j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
        if (j + 1 < Tk) Tm[(size_t)j * Tk + j + 1] = Tm[(size_t)(j + 1) * Tk + j] = std::sqrt(beta[j]) / alpha[j];
    }
    if (!sym_eig(Tk, Tm.data(), w.data()) || !(w[0] > 0.0)) return FKT_EDEVICE;
    *cond = w[Tk - 1] / w[0];
    std::vector<double> cc(2 * (size_t)Tk);
    for (int j = 0; j < Tk; ++j) {
        cc[j] = Tm[(size_t)(Tk - 1) * Tk + j];  // eigenvector of lambda_max (row Tk-1)
        cc[Tk + j] = Tm[j];                     // and of lambda_min (row 0)
    }
    if (hipMemcpyAsync(cd, cc.data(), sizeof(double) * cc.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return FKT_EDEVICE;
    hipLaunchKernelGGL(k_combine, dim3(blocks_of(n)), dim3(kT), 0, s, n, Tk, cd, Z, ua);
    hipLaunchKernelGGL(k_combine, dim3(blocks_of(n)), dim3(kT), 0, s, n, Tk, cd + Tk, Z, ub);
    const size_t lds = sizeof(double) * L->maxleaf;
    hipLaunchKernelGGL(k_spec_proj1, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off, L->Vt,
                       L->perm, 1, 0, ua, ta);
    hipLaunchKernelGGL(k_spec_proj1, dim3(L->nleaf), dim3(kT), lds, s, L->leaf_begin, L->leaf_count, L->off, L->Vt,
                       L->perm, 1, 0, ub, tb);
    hipLaunchKernelGGL(k_dout_cond, dim3(blocks_of(L->Sp)), dim3(kT), 0, s, n, L->Sp, L->h, ta, tb, L->go);
    if (backward(L) != hipSuccess) return FKT_EDEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return FKT_EDEVICE;
    return FKT_OK;
}

fkt_status learn_train_cond(fkt_plan_t P, LearnState* L, int prec, double sigma2, int steps, int T, double lr,
                            uint64_t seed, double* cond_first, double* cond_last)
{
    double* b = nullptr;
    if (hipMalloc(&b, sizeof(double) * L->n) != hipSuccess) return FKT_ENOMEM;
    fkt_status st = FKT_OK;
    for (int it = 0; it < steps; ++it) {
        const uint64_t key = seed * 0x2545F4914F6CDD1Dull + (uint64_t)it * 0x9E3779B97F4A7C15ull;
        hipLaunchKernelGGL(k_randn, dim3(blocks_of(L->n)), dim3(kT), 0, L->s, L->n, key, b);
        double cond = 0.0;
        st = learn_cond_grad(P, L, prec, sigma2, b, T, &cond);
        if (st != FKT_OK) break;
        if (it == 0 && cond_first) *cond_first = cond;
        if (cond_last) *cond_last = cond;
        L->adam_t += 1;
        const float c1 = 1.f - std::pow(0.9f, (float)L->adam_t), c2 = 1.f - std::pow(0.999f, (float)L->adam_t);
        hipLaunchKernelGGL(k_adam, dim3(blocks_of(kNP)), dim3(kT), 0, L->s, kNP, L->P, L->G, L->Am, L->Av, (float)lr, c1,
                           c2);
        if (hipGetLastError() != hipSuccess) {
            st = FKT_EDEVICE;
            break;
        }
    }
    (void)hipStreamSynchronize(L->s);
    (void)hipFree(b);
    return st;
}

hipError_t learn_randn(LearnState* L, void* x, int64_t n, bool f32, uint64_t key)
{
    double* tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, sizeof(double) * (n ? n : 1));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_randn, dim3(blocks_of(n)), dim3(kT), 0, L->s, n, key, tmp);
    if (f32)
        hipLaunchKernelGGL((k_cvt<float>), dim3(blocks_of(n)), dim3(kT), 0, L->s, n, (const double*)tmp, (float*)x);
    else
        (void)hipMemcpyAsync(x, tmp, sizeof(double) * n, hipMemcpyDeviceToDevice, L->s);
    e = hipStreamSynchronize(L->s);
    (void)hipFree(tmp);
    return e;
}

hipError_t learn_grad(LearnState* L, float* host)
{
    hipError_t e = hipStreamSynchronize(L->s);
    if (e != hipSuccess) return e;
    return hipMemcpy(host, L->G, sizeof(float) * kNP, hipMemcpyDeviceToHost);
}

fkt_status learn_train(fkt_plan_t P, LearnState* L, int prec, double sigma2, int steps, int B, double lr, uint64_t seed,
                       double* loss_first, double* loss_last)
{
    const int64_t m = L->n * B;
    double* v = nullptr;
    if (hipMalloc(&v, sizeof(double) * m) != hipSuccess) return FKT_ENOMEM;
    fkt_status st = FKT_OK;
    for (int it = 0; it < steps; ++it) {
        const uint64_t key = seed * 0x2545F4914F6CDD1Dull + (uint64_t)it * 0x9E3779B97F4A7C15ull;
        hipLaunchKernelGGL(k_randn, dim3(blocks_of(m)), dim3(kT), 0, L->s, m, key, v);
        double loss = 0.0;
        st = learn_loss_grad(P, L, prec, sigma2, v, B, &loss);
        if (st != FKT_OK) break;
        if (it == 0 && loss_first) *loss_first = loss;
        if (loss_last) *loss_last = loss;
        L->adam_t += 1;
        const float c1 = 1.f - std::pow(0.9f, (float)L->adam_t), c2 = 1.f - std::pow(0.999f, (float)L->adam_t);
        hipLaunchKernelGGL(k_adam, dim3(blocks_of(kNP)), dim3(kT), 0, L->s, kNP, L->P, L->G, L->Am, L->Av, (float)lr, c1,
                           c2);
        if (hipGetLastError() != hipSuccess) {
            st = FKT_EDEVICE;
            break;
        }
    }
    (void)hipStreamSynchronize(L->s);
    (void)hipFree(v);
    return st;
}

}  // namespace fkt
