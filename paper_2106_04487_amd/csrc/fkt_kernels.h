// Device templates of the FKT matrix-vector product for CDNA4 (gfx950),
// included by the .hip translation units that instantiate them.
//
// One 64-lane wavefront owns a block of up to 64 consecutive targets inside
// one leaf (one lane per target). Source data that every lane needs at the
// same time -- source points of a near leaf, a far node's centre and
// moments, the constant tables -- is indexed uniformly across the wave, so it
// is fetched with scalar loads and used as scalar operands; per-target data
// lives in vector registers. Lane masks from the plan select, per target,
// exactly the near leaves and far nodes of that target's own walk.
//
// Expansion (paper Theorem 3.1, eq. finaltrunc), per far node b with centre
// c and scale s = node radius, for a source at r' = x_s - c and a target at
// r = t - c:
//   K~(r', r) = sum_{k<=p} sum_h Yhat_kh(r^) Yhat_kh(r'^)
//               sum_{j=k,k+2..<=p} r'^j F_kj(|r|),
//   F_kj(r)  = [j=0] K(r) + sum_{m=1}^{j} K^(m)(r) r^(m-j) Tbar_kjm,
// where the harmonics are normalised so that sum_h Yhat(u) Yhat(v) =
// C_k^alpha(u.v) (addition theorem, Appendix A.1; this absorbs Z_k).
// s2m stores, in units of s,
//   M_b[kh, j] = sum_s Yhat_kh(r'^) (|r'|/s)^j x_s
//              = sum_s Rhat_kh(r'/s) (|r'|/s)^(j-k) x_s   (solid harmonics),
// and m2t evaluates sum_kh Yhat_kh(r^) sum_j (s/|r|)^j (F_kj |r|^j) M_b[kh, j].
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "../../include/fkt.h"
#include "fkt_device.h"

namespace fkt {
namespace {

constexpr int kWave = 64;

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

constexpr int cbinom(int a, int b)
{
    if (b < 0 || b > a) return 0;
    long long r = 1;
    for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return (int)r;
}

// number of radial powers j = k, k+2, ..., <= p for harmonic degree k
constexpr int nj_of(int p, int k) { return (p - k) / 2 + 1; }
// offset of degree k's F_kj entries in a flat per-pair array
constexpr int f_off(int p, int k)
{
    int o = 0;
    for (int q = 0; q < k; ++q) o += nj_of(p, q);
    return o;
}
// radial rows of degree k kept by a compressed expansion (keep 0: all)
constexpr int nk_of(int p, int k, int keep) { return keep > 0 && keep < nj_of(p, k) ? keep : nj_of(p, k); }
constexpr int fk_off(int p, int k, int keep)
{
    int o = 0;
    for (int q = 0; q < k; ++q) o += nk_of(p, q, keep);
    return o;
}
// terms per node: sum_k |H_k| nk, |H_k| = C(k+d-1, d-1) - C(k+d-3, d-1)
constexpr int crank(int d, int p, int keep)
{
    int o = 0;
    for (int k = 0; k <= p; ++k)
        o += (cbinom(k + d - 1, d - 1) - (k >= 2 ? cbinom(k + d - 3, d - 1) : 0)) * nk_of(p, k, keep);
    return o;
}

// Hides a table pointer's value from the optimiser so that loads from fixed
// offsets are issued where they are used (cheap scalar-cache hits) instead of
// being hoisted out of a loop into dozens of long-lived registers.
template <typename P>
__device__ __forceinline__ P* opaque(P* p)
{
    asm volatile("" : "+s"(p));
    return p;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// ------------------------------------------------- expansion coefficients
//
// Tbar_{k,j,m} depends only on the dimension and the indices (Appendix
// A.2), so it is evaluated at compile time:
//   Tbar_kjm = sum_{n = max((j+k)/2, m)}^{j} A_{k,2n-j} (-2)^{2n-j} C(n, 2n-j) B_{n,m} / n!
//   A_{k,i}  = i! (alpha + k) / (2^i ((i-k)/2)! (alpha)_{(i+k)/2+1})  (k = i mod 2)
//   B_{n,m}  = (-1)^{n+m} (2n-2m-1)!! C(2n-m-1, m-1) / 2^n,
// with alpha = d/2 - 1 and the binomial of the binomial expansion of eps^n
// kept in Tbar.
constexpr double cx_fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}
constexpr double cx_dfact(int n)
{
    double r = 1.0;
    for (int i = n; i > 1; i -= 2) r *= i;
    return r;
}
constexpr double cx_rising(double a, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= a + i;
    return r;
}
constexpr double cx_binom(int a, int b)
{
    if (b < 0 || b > a) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return r;
}
constexpr double cx_pow(double x, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}
constexpr double cx_A(int k, int i, double alpha)
{
    if (k > i || ((i - k) & 1)) return 0.0;
    return cx_fact(i) * (alpha + k) / (cx_pow(2.0, i) * cx_fact((i - k) / 2) * cx_rising(alpha, (i + k) / 2 + 1));
}
constexpr double cx_B(int n, int m)
{
    if (m < 1 || m > n) return 0.0;
    return (((n + m) & 1) ? -1.0 : 1.0) * cx_dfact(2 * n - 2 * m - 1) * cx_binom(2 * n - m - 1, m - 1) / cx_pow(2.0, n);
}
constexpr double cx_tbar(int d, int k, int j, int m)
{
    const double alpha = 0.5 * d - 1.0;
    double s = 0.0;
    const int n0 = (j + k) / 2 > m ? (j + k) / 2 : m;
    for (int n = n0; n <= j; ++n) {
        const int i = 2 * n - j;
        s += cx_A(k, i, alpha) * cx_pow(-2.0, i) * cx_binom(n, i) * cx_B(n, m) / cx_fact(n);
    }
    return s;
}

// ------------------------------------------------------------ harmonics
//
// All solid harmonics of degree <= P of x (D coordinates), each handed to
// emit(integral_constant<degree>, value). A degree-k harmonic in e dims is
//   G_{k-mu}^{lam}(x_{e-1}; rho_e^2) * H_mu(x_0..x_{e-2}),  lam = mu + (e-2)/2,
// with G_n^lam(z; rho^2) = rho^n C_n^lam(z / rho) from the Gegenbauer
// three-term recurrence (Appendix A.1) multiplied through by rho^n, and H_mu
// a degree-mu harmonic of one dimension less; in two dimensions the
// harmonics are Re and Im of (x_0 + i x_1)^m.
//
// With NORM the values are multiplied by the square of the orthonormal
// normalisation times Z_k (table hn2, and 1/(2 pi), 1/pi at the base), so
// that the product of a NORM harmonic and a plain one of the same (k, h)
// summed over h is C_k^alpha of the cosine between the two unit vectors.
// s2m folds that factor into the moments; m2t then needs none.
template <int E, int P, bool NORM, typename T, class Emit>
__device__ __forceinline__ void harmonics(const T* x, const T* rho2, const T* __restrict__ hn2, Emit& emit)
{
    if constexpr (E == 2) {
        T cr = T(1), ci = T(0);
        auto base = [&](auto mc) {
            constexpr int m = decltype(mc)::value;
            if constexpr (m == 0) {
                emit(mc, NORM ? T(0.159154943091895335768884) : T(1));  // 1 / (2 pi)
            } else {
                const T nr = cr * x[0] - ci * x[1];
                const T ni = cr * x[1] + ci * x[0];
                cr = nr;
                ci = ni;
                if constexpr (NORM) {
                    emit(mc, cr * T(0.318309886183790671537768));  // 1 / pi
                    emit(mc, ci * T(0.318309886183790671537768));
                } else {
                    emit(mc, cr);
                    emit(mc, ci);
                }
            }
        };
        static_for<0, P + 1>(base);
    } else {
        const T z = x[E - 1];
        const T r2 = rho2[E];
        auto level = [&](auto muc, T H) {
            constexpr int mu = decltype(muc)::value;
            constexpr double lam = mu + 0.5 * (E - 2);
            T g1 = T(1), g2 = T(0);
            auto step = [&](auto nc) {
                constexpr int n = decltype(nc)::value;
                T g;
                if constexpr (n == 0) {
                    g = T(1);
                } else if constexpr (n == 1) {
                    g = T(2.0 * lam) * z;
                } else {
                    g = T(2.0 * (n + lam - 1.0) / n) * z * g1 - T((n + 2.0 * lam - 2.0) / n) * r2 * g2;
                }
                if constexpr (n >= 1) {
                    g2 = g1;
                    g1 = g;
                }
                if constexpr (NORM)
                    emit(std::integral_constant<int, mu + n>{}, H * (g * hn2[((E - 3) * (P + 1) + mu) * (P + 1) + n]));
                else
                    emit(std::integral_constant<int, mu + n>{}, H * g);
            };
            static_for<0, P - mu + 1>(step);
        };
        harmonics<E - 1, P, NORM, T>(x, rho2, hn2, level);
    }
}

// ------------------------------------------------------------ FP64 helpers
//
// 1/sqrt(d2) for d2 > 0: hardware estimate, then one third-order correction
// y (1 + e/2 + 3e^2/8) with e = 1 - d2 y^2.
__device__ __forceinline__ double rsqrt_pos(double d2)
{
    const double y = __builtin_amdgcn_rsq(d2);
    const double e = fma(-d2 * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// exp(x) for finite x <= 0: x = k ln2 + f with |f| <= ln2/2 (ln2 split in a
// high part exact in k * hi and a low part, as in fdlibm's exp), e^f by its
// Taylor polynomial to degree 12 (truncation < 2e-16 relative), times 2^k.
__device__ __forceinline__ double exp_nonpos(double x)
{
    const double k = __builtin_rint(x * 1.44269504088896340736);
    double f = fma(k, -6.93147180369123816490e-01, x);
    f = fma(k, -1.90821492927058770002e-10, f);
    double p = 2.08767569878680989792e-09;      // 1/12!
    p = fma(p, f, 2.50521083854417187751e-08);  // 1/11!
    p = fma(p, f, 2.75573192239858906526e-07);  // 1/10!
    p = fma(p, f, 2.75573192239858906526e-06);  // 1/9!
    p = fma(p, f, 2.48015873015873015873e-05);  // 1/8!
    p = fma(p, f, 1.98412698412698412698e-04);  // 1/7!
    p = fma(p, f, 1.38888888888888888889e-03);  // 1/6!
    p = fma(p, f, 8.33333333333333333333e-03);  // 1/5!
    p = fma(p, f, 4.16666666666666666667e-02);  // 1/4!
    p = fma(p, f, 1.66666666666666666667e-01);  // 1/3!
    p = fma(p, f, 0.5);
    p = fma(p, f, 1.0);
    p = fma(p, f, 1.0);
    return __builtin_ldexp(p, (int)k);
}

// exp(x) for finite x <= 0 through a table of 2^(j/256) held in LDS (Tang's
// table-driven method): x = (n/256) ln2 + f with n = round(256 x / ln2) and
// |f| <= ln2/512, so e^x = 2^(n >> 8) 2^((n & 255)/256) e^f, with e^f by its
// Taylor polynomial to degree 4 (truncation < 4e-17 relative). n is read from
// the low word of x 256/ln2 + 1.5 2^52, whose rounding is the rounding of n.
// f takes one FMA with ln2/256 rounded to FP64: its error, at most
// |n| 2^-62 <= 369 |x| 2^-62, changes e^x by a relative 8e-17 |x|, i.e. by at
// most 8e-17 e^x |x| <= 3e-17 absolute. x is clamped at -1100, where e^x is
// already zero in FP64. exp_tab_scaled applies scale() to the polynomial
// value before the table entry, so a factor such as 1 + a costs one FMA.
constexpr int kExpTabLen = 256;
template <class Scale>
__device__ __forceinline__ double exp_tab_scaled(double x, const double* __restrict__ tab, Scale scale)
{
    constexpr double kShift = 6755399441055744.0;               // 1.5 * 2^52
    constexpr double kInvL = 369.3299304675746;                 // 256 / ln2
    constexpr double kL = 0x1.62e42ff000000p-9 + -1.6409824502660487e-13;  // ln2/256 to FP64
    x = fmax(x, -1100.0);
    const double kn = fma(x, kInvL, kShift);
    const int n = __double2loint(kn);
    const double k = kn - kShift;
    const double f = fma(k, -kL, x);
    double q = fma(f, 4.16666666666666666667e-02, 1.66666666666666666667e-01);
    q = fma(q, f, 0.5);
    q = fma(q, f, 1.0);
    q = fma(q, f, 1.0);
    return __builtin_ldexp(tab[n & (kExpTabLen - 1)] * scale(q), n >> 8);
}
__device__ __forceinline__ double exp_tab(double x, const double* __restrict__ tab)
{
    return exp_tab_scaled(x, tab, [](double q) { return q; });
}
// (1 + a) e^x: the factor enters the polynomial value as one FMA, q + q a
__device__ __forceinline__ double exp_tab_1p(double x, double a, const double* __restrict__ tab)
{
    return exp_tab_scaled(x, tab, [a](double q) { return fma(q, a, q); });
}

// c sqrt(d2) for d2 > 0: estimate y of 1/sqrt(d2), g = d2 y, then one Newton
// step for the square root, c g (1 + e/2) with e = 1 - g y, written as
// g (1.5 c - 0.5 c g y) (4 instructions after the estimate). The estimate's
// relative error, at most 5.3e-8 measured over 2.6e5 inputs spanning
// [1e-300, 1e300], gives |e| <= 1.1e-7, and the step leaves a relative error
// of about 3 e^2 / 8 <= 4.3e-15 plus rounding.
__device__ __forceinline__ double scaled_sqrt_pos(double d2, double c)
{
    const double y = __builtin_amdgcn_rsq(d2);
    const double g = d2 * y;
    return g * fma(-0.5 * c * g, y, 1.5 * c);
}

// ------------------------------------------------------- radial derivatives
//
// K^(m)(r), m = 0..P, in FP64 (closed forms / recurrences per kernel).
template <int KIND, int P>
__device__ __forceinline__ void radial_derivs(const DevPlan& a, double r, double (&D)[P + 1])
{
    const double var = a.var;
    if constexpr (KIND == FKT_GAUSSIAN) {  // exp(-u^2), u = r s: d^m/dr^m = (-s)^m H_m(u) exp(-u^2)
        const double s = 0.70710678118654752440 / a.ell, u = r * s, e = var * exp_nonpos(-u * u);
        double h1 = 1.0, h2 = 0.0, sc = 1.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            double h = (m == 0) ? 1.0 : 2.0 * u * h1 - 2.0 * (m - 1) * h2;
            if (m >= 1) { h2 = h1; h1 = h; }
            D[m] = sc * h * e;
            sc *= -s;
        }
    } else if constexpr (KIND == FKT_EXPONENTIAL) {
        const double c = 1.0 / a.ell, e = var * exp_nonpos(-c * r);
        double sc = 1.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) { D[m] = sc * e; sc *= -c; }
    } else if constexpr (KIND == FKT_MATERN32) {  // (1 + cr) e^{-cr}: (-c)^m (1 - m + cr) e^{-cr}
        const double c = 1.7320508075688772935 / a.ell, cr = c * r, e = var * exp_nonpos(-cr);
        double sc = 1.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) { D[m] = sc * (1.0 - m + cr) * e; sc *= -c; }
    } else if constexpr (KIND == FKT_MATERN52) {  // Q e^{-cr}, Q = 1 + cr + (cr)^2/3 (Leibniz rule)
        const double c = 2.2360679774997896964 / a.ell, cr = c * r, e = var * exp_nonpos(-cr);
        const double q0 = 1.0 + cr + cr * cr / 3.0, q1 = c + 2.0 * c * cr / 3.0, q2 = 2.0 * c * c / 3.0;
        double s0 = 1.0, s1 = 0.0, s2 = 0.0;  // (-c)^m, (-c)^(m-1), (-c)^(m-2)
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            D[m] = e * (s0 * q0 + m * s1 * q1 + 0.5 * m * (m - 1) * s2 * q2);
            s2 = s1;
            s1 = (m == 0) ? 1.0 : s1 * -c;
            s0 *= -c;
        }
    } else if constexpr (KIND == FKT_RATQUAD || KIND == FKT_CAUCHY) {
        // w(r+h)^beta, w quadratic in h: J.C.P. Miller's power-series recurrence
        double g0, g1, g2, beta;
        if constexpr (KIND == FKT_RATQUAD) {
            const double c = 0.5 / (a.alpha * a.ell * a.ell);
            g0 = 1.0 + c * r * r; g1 = 2.0 * c * r; g2 = c; beta = -a.alpha;
        } else {
            const double c = 1.0 / (a.ell * a.ell);
            g0 = 1.0 + c * r * r; g1 = 2.0 * c * r; g2 = c; beta = -1.0;
        }
        const double ig0 = 1.0 / g0;
        double f[P + 1];
        if constexpr (KIND == FKT_CAUCHY) f[0] = ig0; else f[0] = pow(g0, beta);
        double fact = 1.0;
        D[0] = var * f[0];
#pragma unroll
        for (int m = 1; m <= P; ++m) {
            double acc = ((beta + 1.0) - m) * g1 * f[m - 1];
            if (m >= 2) acc += (2.0 * (beta + 1.0) - m) * g2 * f[m - 2];
            f[m] = acc * ig0 / m;
            fact *= m;
            D[m] = var * fact * f[m];
        }
    } else if constexpr (KIND == FKT_LAPLACE) {  // 1/r: (-1)^m m! / r^(m+1)
        const double ir = 1.0 / r;
        D[0] = var * ir;
#pragma unroll
        for (int m = 1; m <= P; ++m) D[m] = D[m - 1] * (-(double)m) * ir;
    } else {
        static_assert(KIND == FKT_GAUSSIAN, "unknown kernel kind");
    }
}

template <typename T> __device__ __forceinline__ const T* hn_ptr(const DevPlan& a);
template <> __device__ __forceinline__ const double* hn_ptr<double>(const DevPlan& a) { return a.hn64; }
template <> __device__ __forceinline__ const float* hn_ptr<float>(const DevPlan& a) { return a.hn32; }

// ------------------------------------------------------------------ gather
//
// Packed source records in tree order: D coordinates then the weights of
// the NC right-hand-side columns of the pass, stride src_stride(D, NC)
// elements (even); the per-target accumulators ([n][NC]) are cleared on the
// way. Columns past ncols (a pass padded to NC) get weight 0.
constexpr int src_stride(int d, int nc = 1) { return (d + nc + 1) & ~1; }

template <int D, typename T, int NC = 1>
__global__ __launch_bounds__(256) void k_gather(int n, const int64_t* __restrict__ perm, const T* __restrict__ pts,
                                                const T* __restrict__ x, int nrhs, int col, int ncols,
                                                T* __restrict__ src, T* __restrict__ zacc,
                                                unsigned* __restrict__ ctr = nullptr)
{
    constexpr int S = src_stride(D, NC);
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (ctr && i == 0) *ctr = 0u;  // work-queue counter of the pass's persistent launch
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < NC; ++c) zacc[(size_t)i * NC + c] = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) src[(size_t)i * S + a] = pts[(size_t)i * D + a];
    const int64_t row = perm[i] * nrhs + col;
#pragma unroll
    for (int c = 0; c < NC; ++c) src[(size_t)i * S + D + c] = c < ncols ? x[row + c] : T(0);
#pragma unroll
    for (int a = D + NC; a < S; ++a) src[(size_t)i * S + a] = T(0);
}

// --------------------------------------------------------------------- s2m
//
// Moments of every far node straight from its own points (Algorithm 1,
// source2mult; no translation between levels). One wave per work unit of at
// most kUnitPoints points of one node; each lane accumulates its points'
// contributions to moment entries [C0, C1) in registers, then the wave sums.
// Moments carry the harmonics' normalisation (see harmonics<NORM>).
// The weights are column col of records of stride S (a multi-column pass
// runs one launch per column; mom and part point at that column's block).
template <int D, int P, typename T, int C0, int C1>
__global__ __launch_bounds__(kWave) void k_s2m(const DevPlan a, const T* __restrict__ src, int S, int col,
                                               T* __restrict__ mom, T* __restrict__ part)
{
    constexpr int R = cbinom(P + D, D);
    constexpr int NC = C1 - C0;
    const int u = blockIdx.x;
    const int lane = threadIdx.x;
    const int slot = a.unit_slot[u];
    if (a.inst_active && !a.inst_active[a.slot_inst[slot]]) return;  // instance not needed by this MVM
    const int beg = a.unit_begin[u], end = a.unit_end[u];
    double c[D];
#pragma unroll
    for (int i = 0; i < D; ++i) c[i] = a.slot_ctr[slot * D + i];
    const double is = 1.0 / a.slot_scale[slot];
    const T* __restrict__ hn2 = hn_ptr<T>(a);

    T acc[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) acc[i] = T(0);

    for (int s = beg + lane; s < end; s += kWave) {
        const T* __restrict__ hnl = opaque(hn2);
        T x[D], rho2[D + 1];
        rho2[0] = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            x[i] = T((a.pts64[(size_t)s * D + i] - c[i]) * is);
            rho2[i + 1] = rho2[i] + x[i] * x[i];
        }
        T q[P / 2 + 1];
        q[0] = src[(size_t)s * S + D + col];
#pragma unroll
        for (int i = 1; i <= P / 2; ++i) q[i] = q[i - 1] * rho2[D];
        int off = 0;
        auto emit = [&](auto kc, T v) {
            constexpr int k = decltype(kc)::value;
            constexpr int nj = nj_of(P, k);
            auto put = [&](auto jc) {
                constexpr int jj = decltype(jc)::value;
                const int idx = off + jj;
                if (idx >= C0 && idx < C1) acc[idx - C0] += v * q[jj];
            };
            static_for<0, nj>(put);
            off += nj;
        };
        harmonics<D, P, true, T>(x, rho2, hnl, emit);
    }

    const int dst = a.unit_dst[u];
    T* out = dst >= 0 ? mom + (size_t)dst * R : part + (size_t)(-1 - dst) * R;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const T v = wave_sum(acc[i]);
        if (lane == 0) out[C0 + i] = v;
    }
}

// Nodes split over several units: moments = ordered sum of the partials.
template <typename T>
__global__ __launch_bounds__(256) void k_s2m_reduce(int nred, int R, const int* __restrict__ red_slot,
                                                    const int* __restrict__ red_off, const T* __restrict__ part,
                                                    T* __restrict__ mom)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)nred * R) return;
    const int r = (int)(g / R), i = (int)(g % R);
    T s = T(0);
    for (int q = red_off[r]; q < red_off[r + 1]; ++q) s += part[(size_t)q * R + i];
    mom[(size_t)red_slot[r] * R + i] = s;
}

// --------------------------------------------------------------------- m2t
//
// Far-field value of one (target, far node) pair: the plain harmonics of
// the unit vector towards the target contracted with the node's moments M,
// S_kj = sum_h Y_kh(r^) M[kh, j], then the radial functions (FP64):
// sum_kj (s/|r|)^j (F_kj(|r|) |r|^j) S_kj. r = target - centre, scale = s.
// With KEEP > 0 (radial compression, Appendix A.4) only the first
// nk_of(P, k, KEEP) radial rows of each degree are evaluated, against moments
// already combined into them (k_compress).
//
// With UNIFORM_M the moments are the same for the whole wave (node-major
// jobs): each harmonic's few moments are then loaded through a pointer the
// optimiser cannot see through, so the scalar loads are issued where they
// are used instead of all at once (which spills the scalar registers).
// With NCOL columns, column c's moments start at M + c * cs and out
// receives one value per column; the harmonics and radial functions are
// shared by the columns.
template <int D, int P, int KIND, typename T, bool UNIFORM_M = false, int KEEP = 0, int NCOL = 1>
__device__ __forceinline__ void far_pair(const DevPlan& a, const double (&r)[D], double scale, const T* M,
                                         size_t cs, double (&out)[NCOL])
{
    constexpr int NF = fk_off(P, P + 1, KEEP);
    double r2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) r2 = fma(r[i], r[i], r2);
    const double ir = rsqrt_pos(r2);  // r2 > 0: a far target is never at the centre
    const double rr = r2 * ir;

    // angular part: S_kj over harmonics of r^ (|r^| = 1 at the top level)
    T x[D], rho2[D + 1];
    rho2[0] = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        x[i] = T(r[i] * ir);
        rho2[i + 1] = rho2[i] + x[i] * x[i];
    }
    rho2[D] = T(1);
    T Skj[NF * NCOL];
#pragma unroll
    for (int i = 0; i < NF * NCOL; ++i) Skj[i] = T(0);
    int off = 0;
    auto emit = [&](auto kc, T yv) {
        constexpr int k = decltype(kc)::value;
        constexpr int nj = nk_of(P, k, KEEP);
        // constant address space: uniform loads from it go through the
        // scalar cache (the moments are written by an earlier launch)
        using CT = const __attribute__((address_space(4))) T;
        CT* Mc[NCOL];
#pragma unroll
        for (int c = 0; c < NCOL; ++c) {
            Mc[c] = (CT*)(M + c * cs + off);
            if constexpr (UNIFORM_M) asm volatile("" : "+s"(Mc[c]));
        }
        auto dot = [&](auto jc) {
            constexpr int jj = decltype(jc)::value;
#pragma unroll
            for (int c = 0; c < NCOL; ++c) {
                if constexpr (UNIFORM_M)
                    Skj[(fk_off(P, k, KEEP) + jj) * NCOL + c] += yv * Mc[c][jj];
                else
                    Skj[(fk_off(P, k, KEEP) + jj) * NCOL + c] += yv * M[c * cs + off + jj];
            }
        };
        static_for<0, nj>(dot);
        off += nj;
    };
    harmonics<D, P, false, T>(x, rho2, (const T*)nullptr, emit);

    // radial part (FP64): F_kj(r) r^j = [j=0] K + sum_m K^(m) r^m Tbar_kjm
    double Dm[P + 1];
    radial_derivs<KIND, P>(a, rr, Dm);
    double um[P + 1];
    um[0] = Dm[0];
    double rp = 1.0;
#pragma unroll
    for (int m = 1; m <= P; ++m) { rp *= rr; um[m] = Dm[m] * rp; }
    const double v = scale * ir;  // s / |r| < theta
    double vp[P + 1];
    vp[0] = 1.0;
#pragma unroll
    for (int jp = 1; jp <= P; ++jp) vp[jp] = vp[jp - 1] * v;
#pragma unroll
    for (int c = 0; c < NCOL; ++c) out[c] = 0.0;
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
            const double vf = vp[jv] * f;
#pragma unroll
            for (int c = 0; c < NCOL; ++c) out[c] = fma(vf, (double)Skj[(fk_off(P, k, KEEP) + jj) * NCOL + c], out[c]);
        };
        static_for<0, nk_of(P, k, KEEP)>(radial_j);
    };
    static_for<0, P + 1>(radial_k);
}

// One wave per 64-target block and unit of up to job_seg of its jobs (units
// spread the heavy blocks over the machine). The block's (target, far node)
// pairs come packed in jobs of 64 lanes, one pair per lane, with at most
// MAXN nodes per job; a job's node moments and centres are staged in LDS
// (two buffers: the next job is fetched into registers while the current
// one computes), and each lane adds its pair's value to its target's LDS
// accumulator. The unit then adds its 64 sums to zacc (other units of the
// block and the near field, possibly running concurrently, add to the same
// accumulators).
template <int D, int P, int KIND, typename T>
__global__ __launch_bounds__(kWave) void k_m2t(const DevPlan a, const T* __restrict__ mom, T* __restrict__ zacc)
{
    constexpr int R = cbinom(P + D, D);
    constexpr int NF = f_off(P, P + 1);
    constexpr int MAXN = m2t_max_job_nodes(D, P, (int)sizeof(T));
    constexpr int PF = (MAXN * R + kWave - 1) / kWave;
    constexpr int G = D + 1;  // centre and scale per node
    static_assert(MAXN * G <= kWave, "node geometry is fetched one value per lane");
    __shared__ T smom[2][PF * kWave];  // whole 64-lane rows: the fill below writes PF * 64 entries
    __shared__ double sgeo[2][MAXN * G];
    __shared__ double zblk[kWave];
    const int blk = blockIdx.x;
    const int lane = threadIdx.x;
    // this unit's jobs of the block
    const int j0 = a.job_off[blk] + (int)blockIdx.y * a.job_seg;
    const int j1 = min(a.job_off[blk + 1], j0 + a.job_seg);
    if (j0 >= j1) return;  // whole-wave exit
    const int tb = a.blk_begin[blk], cnt = a.blk_count[blk];
    zblk[lane] = 0.0;
    // each lane holds its own target; pairs fetch it by cross-lane shuffle
    double tx[D];
#pragma unroll
    for (int i = 0; i < D; ++i) tx[i] = a.pts64[(size_t)(tb + (lane < cnt ? lane : 0)) * D + i];

    T pre[PF];
    double pgeo = 0.0;
    // Fetch job j's node moments and centres into registers: lane i of row q
    // holds entry q*64 + i of the job's concatenated moments. Entries past
    // the job's nn * R are clamped to its last entry (a valid address; the
    // value is never read).
    auto fetch = [&](int j) {
        const int n0 = a.job_noff[j], nn = a.job_noff[j + 1] - n0;
        const int myslot = a.job_nodes[n0 + (lane < nn ? lane : nn - 1)];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int i = min(q * kWave + lane, nn * R - 1);
            const int node = i / R;
            const int slot = __shfl(myslot, node, kWave);
            pre[q] = mom[(unsigned)(slot * R + (i - node * R))];
        }
        int node = lane / G;
        node = node < nn ? node : nn - 1;
        const int c = lane - (lane / G) * G;
        const int slot = __shfl(myslot, node, kWave);
        pgeo = (c < D) ? a.slot_ctr[(unsigned)(slot * D + c)] : a.slot_scale[slot];
    };
    if (j0 < j1) fetch(j0);

    int buf = 0;
    for (int j = j0; j < j1; ++j) {
#pragma unroll
        for (int q = 0; q < PF; ++q) smom[buf][q * kWave + lane] = pre[q];
        if (lane < MAXN * G) sgeo[buf][lane] = pgeo;
        __syncthreads();
        const unsigned pw = a.job_pairs[(size_t)j * kWave + lane];
        if (j + 1 < j1) fetch(j + 1);
        const int lt = pw & 63;
        double txl[D];
#pragma unroll
        for (int i = 0; i < D; ++i) txl[i] = __shfl(tx[i], lt, kWave);
        if (pw != 0xffffu) {
            const int ni = pw >> 6;
            const double* __restrict__ geo = sgeo[buf] + ni * G;
            double r[D];
#pragma unroll
            for (int i = 0; i < D; ++i) r[i] = txl[i] - geo[i];
            double acc[1];
            far_pair<D, P, KIND, T>(a, r, geo[D], smom[buf] + ni * R, 0, acc);
            atomicAdd(&zblk[lt], acc[0]);
        }
        buf ^= 1;
    }
    __syncthreads();
    if (lane < cnt) unsafeAtomicAdd(zacc + tb + lane, T(zblk[lane]));
}

// Far field, node-major: every job is one far node and up to 64 of its far
// targets (one per lane, taken from any target blocks, in tree order), so
// the node's centre, scale and moments are the same for the whole wave and
// are read through the scalar cache as operands of the vector FMAs: no LDS
// staging and no per-lane moment addresses. Every pair adds its value to its
// target's accumulator with one atomic (the near field, possibly running
// concurrently, adds to the same accumulators). Four jobs per workgroup.
// With NCOL columns, column c's moments are the block mom + c * cs and the
// accumulators are [n][NCOL].
// Node-major jobs whose moments are staged in LDS: at high expansion rank
// the scalar-operand moments need more scalar registers than there are
// (the compiler spills them into vector lanes); wave-uniform LDS reads
// broadcast to all lanes without bank conflicts and need no scalar
// registers. Used when the four waves' moment sets fit in 64 KB.
template <int D, int P, typename T, int KEEP, int NCOL>
constexpr bool m2t_nodes_lds()
{
    return crank(D, P, KEEP) > 120 && 4 * NCOL * crank(D, P, KEEP) * (int)sizeof(T) <= 65536;
}

// one node-major job j (wave-uniform) of 64 lanes; with MLDS the node's
// moments are at M (LDS, column c at M + c * R), else at mom + slot * R
// (column c at + c * cs)
template <int D, int P, int KIND, typename T, int KEEP, int NCOL, bool MLDS = false>
__device__ __forceinline__ void m2t_node_job(const DevPlan& a, int j, const T* __restrict__ mom, size_t cs,
                                             T* __restrict__ zacc, const T* M = nullptr)
{
    constexpr int R = crank(D, P, KEEP);
    const int lane = threadIdx.x & 63;
    const int slot = a.nj_slot[j];
    if (!MLDS && a.inst_active && !a.inst_active[a.slot_inst[slot]]) return;
    const int t = a.nj_tgt[(size_t)j * kWave + lane];
    const int tt = t >= 0 ? t : a.nj_tgt[(size_t)j * kWave];  // lane 0 of a job always holds a target
    double r[D];
#pragma unroll
    for (int i = 0; i < D; ++i) r[i] = a.pts64[(size_t)tt * D + i] - a.slot_ctr[slot * D + i];
    double acc[NCOL];
    if constexpr (MLDS)
        far_pair<D, P, KIND, T, false, KEEP, NCOL>(a, r, a.slot_scale[slot], M, (size_t)R, acc);
    else
        far_pair<D, P, KIND, T, true, KEEP, NCOL>(a, r, a.slot_scale[slot], mom + (size_t)slot * R, cs, acc);
    if (t >= 0) {
#pragma unroll
        for (int c = 0; c < NCOL; ++c) unsafeAtomicAdd(zacc + (size_t)t * NCOL + c, T(acc[c]));
    }
}

template <int D, int P, int KIND, typename T, int KEEP = 0, int NCOL = 1>
__global__ __launch_bounds__(256) void k_m2t_nodes(const DevPlan a, const T* __restrict__ mom, size_t cs,
                                                   T* __restrict__ zacc)
{
    const int j = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if constexpr (m2t_nodes_lds<D, P, T, KEEP, NCOL>()) {
        constexpr int R = crank(D, P, KEEP);
        __shared__ T smom[4 * NCOL * R];
        T* my = smom + (threadIdx.x >> 6) * NCOL * R;
        const int lane = threadIdx.x & 63;
        bool run = j < a.nnjobs;
        if (run) {
            const int slot = a.nj_slot[j];
            run = !(a.inst_active && !a.inst_active[a.slot_inst[slot]]);
            if (run)
                for (int c = 0; c < NCOL; ++c)
                    for (int i = lane; i < R; i += kWave) my[c * R + i] = mom[c * cs + (size_t)slot * R + i];
        }
        __syncthreads();  // every wave of the block reaches it
        if (run) m2t_node_job<D, P, KIND, T, KEEP, NCOL, true>(a, j, mom, cs, zacc, my);
    } else {
        if (j >= a.nnjobs) return;
        m2t_node_job<D, P, KIND, T, KEEP, NCOL>(a, j, mom, cs, zacc);
    }
}

// Radial compression of the moments (Appendix A.4, eq. f_g): for every far
// node and harmonic (k, h), the kept rows i < nk take the others in,
//   M'_i = M_i + sum_{jj >= nk} c[k][jj][i] sigma^(2 (jj - i)) M_jj,
// sigma = s / l, with the exact interpolative coefficients of the host
// (L_{k+2jj} = sum_i c L_{k+2i}); arithmetic in FP64. One thread per node
// walks the harmonics in the order s2m and m2t lay them out (their values
// are not needed, only the degree of each).
template <int D, int P, typename T, int KEEP>
__global__ __launch_bounds__(256) void k_compress(const DevPlan a, const T* __restrict__ mom, T* __restrict__ momc)
{
    constexpr int R = cbinom(P + D, D);
    constexpr int RC = crank(D, P, KEEP);
    constexpr int MJ = P / 2 + 1;
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= a.nslots) return;
    const double sg = a.slot_scale[slot] * a.comp_invlen;
    const double s2 = sg * sg;
    const T* M = mom + (size_t)slot * R;
    T* O = momc + (size_t)slot * RC;
    int fo = 0, co = 0;
    T x[D], rho2[D + 1];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = T(0);
#pragma unroll
    for (int i = 0; i <= D; ++i) rho2[i] = T(0);
    auto emit = [&](auto kc, T) {
        constexpr int k = decltype(kc)::value;
        constexpr int nj = nj_of(P, k), nk = nk_of(P, k, KEEP);
        for (int i = 0; i < nk; ++i) {
            double acc = (double)M[fo + i];
            double w = 1.0;
            for (int t = i; t < nk; ++t) w *= s2;  // sigma^(2 (nk - i))
            for (int jj = nk; jj < nj; ++jj) {
                acc = fma(a.comp_coef[(k * MJ + jj) * MJ + i] * w, (double)M[fo + jj], acc);
                w *= s2;
            }
            O[co + i] = T(acc);
        }
        fo += nj;
        co += nk;
    };
    harmonics<D, P, false, T>(x, rho2, (const T*)nullptr, emit);
}

// -------------------------------------------------------------- near field
//
// Dense near blocks (Algorithm 1, near_mat): for each near leaf of the
// block's list, the lanes whose target has that leaf in its own near set
// sum K(|t - x_s|) x_s over the leaf's points; the points stream through
// scalar registers. The far-field result is added and the sum scattered to
// the caller's order.
template <int KIND, typename T>
struct NearKernel;

// FP64 evaluations take the exponential table in LDS (exp_tab); the FP32
// ones ignore it. kBias is added to every squared distance: kernels that take
// a square root get d2 >= 1e-300 > 0, which keeps coincident points off the
// singular path of the reciprocal square root (their r becomes ~1e-150, where
// K(r) = K(0) in FP64) without a branch.
template <> struct NearKernel<FKT_GAUSSIAN, double> {
    static constexpr bool kTable = true;
    static constexpr double kBias = 0.0;
    static __device__ __forceinline__ double eval(double d2, double c0, double, const double* tab)
    {
        return exp_tab(c0 * d2, tab);
    }
};
template <> struct NearKernel<FKT_EXPONENTIAL, double> {
    static constexpr bool kTable = true;
    static constexpr double kBias = 1e-300;
    static __device__ __forceinline__ double eval(double d2, double c0, double, const double* tab)
    {
        return exp_tab(scaled_sqrt_pos(d2, c0), tab);  // c0 = -1/ell
    }
};
template <> struct NearKernel<FKT_MATERN32, double> {
    static constexpr bool kTable = true;
    static constexpr double kBias = 1e-300;
    static __device__ __forceinline__ double eval(double d2, double c0, double, const double* tab)
    {
        const double ar = scaled_sqrt_pos(d2, c0);
        return exp_tab_1p(-ar, ar, tab);
    }
};
template <> struct NearKernel<FKT_MATERN52, double> {
    static constexpr bool kTable = true;
    static constexpr double kBias = 1e-300;
    static __device__ __forceinline__ double eval(double d2, double c0, double, const double* tab)
    {
        const double ar = scaled_sqrt_pos(d2, c0);
        return fma(ar, fma(ar, 1.0 / 3.0, 1.0), 1.0) * exp_tab(-ar, tab);
    }
};
template <> struct NearKernel<FKT_RATQUAD, double> {
    static constexpr bool kTable = false;
    static constexpr double kBias = 0.0;
    static __device__ __forceinline__ double eval(double d2, double c0, double c1, const double*)
    {
        return pow(1.0 + c0 * d2, c1);
    }
};
template <> struct NearKernel<FKT_CAUCHY, double> {
    static constexpr bool kTable = false;
    static constexpr double kBias = 0.0;
    static __device__ __forceinline__ double eval(double d2, double c0, double, const double*)
    {
        const double b = 1.0 + c0 * d2;  // >= 1
        double y = __builtin_amdgcn_rcp(b);
        y = fma(fma(-b, y, 1.0), y, y);
        return fma(fma(-b, y, 1.0), y, y);
    }
};
template <> struct NearKernel<FKT_LAPLACE, double> {
    static constexpr bool kTable = false;
    static constexpr double kBias = 0.0;
    static __device__ __forceinline__ double eval(double d2, double, double, const double*)
    {
        const double y = rsqrt_pos(d2);
        return d2 > 0.0 ? y : 0.0;
    }
};

// FP32: hardware transcendental approximations (v_exp_f32 / v_log_f32 are
// base 2; c0 is pre-scaled by log2(e) where an exponential follows).
template <> struct NearKernel<FKT_GAUSSIAN, float> {
    static constexpr bool kTable = false;
    static constexpr float kBias = 0.0f;
    static __device__ __forceinline__ float eval(float d2, float c0, float, const double*) { return __builtin_amdgcn_exp2f(c0 * d2); }
};
template <> struct NearKernel<FKT_EXPONENTIAL, float> {
    static constexpr bool kTable = false;
    static constexpr float kBias = 0.0f;
    static __device__ __forceinline__ float eval(float d2, float c0, float, const double*)
    {
        return __builtin_amdgcn_exp2f(c0 * __builtin_amdgcn_sqrtf(d2));
    }
};
template <> struct NearKernel<FKT_MATERN32, float> {
    static constexpr bool kTable = false;
    static constexpr float kBias = 0.0f;
    static __device__ __forceinline__ float eval(float d2, float c0, float c1, const double*)
    {
        const float r = __builtin_amdgcn_sqrtf(d2);
        return (1.0f + c1 * r) * __builtin_amdgcn_exp2f(c0 * r);
    }
};
template <> struct NearKernel<FKT_MATERN52, float> {
    static constexpr bool kTable = false;
    static constexpr float kBias = 0.0f;
    static __device__ __forceinline__ float eval(float d2, float c0, float c1, const double*)
    {
        const float ar = c1 * __builtin_amdgcn_sqrtf(d2);
        return (1.0f + ar + ar * ar * (1.0f / 3.0f)) * __builtin_amdgcn_exp2f(c0 * ar);
    }
};
template <> struct NearKernel<FKT_RATQUAD, float> {
    static constexpr bool kTable = false;
    static constexpr float kBias = 0.0f;
    static __device__ __forceinline__ float eval(float d2, float c0, float c1, const double*)
    {
        return __builtin_amdgcn_exp2f(c1 * __builtin_amdgcn_logf(1.0f + c0 * d2));
    }
};
template <> struct NearKernel<FKT_CAUCHY, float> {
    static constexpr bool kTable = false;
    static constexpr float kBias = 0.0f;
    static __device__ __forceinline__ float eval(float d2, float c0, float, const double*)
    {
        return __builtin_amdgcn_rcpf(1.0f + c0 * d2);
    }
};
template <> struct NearKernel<FKT_LAPLACE, float> {
    static constexpr bool kTable = false;
    static constexpr float kBias = 0.0f;
    static __device__ __forceinline__ float eval(float d2, float, float, const double*)
    {
        return d2 > 0.0f ? __builtin_amdgcn_rsqf(d2) : 0.0f;
    }
};

// One near unit u (wave-uniform): a source leaf and up to kNearUnitTargets
// of its targets, 64 at a time. With NCOL columns each kernel value
// multiplies NCOL weights. tab: the exponential table in LDS (FP64 kernels
// that use it).
template <int D, int KIND, typename T, int NCOL>
__device__ __forceinline__ void near_unit(const DevPlan& a, int u, const T* __restrict__ src, T* __restrict__ zacc,
                                          T c0, T c1, T scale, const double* tab)
{
    constexpr int S = src_stride(D, NCOL);
    using NK = NearKernel<KIND, T>;
    const int lane = threadIdx.x & 63;
    if (a.inst_active && !a.inst_active[a.nu_inst[u]]) return;
    const int s0 = a.nu_beg[u], m = a.nu_end[u] - s0;
    const int toff = a.nu_toff[u], tcnt = a.nu_tcnt[u];
    const T* __restrict__ q = src + (size_t)s0 * S;
    for (int c = 0; c < tcnt; c += kWave) {
        const int i = c + lane;
        const bool valid = i < tcnt;
        const int t = a.near_tgt[toff + (valid ? i : 0)];
        T tx[D];
#pragma unroll
        for (int k = 0; k < D; ++k) tx[k] = src[(size_t)t * S + k];
        auto kval = [&](const T* __restrict__ p) {
            T d2 = T(NK::kBias);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const T w = tx[k] - p[k];
                d2 = fma(w, w, d2);
            }
            return NK::eval(d2, c0, c1, tab);
        };
        if constexpr (NCOL == 1) {
            auto pair = [&](const T* __restrict__ p) { return kval(p) * p[D]; };
            T acc0 = T(0), acc1 = T(0);
            int s = 0;
            for (; s + 4 <= m; s += 4) {
                acc0 += pair(q + (s + 0) * S);
                acc1 += pair(q + (s + 1) * S);
                acc0 += pair(q + (s + 2) * S);
                acc1 += pair(q + (s + 3) * S);
            }
            for (; s < m; ++s) acc0 += pair(q + s * S);
            if (valid) unsafeAtomicAdd(zacc + t, scale * (acc0 + acc1));
        } else {
            T acc[2][NCOL];
#pragma unroll
            for (int c = 0; c < NCOL; ++c) acc[0][c] = acc[1][c] = T(0);
            auto pair = [&](const T* __restrict__ p, T (&ac)[NCOL]) {
                const T kv = kval(p);
#pragma unroll
                for (int c = 0; c < NCOL; ++c) ac[c] = fma(kv, p[D + c], ac[c]);
            };
            int s = 0;
            for (; s + 2 <= m; s += 2) {
                pair(q + (s + 0) * S, acc[0]);
                pair(q + (s + 1) * S, acc[1]);
            }
            if (s < m) pair(q + s * S, acc[0]);
            if (valid) {
#pragma unroll
                for (int c = 0; c < NCOL; ++c) unsafeAtomicAdd(zacc + (size_t)t * NCOL + c, scale * (acc[0][c] + acc[1][c]));
            }
        }
    }
}

// Source-major near field: one wave per work unit (a source leaf l and up to
// kNearUnitTargets targets of N_l, 64 at a time, one per lane). The leaf's
// points stream through scalar registers; each target's sum is added to its
// accumulator with one FP64/FP32 atomic per (target, leaf), so no lane ever
// idles on a target whose own walk does not reach l.
template <int D, int KIND, typename T, int NCOL = 1>
__global__ __launch_bounds__(kWave) void k_near(const DevPlan a, const T* __restrict__ src, T* __restrict__ zacc,
                                                T c0, T c1, T scale)
{
    using NK = NearKernel<KIND, T>;
    __shared__ double tab[NK::kTable ? kExpTabLen : 1];
    const int lane = threadIdx.x;
    if constexpr (NK::kTable) {
        double tv[kExpTabLen / kWave];
#pragma unroll
        for (int j = 0; j < kExpTabLen / kWave; ++j) tv[j] = a.exp2tab[j * kWave + lane];
#pragma unroll
        for (int j = 0; j < kExpTabLen / kWave; ++j) tab[j * kWave + lane] = tv[j];
        __syncthreads();
    }
    near_unit<D, KIND, T, NCOL>(a, blockIdx.x, src, zacc, c0, c1, scale, tab);
}

// Near and far field in one persistent launch over a global work queue
// (the accumulators and moments are those of the pass; the counter is
// cleared by the gather kernel). Every wave takes the next item with one
// atomic: items alternate between a chunk of kFusedJobs node-major far jobs
// and one near unit while both remain, so each SIMD holds waves of both
// kinds (the far jobs are heavy in scalar instructions, the near units in
// vector ones, and the two issue side by side); a wave exits when the queue
// is empty, so every wave reaches the end.
constexpr int kFusedJobs = 8;

template <int D, int P, int KIND, typename T, int NCOL>
__global__ __launch_bounds__(256) void k_fused(const DevPlan a, const T* __restrict__ src, const T* __restrict__ mom,
                                               size_t cs, T* __restrict__ zacc, unsigned* __restrict__ ctr, T c0,
                                               T c1, T scale)
{
    using NK = NearKernel<KIND, T>;
    __shared__ double tab[NK::kTable ? kExpTabLen : 1];
    if constexpr (NK::kTable) {
        for (int j = threadIdx.x; j < kExpTabLen; j += blockDim.x) tab[j] = a.exp2tab[j];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int nm = (a.nnjobs + kFusedJobs - 1) / kFusedJobs;
    const int nu = a.nnear_units;
    const int both = nm < nu ? nm : nu;
    const int total = nm + nu;
    for (;;) {
        int item = 0;
        if (lane == 0) item = (int)atomicAdd(ctr, 1u);
        item = __builtin_amdgcn_readlane(item, 0);
        if (item >= total) break;
        bool far;
        int idx;
        if (item < 2 * both) {
            far = (item & 1) == 0;
            idx = item >> 1;
        } else {
            far = nm > nu;
            idx = both + (item - 2 * both);
        }
        if (far) {
            const int j1 = min(a.nnjobs, (idx + 1) * kFusedJobs);
#pragma unroll 1
            for (int j = idx * kFusedJobs; j < j1; ++j) m2t_node_job<D, P, KIND, T, 0, NCOL>(a, j, mom, cs, zacc);
        } else {
            near_unit<D, KIND, T, NCOL>(a, idx, src, zacc, c0, c1, scale, tab);
        }
    }
}

// y (caller order, columns col .. col + ncols - 1) <- zacc (tree order, [n][NC])
template <typename T, int NC = 1>
__global__ __launch_bounds__(256) void k_scatter(int n, const int64_t* __restrict__ perm, const T* __restrict__ zacc,
                                                 T* __restrict__ y, int nrhs, int col, int ncols)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t row = perm[i] * nrhs + col;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < ncols) y[row + c] = zacc[(size_t)i * NC + c];
}

// ------------------------------------------------- built orders per dimension

template <int D> struct PMax;
template <> struct PMax<3> { static constexpr int value = 8; };
template <> struct PMax<4> { static constexpr int value = 8; };
template <> struct PMax<5> { static constexpr int value = 8; };

// s2m moment entries accumulated per lane and launch: the rank split into
// equal chunks of at most 48 FP64 or 96 FP32 accumulators (96 or 192 bytes
// of registers per lane), so a unit keeps several waves per SIMD; every
// chunk regenerates the harmonics, which costs less than the accumulation.
template <typename T>
constexpr int s2m_chunk(int R)
{
    const int cap = sizeof(T) == 8 ? 48 : 96;
    const int nch = (R + cap - 1) / cap;
    return (R + nch - 1) / nch;
}

}  // namespace

// Launchers implemented in the per-stage translation units.
// nc: columns of the pass, 1 or kMvmCols (moments [column][slot][entry]).
bool launch_s2m(const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc = 1);
#define FKT_DECLARE_S2M(D, PR) \
    bool launch_s2m_d##D##_p##PR(const DevPlan& a, const DevWork& wk, hipStream_t s, int nc);
FKT_DECLARE_S2M(3, 0)
FKT_DECLARE_S2M(3, 1)
FKT_DECLARE_S2M(4, 0)
FKT_DECLARE_S2M(4, 1)
FKT_DECLARE_S2M(5, 0)
FKT_DECLARE_S2M(5, 1)
#undef FKT_DECLARE_S2M
bool launch_m2t(int kind, const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc = 1);
// near and far field in one persistent launch (k_fused); c0, c1, scale: the
// near-kernel constants in the pass's precision (as doubles)
bool launch_fused(int kind, const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc, double c0,
                  double c1, double scale);
#define FKT_DECLARE_FUSED(K)                                                                                      \
    bool launch_fused_kind##K(const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc, double c0, \
                              double c1, double scale);
FKT_DECLARE_FUSED(0)
FKT_DECLARE_FUSED(1)
FKT_DECLARE_FUSED(2)
FKT_DECLARE_FUSED(3)
FKT_DECLARE_FUSED(4)
FKT_DECLARE_FUSED(5)
FKT_DECLARE_FUSED(6)
#undef FKT_DECLARE_FUSED
#define FKT_DECLARE_M2T(K) \
    bool launch_m2t_kind##K(const DevPlan& a, const DevWork& wk, int prec, hipStream_t s, int nc);
FKT_DECLARE_M2T(0)
FKT_DECLARE_M2T(1)
FKT_DECLARE_M2T(2)
FKT_DECLARE_M2T(3)
FKT_DECLARE_M2T(4)
FKT_DECLARE_M2T(5)
FKT_DECLARE_M2T(6)
#undef FKT_DECLARE_M2T

}  // namespace fkt
