// HIP kernels of the FKT matrix-vector product for CDNA4 (gfx950).
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

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// ------------------------------------------------------------ harmonics
//
// All solid harmonics of degree <= P of x (D coordinates), each handed to
// emit(integral_constant<degree>, value). A degree-k harmonic in e dims is
//   G_{k-mu}^{lam}(x_{e-1}; rho_e^2) * H_mu(x_0..x_{e-2}),  lam = mu + (e-2)/2,
// with G_n^lam(z; rho^2) = rho^n C_n^lam(z / rho) from the Gegenbauer
// three-term recurrence (Appendix A.1) multiplied through by rho^n, and H_mu
// a degree-mu harmonic of one dimension less; in two dimensions the
// harmonics are Re and Im of (x_0 + i x_1)^m. hn supplies the per-level
// normalisation (and sqrt(Z_k) at the top level).
template <int E, int P, typename T, class Emit>
__device__ __forceinline__ void harmonics(const T* x, const T* rho2, const T* __restrict__ hn, Emit& emit)
{
    if constexpr (E == 2) {
        T cr = T(1), ci = T(0);
        auto base = [&](auto mc) {
            constexpr int m = decltype(mc)::value;
            if constexpr (m == 0) {
                emit(mc, T(0.398942280401432677939946));  // 1 / sqrt(2 pi)
            } else {
                const T nr = cr * x[0] - ci * x[1];
                const T ni = cr * x[1] + ci * x[0];
                cr = nr;
                ci = ni;
                emit(mc, cr * T(0.564189583547756286948079));  // 1 / sqrt(pi)
                emit(mc, ci * T(0.564189583547756286948079));
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
                emit(std::integral_constant<int, mu + n>{}, H * (g * hn[((E - 3) * (P + 1) + mu) * (P + 1) + n]));
            };
            static_for<0, P - mu + 1>(step);
        };
        harmonics<E - 1, P, T>(x, rho2, hn, level);
    }
}

// ------------------------------------------------------- radial derivatives
//
// K^(m)(r), m = 0..P, in FP64 (closed forms / recurrences per kernel).
template <int P>
__device__ __forceinline__ void radial_derivs(const DevPlan& a, double r, double (&D)[P + 1])
{
    const double var = a.var;
    switch (a.kind) {
    case FKT_GAUSSIAN: {  // exp(-u^2), u = r s: d^m/dr^m = (-s)^m H_m(u) exp(-u^2)
        const double s = 0.70710678118654752440 / a.ell, u = r * s, e = var * exp(-u * u);
        double h1 = 1.0, h2 = 0.0, sc = 1.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            double h = (m == 0) ? 1.0 : 2.0 * u * h1 - 2.0 * (m - 1) * h2;
            if (m >= 1) { h2 = h1; h1 = h; }
            D[m] = sc * h * e;
            sc *= -s;
        }
        break;
    }
    case FKT_EXPONENTIAL: {
        const double c = 1.0 / a.ell, e = var * exp(-c * r);
        double sc = 1.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) { D[m] = sc * e; sc *= -c; }
        break;
    }
    case FKT_MATERN32: {  // (1 + cr) e^{-cr}: (-c)^m (1 - m + cr) e^{-cr}
        const double c = 1.7320508075688772935 / a.ell, cr = c * r, e = var * exp(-cr);
        double sc = 1.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) { D[m] = sc * (1.0 - m + cr) * e; sc *= -c; }
        break;
    }
    case FKT_MATERN52: {  // Q e^{-cr}, Q = 1 + cr + (cr)^2/3 (Leibniz rule)
        const double c = 2.2360679774997896964 / a.ell, cr = c * r, e = var * exp(-cr);
        const double q0 = 1.0 + cr + cr * cr / 3.0, q1 = c + 2.0 * c * cr / 3.0, q2 = 2.0 * c * c / 3.0;
        double s0 = 1.0, s1 = 0.0, s2 = 0.0;  // (-c)^m, (-c)^(m-1), (-c)^(m-2)
#pragma unroll
        for (int m = 0; m <= P; ++m) {
            D[m] = e * (s0 * q0 + m * s1 * q1 + 0.5 * m * (m - 1) * s2 * q2);
            s2 = s1;
            s1 = (m == 0) ? 1.0 : s1 * -c;
            s0 *= -c;
        }
        break;
    }
    case FKT_RATQUAD:
    case FKT_CAUCHY: {  // w(r+h)^beta, w quadratic in h: J.C.P. Miller's power recurrence
        double g0, g1, g2, beta;
        if (a.kind == FKT_RATQUAD) {
            const double c = 0.5 / (a.alpha * a.ell * a.ell);
            g0 = 1.0 + c * r * r; g1 = 2.0 * c * r; g2 = c; beta = -a.alpha;
        } else {
            const double c = 1.0 / (a.ell * a.ell);
            g0 = 1.0 + c * r * r; g1 = 2.0 * c * r; g2 = c; beta = -1.0;
        }
        const double ig0 = 1.0 / g0;
        double f[P + 1];
        f[0] = (a.kind == FKT_CAUCHY) ? ig0 : pow(g0, beta);
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
        break;
    }
    case FKT_LAPLACE: {  // 1/r: (-1)^m m! / r^(m+1)
        const double ir = 1.0 / r;
        D[0] = var * ir;
#pragma unroll
        for (int m = 1; m <= P; ++m) D[m] = D[m - 1] * (-(double)m) * ir;
        break;
    }
    default:
#pragma unroll
        for (int m = 0; m <= P; ++m) D[m] = 0.0;
    }
}

template <typename T> __device__ __forceinline__ const T* hn_ptr(const DevPlan& a);
template <> __device__ __forceinline__ const double* hn_ptr<double>(const DevPlan& a) { return a.hn64; }
template <> __device__ __forceinline__ const float* hn_ptr<float>(const DevPlan& a) { return a.hn32; }

// ------------------------------------------------------------------ gather

template <typename T>
__global__ __launch_bounds__(256) void k_gather(int n, const int64_t* __restrict__ perm, const T* __restrict__ x,
                                                int nrhs, int col, T* __restrict__ w)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) w[i] = x[perm[i] * nrhs + col];
}

// --------------------------------------------------------------------- s2m
//
// Moments of every far node straight from its own points (Algorithm 1,
// source2mult; no translation between levels). One wave per work unit of at
// most kUnitPoints points of one node; each lane accumulates its points'
// contributions to moment entries [C0, C1) in registers, then the wave sums.
template <int D, int P, typename T, int C0, int C1>
__global__ __launch_bounds__(kWave) void k_s2m(const DevPlan a, const T* __restrict__ w, T* __restrict__ mom,
                                               T* __restrict__ part)
{
    constexpr int R = cbinom(P + D, D);
    constexpr int NC = C1 - C0;
    const int u = blockIdx.x;
    const int lane = threadIdx.x;
    const int slot = a.unit_slot[u];
    const int beg = a.unit_begin[u], end = a.unit_end[u];
    double c[D];
#pragma unroll
    for (int i = 0; i < D; ++i) c[i] = a.slot_ctr[slot * D + i];
    const double is = 1.0 / a.slot_scale[slot];
    const T* __restrict__ hn = hn_ptr<T>(a);

    T acc[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) acc[i] = T(0);

    for (int s = beg + lane; s < end; s += kWave) {
        T x[D], rho2[D + 1];
        rho2[0] = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            x[i] = T((a.pts64[(size_t)s * D + i] - c[i]) * is);
            rho2[i + 1] = rho2[i] + x[i] * x[i];
        }
        T q[P / 2 + 1];
        q[0] = w[s];
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
        harmonics<D, P, T>(x, rho2, hn, emit);
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
// Far field of every target: for each far node of its own walk, the radial
// functions (FP64) and the harmonics of the direction to the target,
// contracted with the node's moments.
template <int D, int P, typename T>
__global__ __launch_bounds__(kWave) void k_m2t(const DevPlan a, const T* __restrict__ mom, T* __restrict__ zfar)
{
    constexpr int R = cbinom(P + D, D);
    constexpr int NF = f_off(P, P + 1);
    const int blk = blockIdx.x;
    const int lane = threadIdx.x;
    const int tb = a.blk_begin[blk], cnt = a.blk_count[blk];
    const bool valid = lane < cnt;
    const int t = tb + (valid ? lane : 0);
    double tx[D];
#pragma unroll
    for (int i = 0; i < D; ++i) tx[i] = a.pts64[(size_t)t * D + i];
    const T* __restrict__ hn = hn_ptr<T>(a);
    const double* __restrict__ tbar = a.tbar;

    T acc = T(0);
    const int e0 = a.far_off[blk], e1 = a.far_off[blk + 1];
    for (int e = e0; e < e1; ++e) {
        const uint64_t msk = a.far_mask[e];
        if (!((msk >> lane) & 1)) continue;
        const int slot = a.far_slot[e];
        double r[D], r2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            r[i] = tx[i] - a.slot_ctr[slot * D + i];
            r2 += r[i] * r[i];
        }
        const double rr = sqrt(r2), ir = 1.0 / rr;
        double Dm[P + 1];
        radial_derivs<P>(a, rr, Dm);
        double um[P + 1];  // K^(m)(r) r^m
        um[0] = Dm[0];
        double rp = 1.0;
#pragma unroll
        for (int m = 1; m <= P; ++m) { rp *= rr; um[m] = Dm[m] * rp; }
        const double v = a.slot_scale[slot] * ir;  // s / |r|  (< theta)
        double vp[P + 1];
        vp[0] = 1.0;
#pragma unroll
        for (int j = 1; j <= P; ++j) vp[j] = vp[j - 1] * v;
        // F[k][jj] = (s/|r|)^j (F_kj(|r|) |r|^j), j = k + 2 jj
        T F[NF];
        auto radial_k = [&](auto kc) {
            constexpr int k = decltype(kc)::value;
            auto radial_j = [&](auto jc) {
                constexpr int jj = decltype(jc)::value;
                constexpr int j = k + 2 * jj;
                double s = (j == 0) ? um[0] : 0.0;
#pragma unroll
                for (int m = 1; m <= j; ++m) s += um[m] * tbar[(k * (P + 1) + j) * (P + 1) + m];
                F[f_off(P, k) + jj] = T(vp[j] * s);
            };
            static_for<0, nj_of(P, k)>(radial_j);
        };
        static_for<0, P + 1>(radial_k);

        T x[D], rho2[D + 1];
        rho2[0] = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            x[i] = T(r[i] * ir);
            rho2[i + 1] = rho2[i] + x[i] * x[i];
        }
        const T* __restrict__ M = mom + (size_t)slot * R;
        int off = 0;
        auto emit = [&](auto kc, T y) {
            constexpr int k = decltype(kc)::value;
            constexpr int nj = nj_of(P, k);
            T s = T(0);
            auto dot = [&](auto jc) {
                constexpr int jj = decltype(jc)::value;
                s += F[f_off(P, k) + jj] * M[off + jj];
            };
            static_for<0, nj>(dot);
            acc += y * s;
            off += nj;
        };
        harmonics<D, P, T>(x, rho2, hn, emit);
    }
    if (valid) zfar[t] = acc;
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

template <> struct NearKernel<FKT_GAUSSIAN, double> {
    static __device__ __forceinline__ double eval(double d2, double c0, double) { return exp(c0 * d2); }
};
template <> struct NearKernel<FKT_EXPONENTIAL, double> {
    static __device__ __forceinline__ double eval(double d2, double c0, double) { return exp(c0 * sqrt(d2)); }
};
template <> struct NearKernel<FKT_MATERN32, double> {
    static __device__ __forceinline__ double eval(double d2, double c0, double)
    {
        const double ar = c0 * sqrt(d2);
        return (1.0 + ar) * exp(-ar);
    }
};
template <> struct NearKernel<FKT_MATERN52, double> {
    static __device__ __forceinline__ double eval(double d2, double c0, double)
    {
        const double ar = c0 * sqrt(d2);
        return (1.0 + ar + ar * ar * (1.0 / 3.0)) * exp(-ar);
    }
};
template <> struct NearKernel<FKT_RATQUAD, double> {
    static __device__ __forceinline__ double eval(double d2, double c0, double c1) { return pow(1.0 + c0 * d2, c1); }
};
template <> struct NearKernel<FKT_CAUCHY, double> {
    static __device__ __forceinline__ double eval(double d2, double c0, double) { return 1.0 / (1.0 + c0 * d2); }
};
template <> struct NearKernel<FKT_LAPLACE, double> {
    static __device__ __forceinline__ double eval(double d2, double, double) { return d2 > 0.0 ? rsqrt(d2) : 0.0; }
};

// FP32: hardware transcendental approximations (v_exp_f32 / v_log_f32 are
// base 2; c0 is pre-scaled by log2(e) where an exponential follows).
template <> struct NearKernel<FKT_GAUSSIAN, float> {
    static __device__ __forceinline__ float eval(float d2, float c0, float) { return __builtin_amdgcn_exp2f(c0 * d2); }
};
template <> struct NearKernel<FKT_EXPONENTIAL, float> {
    static __device__ __forceinline__ float eval(float d2, float c0, float)
    {
        return __builtin_amdgcn_exp2f(c0 * __builtin_amdgcn_sqrtf(d2));
    }
};
template <> struct NearKernel<FKT_MATERN32, float> {
    static __device__ __forceinline__ float eval(float d2, float c0, float c1)
    {
        const float r = __builtin_amdgcn_sqrtf(d2);
        return (1.0f + c1 * r) * __builtin_amdgcn_exp2f(c0 * r);
    }
};
template <> struct NearKernel<FKT_MATERN52, float> {
    static __device__ __forceinline__ float eval(float d2, float c0, float c1)
    {
        const float ar = c1 * __builtin_amdgcn_sqrtf(d2);
        return (1.0f + ar + ar * ar * (1.0f / 3.0f)) * __builtin_amdgcn_exp2f(c0 * ar);
    }
};
template <> struct NearKernel<FKT_RATQUAD, float> {
    static __device__ __forceinline__ float eval(float d2, float c0, float c1)
    {
        return __builtin_amdgcn_exp2f(c1 * __builtin_amdgcn_logf(1.0f + c0 * d2));
    }
};
template <> struct NearKernel<FKT_CAUCHY, float> {
    static __device__ __forceinline__ float eval(float d2, float c0, float)
    {
        return __builtin_amdgcn_rcpf(1.0f + c0 * d2);
    }
};
template <> struct NearKernel<FKT_LAPLACE, float> {
    static __device__ __forceinline__ float eval(float d2, float, float)
    {
        return d2 > 0.0f ? __builtin_amdgcn_rsqf(d2) : 0.0f;
    }
};

template <int D, int KIND, typename T>
__global__ __launch_bounds__(kWave) void k_near(const DevPlan a, const T* __restrict__ pts, const T* __restrict__ w,
                                                const T* __restrict__ zfar, T* __restrict__ y, int nrhs, int col,
                                                T c0, T c1, T scale)
{
    const int blk = blockIdx.x;
    const int lane = threadIdx.x;
    const int tb = a.blk_begin[blk], cnt = a.blk_count[blk];
    const bool valid = lane < cnt;
    const int t = tb + (valid ? lane : 0);
    T tx[D];
#pragma unroll
    for (int i = 0; i < D; ++i) tx[i] = pts[(size_t)t * D + i];
    T acc = T(0);
    const int e0 = a.near_off[blk], e1 = a.near_off[blk + 1];
    for (int e = e0; e < e1; ++e) {
        const uint64_t msk = a.near_mask[e];
        if (!((msk >> lane) & 1)) continue;
        const int s0 = a.near_beg[e], s1 = a.near_end[e];
        for (int s = s0; s < s1; ++s) {
            T d2 = T(0);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const T u = tx[i] - pts[(size_t)s * D + i];
                d2 += u * u;
            }
            acc += NearKernel<KIND, T>::eval(d2, c0, c1) * w[s];
        }
    }
    if (valid) {
        T out = scale * acc;
        if (zfar) out += zfar[t];
        y[a.perm[t] * nrhs + col] = out;
    }
}

// ---------------------------------------------------------------- dispatch

template <int D> struct PMax;
template <> struct PMax<3> { static constexpr int value = 8; };
template <> struct PMax<4> { static constexpr int value = 6; };
template <> struct PMax<5> { static constexpr int value = 6; };

constexpr int kChunk = 128;  // s2m moment entries accumulated per lane and launch

template <int D, int P, typename T, int C0>
void launch_s2m_chunks(const DevPlan& a, const T* w, T* mom, T* part, hipStream_t s)
{
    constexpr int R = cbinom(P + D, D);
    if constexpr (C0 < R) {
        constexpr int C1 = (C0 + kChunk < R) ? C0 + kChunk : R;
        hipLaunchKernelGGL((k_s2m<D, P, T, C0, C1>), dim3(a.nunits), dim3(kWave), 0, s, a, w, mom, part);
        launch_s2m_chunks<D, P, T, C1>(a, w, mom, part, s);
    }
}

template <int D, int P, typename T>
void far_field(const DevPlan& a, const DevWork& wk, hipStream_t s, hipEvent_t* ev)
{
    constexpr int R = cbinom(P + D, D);
    const T* w = (const T*)wk.w;
    T* mom = (T*)wk.mom;
    T* part = (T*)wk.part;
    launch_s2m_chunks<D, P, T, 0>(a, w, mom, part, s);
    if (a.nred > 0) {
        const int64_t tot = (int64_t)a.nred * R;
        hipLaunchKernelGGL((k_s2m_reduce<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a.nred, R,
                           a.red_slot, a.red_off, part, mom);
    }
    if (ev) (void)hipEventRecord(ev[2], s);
    hipLaunchKernelGGL((k_m2t<D, P, T>), dim3(a.nblocks), dim3(kWave), 0, s, a, (const T*)mom, (T*)wk.zfar);
}

template <int D, typename T, int P = 0>
bool dispatch_far(int p, const DevPlan& a, const DevWork& wk, hipStream_t s, hipEvent_t* ev)
{
    if constexpr (P > PMax<D>::value) {
        return false;
    } else {
        if (p == P) { far_field<D, P, T>(a, wk, s, ev); return true; }
        return dispatch_far<D, T, P + 1>(p, a, wk, s, ev);
    }
}

template <typename T>
bool run_far(const DevPlan& a, const DevWork& wk, hipStream_t s, hipEvent_t* ev)
{
    switch (a.d) {
    case 3: return dispatch_far<3, T>(a.p, a, wk, s, ev);
    case 4: return dispatch_far<4, T>(a.p, a, wk, s, ev);
    case 5: return dispatch_far<5, T>(a.p, a, wk, s, ev);
    default: return false;
    }
}

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

template <int D, typename T>
bool run_near_d(const DevPlan& a, const T* pts, const T* w, const T* zfar, T* y, int nrhs, int col, hipStream_t s)
{
    T c0, c1;
    near_consts<T>(a, c0, c1);
    const T scale = (T)a.var;
    dim3 g(a.nblocks), b(kWave);
    switch (a.kind) {
#define FKT_NEAR_CASE(K) \
    case K: hipLaunchKernelGGL((k_near<D, K, T>), g, b, 0, s, a, pts, w, zfar, y, nrhs, col, c0, c1, scale); return true;
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

template <typename T>
hipError_t mvm_column(const DevPlan& a, const DevWork& wk, const T* x, T* y, int nrhs, int col, hipStream_t s,
                      hipEvent_t* ev)
{
    const T* pts = std::is_same<T, float>::value ? (const T*)a.pts32 : (const T*)a.pts64;
    if (ev) (void)hipEventRecord(ev[0], s);
    hipLaunchKernelGGL((k_gather<T>), dim3((a.n + 255) / 256), dim3(256), 0, s, a.n, a.perm, x, nrhs, col, (T*)wk.w);
    if (ev) (void)hipEventRecord(ev[1], s);
    const T* zfar = nullptr;
    if (a.nslots > 0) {
        if (!run_far<T>(a, wk, s, ev)) return hipErrorInvalidValue;
        zfar = (const T*)wk.zfar;
    } else if (ev) {
        (void)hipEventRecord(ev[2], s);
    }
    if (ev) (void)hipEventRecord(ev[3], s);
    bool ok = false;
    switch (a.d) {
    case 3: ok = run_near_d<3, T>(a, pts, (const T*)wk.w, zfar, y, nrhs, col, s); break;
    case 4: ok = run_near_d<4, T>(a, pts, (const T*)wk.w, zfar, y, nrhs, col, s); break;
    case 5: ok = run_near_d<5, T>(a, pts, (const T*)wk.w, zfar, y, nrhs, col, s); break;
    default: break;
    }
    if (!ok) return hipErrorInvalidValue;
    if (ev) (void)hipEventRecord(ev[4], s);
    return hipGetLastError();
}

}  // namespace

bool far_supported(int d, int p)
{
    switch (d) {
    case 3: return p >= 0 && p <= PMax<3>::value;
    case 4: return p >= 0 && p <= PMax<4>::value;
    case 5: return p >= 0 && p <= PMax<5>::value;
    default: return false;
    }
}

hipError_t launch_mvm_column(const DevPlan& a, const DevWork& wk, const void* x, void* y, int nrhs, int col, int prec,
                             hipStream_t s, hipEvent_t* ev)
{
    if (prec == 1) return mvm_column<float>(a, wk, (const float*)x, (float*)y, nrhs, col, s, ev);
    return mvm_column<double>(a, wk, (const double*)x, (double*)y, nrhs, col, s, ev);
}

}  // namespace fkt
