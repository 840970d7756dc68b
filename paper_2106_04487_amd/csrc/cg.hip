// Conjugate gradients on (K~ + sigma2 I) x = b with the FKT MVM as operator.
//
// The paper computes Gaussian-process posterior means through kernel MVMs
// only (Sec. 5.3 and eq. gp_posterior); this is the solve that needs. The CG
// vectors and scalars are FP64 whatever the plan's precision; the operator
// runs in the plan's precision (inputs and outputs converted on the fly).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fkt.h"
#include "fkt_device.h"
#include "fkt_learn.h"

namespace {

constexpr int kThreads = 256;
constexpr int kDotBlocks = 512;
constexpr double kReplaceDrop = 0.1;  // residual replacement after each drop by this factor

template <typename T>
__global__ __launch_bounds__(kThreads) void k_to_f64(int64_t m, const T* __restrict__ a, double* __restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < m) b[i] = (double)a[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_from_f64(int64_t m, const double* __restrict__ a, T* __restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < m) b[i] = (T)a[i];
}

// q = Kp_op (plan precision) + sigma2 p ; then per-block partial dots of p.q
template <typename T>
__global__ __launch_bounds__(kThreads) void k_add_shift(int64_t m, const T* __restrict__ kp, const double* __restrict__ p,
                                                        double sigma2, double* __restrict__ q)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < m) q[i] = (double)kp[i] + sigma2 * p[i];
}

// Systems: the rows of segment s (rows [seg_off[s], seg_off[s + 1]): one
// instance of a batched plan, or all rows) and column c form system
// s * nrhs + c, with its own CG scalars.
// partial[s][blk][c] = sum over the rows of segment s in block-stride of a[i][c] * b[i][c]
// (bps blocks per segment: block blockIdx.x is block blockIdx.x % bps of
// segment blockIdx.x / bps)
__global__ __launch_bounds__(kThreads) void k_dot_partial(int nrhs, int bps, const int64_t* __restrict__ seg_off,
                                                          const double* __restrict__ a, const double* __restrict__ b,
                                                          double* __restrict__ partial)
{
    __shared__ double sh[kThreads];
    const int seg = blockIdx.x / bps, blk = blockIdx.x % bps;
    const int64_t r0 = seg_off[seg], r1 = seg_off[seg + 1];
    for (int c = 0; c < nrhs; ++c) {
        double s = 0.0;
        for (int64_t i = r0 + (int64_t)blk * kThreads + threadIdx.x; i < r1; i += (int64_t)bps * kThreads)
            s += a[i * nrhs + c] * b[i * nrhs + c];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int o = kThreads / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * nrhs + c] = sh[0];
        __syncthreads();
    }
}

// system of element g = i * nrhs + c (row_seg: segment of each row, or NULL
// for one segment)
__device__ __forceinline__ int64_t system_of(int64_t g, int nrhs, const int* __restrict__ row_seg)
{
    const int c = (int)(g % nrhs);
    return row_seg ? (int64_t)row_seg[g / nrhs] * nrhs + c : c;
}

// y[i][c] += alpha[system] * x[i][c]
__global__ __launch_bounds__(kThreads) void k_axpy(int64_t n, int nrhs, const int* __restrict__ row_seg,
                                                   const double* __restrict__ alpha, const double* __restrict__ x,
                                                   double* __restrict__ y)
{
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g < n * nrhs) y[g] += alpha[system_of(g, nrhs, row_seg)] * x[g];
}

// p[i][c] = r[i][c] + beta[system] * p[i][c]
__global__ __launch_bounds__(kThreads) void k_xpby(int64_t n, int nrhs, const int* __restrict__ row_seg,
                                                   const double* __restrict__ r, const double* __restrict__ beta,
                                                   double* __restrict__ p)
{
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g < n * nrhs) p[g] = r[g] + beta[system_of(g, nrhs, row_seg)] * p[g];
}

// r = b - q
__global__ __launch_bounds__(kThreads) void k_sub(int64_t m, const double* __restrict__ b, const double* __restrict__ q,
                                                  double* __restrict__ r)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < m) r[i] = b[i] - q[i];
}

// z[:, c] = blockdiag((K_ll + sigma2 I)^-1) r[:, c]: one workgroup per leaf;
// the leaf's residual entries are gathered through the tree permutation into
// LDS, each thread forms rows of the (symmetric) inverse block times it.
__global__ __launch_bounds__(kThreads) void k_bj_apply(const int* __restrict__ begin, const int* __restrict__ count,
                                                       const int64_t* __restrict__ off, const double* __restrict__ inv,
                                                       const int64_t* __restrict__ perm, int nrhs, int col,
                                                       const double* __restrict__ r, double* __restrict__ z)
{
    extern __shared__ double rl[];
    const int l = blockIdx.x;
    const int b = begin[l], m = count[l];
    const double* __restrict__ A = inv + off[l];
    for (int j = threadIdx.x; j < m; j += kThreads) rl[j] = r[perm[b + j] * nrhs + col];
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += kThreads) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += A[(size_t)j * m + i] * rl[j];
        z[perm[b + i] * nrhs + col] = s;
    }
}

unsigned grid_of(int64_t m) { return (unsigned)((m + kThreads - 1) / kThreads); }

int cg_dot_blocks(int nseg) { return std::max(8, kDotBlocks / nseg); }

// CG work buffers: allocated per solve with hipMalloc, or carved (256-byte
// aligned) out of a caller-given region without allocating anything.
struct Buf {
    std::vector<void*> ptrs;
    char* region = nullptr;  // carve from here when set
    size_t used = 0, cap = 0;
    ~Buf()
    {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t get(size_t count, T** out)
    {
        const size_t bytes = sizeof(T) * (count ? count : 1);
        if (region) {
            const size_t need = (bytes + 255) / 256 * 256;
            if (used + need > cap) {
                *out = nullptr;
                return hipErrorOutOfMemory;
            }
            *out = (T*)(region + used);
            used += need;
            return hipSuccess;
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) ptrs.push_back(p);
        *out = (T*)p;
        return e;
    }
};

// Bytes of work buffers a solve needs (the carve of Buf::get, in its order):
// b, x, r, z, p, q (m doubles each), dot partials, coefficients, operator
// input and output (m plan elements each), and the learned filter's best
// iterate.
size_t cg_work_bytes(int64_t m, int nsys, int64_t npart, size_t es, bool best)
{
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t t = 6 * up(sizeof(double) * (size_t)m) + up(sizeof(double) * (size_t)npart) +
               up(sizeof(double) * 3 * (size_t)nsys) + 2 * up(es * (size_t)m);
    if (best) t += up(sizeof(double) * (size_t)m);
    return t;
}

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// ---------------------------------------------------- allocation-free solves
//
// Work buffers of fkt_cg_solve_noalloc: one file-scope device array, of which
// every GPU the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel or a copy (there it
// names a host-side stand-in): the address of each device's copy is looked
// up once, with that device current, and kept per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace fkt {
fkt_status cg_set_error(fkt_status st, const std::string& msg);

// Device address of `device`'s scratch array (that device must be current).
hipError_t cg_scratch(int device, void** ptr, size_t* bytes)
{
    *ptr = nullptr;
    *bytes = kScratchBytes;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* q = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = q;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

size_t cg_work_bytes_for(int64_t n, int nrhs, int nseg, size_t es, bool best)
{
    const int nsys = nseg * nrhs;
    return cg_work_bytes(n * nrhs, nsys, (int64_t)nseg * cg_dot_blocks(nseg) * nrhs, es, best);
}
}  // namespace fkt

namespace fkt {

// Safeguard of the learned preconditioner (when fallback_at is given): PCG
// with it falls back to block-Jacobi, restarted from the best iterate so far,
// once the residual has grown past kFallbackGrow times its best or has set no
// new best for kFallbackStall iterations.
constexpr double kFallbackGrow = 10.0;
constexpr int kFallbackStall = 250;

// T: element type of the MVM (the plan's precision); TI: element type of b
// and x at the boundary (T, or double for a mixed-precision solve on an FP32
// plan, whose iterate then never passes through FP32)
template <typename T, typename TI>
static fkt_status cg_typed(fkt_plan_t P, const CgPlanView& v, double sigma2, const TI* b_in, TI* x_io, int nrhs, double rtol,
                           int maxit, int precond, int* iters, double* relres, int64_t* fallback_at,
                           fkt_plan_t P64 = nullptr, const CgPlanView* v64 = nullptr, int* replaced = nullptr,
                           void* region = nullptr, size_t region_bytes = 0)
{
    const int64_t n = v.n, m = n * nrhs;
    // systems: (instance, column) pairs, each with its own CG scalars; a
    // converged system is frozen (alpha = beta = 0) while the others go on
    const int nseg = v.nseg, nsys = nseg * nrhs;
    const int bps = cg_dot_blocks(nseg);  // dot blocks per instance
    hipStream_t s = v.stream;
    Buf buf;
    buf.region = (char*)region;
    buf.cap = region_bytes;
    double *b, *x, *r, *z, *p, *q, *part, *coef, *xbest = nullptr, *q64 = nullptr;
    T *op_in, *op_out;
    hipError_t e;
    if ((e = buf.get(m, &b)) || (e = buf.get(m, &x)) || (e = buf.get(m, &r)) || (e = buf.get(m, &z)) ||
        (e = buf.get(m, &p)) || (e = buf.get(m, &q)) || (e = buf.get((size_t)nseg * bps * nrhs, &part)) ||
        (e = buf.get((size_t)3 * nsys, &coef)) || (e = buf.get(m, &op_in)) || (e = buf.get(m, &op_out)) ||
        (precond == 2 && fallback_at && (e = buf.get(m, &xbest))) || (P64 && (e = buf.get(m, &q64))))
        return cg_set_error(e == hipErrorOutOfMemory ? FKT_ENOMEM : FKT_EDEVICE, "cg work buffers");
    if (fallback_at) *fallback_at = -1;

    std::vector<double> hpart((size_t)nseg * bps * nrhs), hcoef((size_t)3 * nsys);
    // out[seg * nrhs + c] = (a1, a2) over the rows of instance seg, column c
    auto dots = [&](const double* a1, const double* a2, std::vector<double>& out) -> bool {
        hipLaunchKernelGGL(k_dot_partial, dim3((unsigned)(nseg * bps)), dim3(kThreads), 0, s, nrhs, bps, v.seg_off, a1,
                           a2, part);
        if (hipMemcpyAsync(hpart.data(), part, sizeof(double) * hpart.size(), hipMemcpyDeviceToHost, s) != hipSuccess)
            return false;
        if (hipStreamSynchronize(s) != hipSuccess) return false;
        out.assign(nsys, 0.0);
        for (int g = 0; g < nseg; ++g)
            for (int k = 0; k < bps; ++k)
                for (int c2 = 0; c2 < nrhs; ++c2)
                    out[(size_t)g * nrhs + c2] += hpart[((size_t)g * bps + k) * nrhs + c2];
        return true;
    };
    // masked: skip the operator work of instances whose systems have all
    // converged (their step length is 0, so their rows of the product are
    // not used); the flags are copied to the plan's buffer first
    std::vector<unsigned char> hact(v.active ? nseg : 0);
    auto apply = [&](const double* in, double* out, bool masked = false) -> fkt_status {
        hipLaunchKernelGGL((k_from_f64<T>), dim3(grid_of(m)), dim3(kThreads), 0, s, m, in, op_in);
        fkt_status st;
        if (masked && v.active) {
            if (hipMemcpyAsync(v.active, hact.data(), hact.size(), hipMemcpyHostToDevice, s) != hipSuccess)
                return cg_set_error(FKT_EDEVICE, "cg copy");
            st = mvm_masked(P, op_in, op_out, nrhs);
        } else {
            st = fkt_mvm(P, op_in, op_out, nrhs);
        }
        if (st != FKT_OK) return st;
        hipLaunchKernelGGL((k_add_shift<T>), dim3(grid_of(m)), dim3(kThreads), 0, s, m, op_out, in, sigma2, out);
        return FKT_OK;
    };
    auto precondition = [&](const double* in, double* out) -> bool {
        if (v.coarse && precond >= 1) {
            // two-level: block-Jacobi (h = 1 / lam) or the learned filter on
            // the residual leaf spectra, with the Nystrom coarse correction
            for (int c2 = 0; c2 < nrhs; ++c2)
                if (learn_apply(v.learn, in, out, nrhs, c2, s, precond == 1) != hipSuccess) return false;
            return true;
        }
        if (precond == 1) {
            for (int c2 = 0; c2 < nrhs; ++c2)
                hipLaunchKernelGGL(k_bj_apply, dim3(v.nleaf), dim3(kThreads), sizeof(double) * v.maxleaf, s, v.bj_begin,
                                   v.bj_count, v.bj_off, v.bj_inv, v.perm, nrhs, c2, in, out);
            return hipGetLastError() == hipSuccess;
        }
        if (precond == 2) {
            for (int c2 = 0; c2 < nrhs; ++c2)
                if (learn_apply(v.learn, in, out, nrhs, c2, s) != hipSuccess) return false;
            return true;
        }
        return hipMemcpyAsync(out, in, sizeof(double) * m, hipMemcpyDeviceToDevice, s) == hipSuccess;
    };

    hipLaunchKernelGGL((k_to_f64<TI>), dim3(grid_of(m)), dim3(kThreads), 0, s, m, b_in, b);
    hipLaunchKernelGGL((k_to_f64<TI>), dim3(grid_of(m)), dim3(kThreads), 0, s, m, (const TI*)x_io, x);
    std::vector<double> bb, rr, rz, pq, rz_new;
    // r = b - A x, z = M r, p = z, rz = (r, z), rr = (r, r)
    // refined solves: r = b - (K~64 + sigma2 I) x from the FP64 plan, on its
    // stream once this one has finished writing x
    auto residual64 = [&]() -> fkt_status {
        if (hipStreamSynchronize(s) != hipSuccess) return cg_set_error(FKT_EDEVICE, "cg sync");
        fkt_status st0 = fkt_mvm(P64, x, q64, nrhs);
        if (st0 != FKT_OK) return st0;
        hipLaunchKernelGGL((k_add_shift<double>), dim3(grid_of(m)), dim3(kThreads), 0, v64->stream, m, q64, x, sigma2,
                           q64);
        hipLaunchKernelGGL(k_sub, dim3(grid_of(m)), dim3(kThreads), 0, v64->stream, m, b, q64, r);
        if (hipStreamSynchronize(v64->stream) != hipSuccess) return cg_set_error(FKT_EDEVICE, "cg sync");
        if (replaced) ++*replaced;
        return FKT_OK;
    };
    // r = b - A x (from the FP64 plan in a refined solve), z = M r, p = z
    auto start = [&]() -> fkt_status {
        if (P64) {
            fkt_status st0 = residual64();
            if (st0 != FKT_OK) return st0;
        } else {
            fkt_status st0 = apply(x, q);
            if (st0 != FKT_OK) return st0;
            hipLaunchKernelGGL(k_sub, dim3(grid_of(m)), dim3(kThreads), 0, s, m, b, q, r);
        }
        if (!precondition(r, z)) return cg_set_error(FKT_EDEVICE, "cg preconditioner");
        if (hipMemcpyAsync(p, z, sizeof(double) * m, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return cg_set_error(FKT_EDEVICE, "cg copy");
        if (!dots(r, r, rr) || !dots(r, z, rz)) return cg_set_error(FKT_EDEVICE, "cg reduction");
        return FKT_OK;
    };
    if (!dots(b, b, bb)) return cg_set_error(FKT_EDEVICE, "cg reduction");
    if (replaced) *replaced = 0;
    fkt_status st = start();
    if (st != FKT_OK) return st;
    auto relres_of = [&](const std::vector<double>& rv, int j) {
        const double den = bb[j] > 0.0 ? std::sqrt(bb[j]) : 1.0;
        return std::sqrt(std::max(rv[j], 0.0)) / den;
    };
    auto worst = [&](const std::vector<double>& rv) {
        double w = 0.0;
        for (int j = 0; j < nsys; ++j) w = std::max(w, relres_of(rv, j));
        return w;
    };
    int it = 0;
    double res = worst(rr);
    double res_replaced = res;  // worst residual at the last replacement
    double best = res;
    int it_best = 0;
    if (xbest && hipMemcpyAsync(xbest, x, sizeof(double) * m, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return cg_set_error(FKT_EDEVICE, "cg copy");
    while (res > rtol && it < maxit) {
        if (xbest && precond == 2 && (res > kFallbackGrow * best || it - it_best >= kFallbackStall)) {
            // block-Jacobi from the best iterate (one extra operator application)
            precond = 1;
            if (fallback_at) *fallback_at = it;
            if (hipMemcpyAsync(x, xbest, sizeof(double) * m, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return cg_set_error(FKT_EDEVICE, "cg copy");
            if ((st = start()) != FKT_OK) return st;
            res = worst(rr);
            res_replaced = res;
            continue;
        }
        for (int g = 0; g < (int)hact.size(); ++g) {
            hact[g] = 0;
            for (int c2 = 0; c2 < nrhs; ++c2) hact[g] |= relres_of(rr, g * nrhs + c2) > rtol ? 1 : 0;
        }
        st = apply(p, q, true);
        if (st != FKT_OK) return st;
        if (!dots(p, q, pq)) return cg_set_error(FKT_EDEVICE, "cg reduction");
        // coef = [alpha | -alpha | beta]; host slots are rewritten only after
        // a stream synchronisation (inside dots) has retired the copy.
        std::vector<char> frozen(nsys);
        for (int j = 0; j < nsys; ++j) {
            frozen[j] = relres_of(rr, j) <= rtol;
            hcoef[j] = (!frozen[j] && pq[j] != 0.0) ? rz[j] / pq[j] : 0.0;
            hcoef[nsys + j] = -hcoef[j];
        }
        if (hipMemcpyAsync(coef, hcoef.data(), sizeof(double) * 2 * nsys, hipMemcpyHostToDevice, s) != hipSuccess)
            return cg_set_error(FKT_EDEVICE, "cg copy");
        hipLaunchKernelGGL(k_axpy, dim3(grid_of(m)), dim3(kThreads), 0, s, n, nrhs, v.row_seg, coef, p, x);
        hipLaunchKernelGGL(k_axpy, dim3(grid_of(m)), dim3(kThreads), 0, s, n, nrhs, v.row_seg, coef + nsys, q, r);
        if (!precondition(r, z)) return cg_set_error(FKT_EDEVICE, "cg preconditioner");
        if (!dots(r, r, rr) || !dots(r, z, rz_new)) return cg_set_error(FKT_EDEVICE, "cg reduction");
        if (P64 && (worst(rr) <= rtol || worst(rr) <= kReplaceDrop * res_replaced)) {
            // residual replacement: r = b - (K~64 + sigma2 I) x
            if ((st = residual64()) != FKT_OK) return st;
            if (!precondition(r, z)) return cg_set_error(FKT_EDEVICE, "cg preconditioner");
            if (!dots(r, r, rr) || !dots(r, z, rz_new)) return cg_set_error(FKT_EDEVICE, "cg reduction");
            res_replaced = worst(rr);
        }
        for (int j = 0; j < nsys; ++j) hcoef[2 * nsys + j] = (!frozen[j] && rz[j] != 0.0) ? rz_new[j] / rz[j] : 0.0;
        if (hipMemcpyAsync(coef + 2 * nsys, hcoef.data() + 2 * nsys, sizeof(double) * nsys, hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return cg_set_error(FKT_EDEVICE, "cg copy");
        hipLaunchKernelGGL(k_xpby, dim3(grid_of(m)), dim3(kThreads), 0, s, n, nrhs, v.row_seg, z, coef + 2 * nsys, p);
        rz = rz_new;
        ++it;
        res = worst(rr);
        if (xbest && precond == 2 && res < best) {
            best = res;
            it_best = it;
            if (hipMemcpyAsync(xbest, x, sizeof(double) * m, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return cg_set_error(FKT_EDEVICE, "cg copy");
        }
    }
    if (P64 && res > rtol) {
        // not converged: report the residual under the FP64 operator
        if ((st = residual64()) != FKT_OK) return st;
        if (!dots(r, r, rr)) return cg_set_error(FKT_EDEVICE, "cg reduction");
        res = worst(rr);
    }
    hipLaunchKernelGGL((k_from_f64<TI>), dim3(grid_of(m)), dim3(kThreads), 0, s, m, x, x_io);
    if (hipStreamSynchronize(s) != hipSuccess) return cg_set_error(FKT_EDEVICE, "cg sync");
    if (iters) *iters = it;
    if (relres) *relres = res;
    if (res > rtol) return cg_set_error(FKT_ENOTCONV, "cg reached maxit before rtol");
    return FKT_OK;
}

fkt_status cg_solve_impl(fkt_plan_t P, const CgPlanView& v, double sigma2, const void* b, void* x, int nrhs,
                         double rtol, int maxit, int precond, int* iters, double* relres, int64_t* fallback_at,
                         bool io64, fkt_plan_t P64, const CgPlanView* v64, int* replaced, void* region,
                         size_t region_bytes)
{
    if (precond < 0 || precond > 2 || (precond == 2 && !v.learn))
        return cg_set_error(FKT_EUNSUPPORTED, "unknown preconditioner");
    if (precond == 2) {
        // a zero output layer (initial weights, or a filter the judge
        // rejected) is block-Jacobi exactly: run it as such
        std::vector<float> prm(kLearnParams);
        if (learn_params(v.learn, prm.data(), false) != hipSuccess)
            return cg_set_error(FKT_EDEVICE, "learned preconditioner weights");
        constexpr int kOut = kLearnFeatures * kLearnHidden + kLearnHidden + kLearnHidden * kLearnHidden + kLearnHidden;
        bool zero = true;
        for (int i = kOut; i < kLearnParams; ++i) zero = zero && prm[i] == 0.0f;
        if (zero) precond = 1;
    }
    if (precond == 2 && learn_prepare_filter(v.learn) != hipSuccess)
        return cg_set_error(FKT_EDEVICE, "learned preconditioner forward pass");
    if (v.prec == 1 && io64)
        return cg_typed<float, double>(P, v, sigma2, (const double*)b, (double*)x, nrhs, rtol, maxit, precond, iters,
                                       relres, fallback_at, P64, v64, replaced);
    if (v.prec == 1)
        return cg_typed<float, float>(P, v, sigma2, (const float*)b, (float*)x, nrhs, rtol, maxit, precond, iters,
                                      relres, fallback_at, nullptr, nullptr, nullptr, region, region_bytes);
    return cg_typed<double, double>(P, v, sigma2, (const double*)b, (double*)x, nrhs, rtol, maxit, precond, iters,
                                    relres, fallback_at, nullptr, nullptr, nullptr, region, region_bytes);
}

}  // namespace fkt
