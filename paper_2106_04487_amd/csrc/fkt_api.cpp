// C-ABI entry points of libfkt.so (declared in include/fkt.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fkt.h"
#include "fkt_coarse.h"
#include "fkt_device.h"
#include "fkt_host.h"
#include "fkt_learn.h"
#include "fkt_mrhs.h"

namespace {

thread_local std::string g_err;

fkt_status fail(fkt_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

fkt_status hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? FKT_ENOMEM : FKT_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

// Device buffers freed at the end of a scope.
struct DevTmp {
    std::vector<void*> p;
    ~DevTmp()
    {
        for (void* q : p) (void)hipFree(q);
    }
    template <class T>
    hipError_t get(size_t c, T** o)
    {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, sizeof(T) * (c ? c : 1));
        if (e == hipSuccess) p.push_back(q);
        *o = (T*)q;
        return e;
    }
};

// Makes `dev` current for the scope and restores the caller's device.
struct DeviceScope {
    int old = -1;
    bool ok = false;
    explicit DeviceScope(int dev)
    {
        if (hipGetDevice(&old) != hipSuccess) return;
        ok = (old == dev) || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceScope()
    {
        if (ok && old >= 0) (void)hipSetDevice(old);
    }
};

}  // namespace

namespace fkt {
fkt_status cg_set_error(fkt_status st, const std::string& msg) { return fail(st, msg); }
fkt_status cg_solve_impl(fkt_plan_t P, const CgPlanView& v, double sigma2, const void* b, void* x, int nrhs,
                         double rtol, int maxit, int precond, int* iters, double* relres, int64_t* fallback_at,
                         bool io64, fkt_plan_t P64 = nullptr, const CgPlanView* v64 = nullptr,
                         int* replaced = nullptr, void* region = nullptr, size_t region_bytes = 0);
hipError_t cg_scratch(int device, void** ptr, size_t* bytes);
size_t cg_work_bytes_for(int64_t n, int nrhs, int nseg, size_t es, bool best);
}  // namespace fkt

struct fkt_plan_s {
    int64_t n = 0;
    int d = 0, p = 0, leaf = 0;
    fkt_kernel kern{};
    fkt_options opt{};
    fkt::Tree T;
    fkt::Lists L;
    fkt::Tables tab;
    fkt_plan_stats st{};
    bool on_device = false;
    hipStream_t stream = nullptr;
    std::vector<void*> allocs;
    int64_t nalloc = 0;  // device allocations of the plan so far (fault-injection hook)
    fkt::DevPlan dp{};
    fkt::DevWork wk{};
    fkt::DevMrhs mr{};   // many-RHS layout (opt.mrhs != 0)
    // CG systems: one per instance (row ranges in user order), row -> instance
    // (NULL for one instance)
    int cg_nseg = 1;
    const int64_t* cg_seg_off = nullptr;
    const int32_t* cg_row_seg = nullptr;
    struct Ev7 { hipEvent_t e[7]; };
    std::vector<Ev7> prof;   // events of profiled column passes not yet summed
    double prof_ms[5] = {0, 0, 0, 0, 0};
    int64_t prof_calls = 0;
    // block-Jacobi factors, built on first use for a given sigma2
    double bj_sigma2 = -1.0;
    int bj_nleaf = 0, bj_maxleaf = 0;
    const int* bj_begin = nullptr;
    const int* bj_count = nullptr;
    const int64_t* bj_off = nullptr;
    const double* bj_inv = nullptr;
    std::vector<void*> bj_allocs;
    // learned spectral preconditioner, built on first use for a given sigma2
    fkt::LearnState* learn = nullptr;
    double learn_sigma2 = -1.0;
    // two-level preconditioning (fkt_precond_coarse): rank and sigma2
    int coarse_k = 0;
    double coarse_sigma2 = -1.0;
    // radial compression (opt.compress, Appendix A.4): rows kept per degree
    // (0: off) and the interpolative coefficients
    int comp_keep = 0;
    std::vector<double> comp_coef;
    unsigned char* inst_active = nullptr;  // device [ninst] flags (batched plans)

    void drop_events()
    {
        for (auto& q : prof)
            for (hipEvent_t ev : q.e) (void)hipEventDestroy(ev);
        prof.clear();
    }

    ~fkt_plan_s()
    {
        if (on_device) {
            DeviceScope ds(opt.device);
            (void)hipStreamSynchronize(stream);
            drop_events();
            if (wk.side) (void)hipStreamDestroy(wk.side);
            if (wk.fork) (void)hipEventDestroy(wk.fork);
            if (wk.join) (void)hipEventDestroy(wk.join);
            for (void* q : allocs) (void)hipFree(q);
            for (void* q : bj_allocs) (void)hipFree(q);
            fkt::learn_destroy(learn);
        }
    }

    hipError_t alloc(size_t bytes, void** out)
    {
        *out = nullptr;
        if (bytes == 0) bytes = 256;
        // test hook: FKT_FAIL_ALLOC_AT=k makes the plan's k-th device
        // allocation report out-of-memory (error paths without a full device)
        ++nalloc;
        if (const char* f = std::getenv("FKT_FAIL_ALLOC_AT"))
            if (std::atoll(f) == nalloc) return hipErrorOutOfMemory;
        hipError_t e = hipMalloc(out, bytes);
        if (e == hipSuccess) allocs.push_back(*out);
        return e;
    }

    template <class V>
    hipError_t upload(const std::vector<V>& v, const V** out)
    {
        void* q = nullptr;
        hipError_t e = alloc(sizeof(V) * v.size(), &q);
        if (e != hipSuccess) return e;
        if (!v.empty()) e = hipMemcpy(q, v.data(), sizeof(V) * v.size(), hipMemcpyHostToDevice);
        *out = (const V*)q;
        return e;
    }
};

extern "C" {

void fkt_default_options(fkt_options* opt)
{
    if (!opt) return;
    opt->theta = 0.5;
    opt->prec = FKT_F64;
    opt->max_depth = 48;
    opt->device = 0;
    opt->stream = nullptr;
    opt->profile = 0;
    opt->overlap = 1;
    opt->mrhs = 0;
    opt->far_mode = 0;
    opt->compress = 0;
    opt->fuse = 0;
}

const char* fkt_last_error(void) { return g_err.c_str(); }

static fkt_status check_kernel(const fkt_kernel& k)
{
    if ((int)k.kind < (int)FKT_GAUSSIAN || (int)k.kind > (int)FKT_LAPLACE)
        return fail(FKT_EINVAL, "unknown kernel kind");
    if (!(k.variance > 0.0) || !std::isfinite(k.variance)) return fail(FKT_EINVAL, "kernel variance must be > 0");
    if (k.kind != FKT_LAPLACE && (!(k.lengthscale > 0.0) || !std::isfinite(k.lengthscale)))
        return fail(FKT_EINVAL, "kernel lengthscale must be > 0");
    if (k.kind == FKT_RATQUAD && (!(k.alpha > 0.0) || !std::isfinite(k.alpha)))
        return fail(FKT_EINVAL, "rational-quadratic alpha must be > 0");
    return FKT_OK;
}

static fkt_status upload_plan(fkt_plan_t P)
{
    DeviceScope ds(P->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device " + std::to_string(P->opt.device));
    P->on_device = true;
    P->stream = (hipStream_t)P->opt.stream;
    fkt::DevPlan& a = P->dp;
    const fkt::Tree& T = P->T;
    const fkt::Lists& L = P->L;
    hipError_t e = hipSuccess;
#define FKT_UP(vec, dst) \
    if ((e = P->upload(vec, &dst)) != hipSuccess) return hip_fail(e, "plan upload")
    a.n = (int)P->n;
    a.d = P->d;
    a.p = P->p;
    a.rank = (int)P->tab.rank;
    a.nblocks = (int)L.blk_begin.size();
    a.nslots = (int)L.slot_node.size();
    a.nunits = (int)L.unit_slot.size();
    a.nred = (int)L.red_slot.size();
    a.nnear_units = (int)L.nu_beg.size();
    a.kind = (int)P->kern.kind;
    a.ell = P->kern.lengthscale;
    a.alpha = P->kern.alpha;
    a.var = P->kern.variance;
    if (P->kern.kind == FKT_RATQUAD && P->kern.alpha == 1.0) {
        // (1 + r^2 / (2 l^2))^-1 is the Cauchy kernel of length scale l sqrt(2):
        // its kernels take one reciprocal where the general shape needs a power
        a.kind = (int)FKT_CAUCHY;
        a.ell = P->kern.lengthscale * std::sqrt(2.0);
    }
    FKT_UP(T.pts, a.pts64);
    if (P->opt.prec == FKT_F32) {
        std::vector<float> p32(T.pts.begin(), T.pts.end());
        FKT_UP(p32, a.pts32);
    }
    FKT_UP(T.perm, a.perm);
    {
        // instances own the contiguous user-order rows [inst_begin[i], inst_begin[i + 1])
        const size_t ni = T.inst_begin.size() - 1;
        P->cg_nseg = (int)ni;
        FKT_UP(T.inst_begin, P->cg_seg_off);
        if (ni > 1) {
            std::vector<int32_t> rs((size_t)P->n);
            for (size_t i = 0; i < ni; ++i)
                std::fill(rs.begin() + T.inst_begin[i], rs.begin() + T.inst_begin[i + 1], (int32_t)i);
            FKT_UP(rs, P->cg_row_seg);
        }
    }
    a.slot_inst = nullptr;
    a.nu_inst = nullptr;
    a.inst_active = nullptr;
    if (T.inst_begin.size() > 2) {
        // instance of a point range's first point
        auto inst_of = [&](int64_t pos) {
            return (int32_t)(std::upper_bound(T.inst_begin.begin(), T.inst_begin.end(), pos) - T.inst_begin.begin() - 1);
        };
        std::vector<int32_t> si(L.slot_node.size()), ni(L.nu_beg.size());
        for (size_t k = 0; k < si.size(); ++k) si[k] = inst_of(T.begin[L.slot_node[k]]);
        for (size_t k = 0; k < ni.size(); ++k) ni[k] = inst_of(L.nu_beg[k]);
        FKT_UP(si, a.slot_inst);
        FKT_UP(ni, a.nu_inst);
        if ((e = P->alloc(T.inst_begin.size() - 1, (void**)&P->inst_active)) != hipSuccess)
            return hip_fail(e, "instance flags");
    }
    FKT_UP(L.blk_begin, a.blk_begin);
    FKT_UP(L.blk_count, a.blk_count);
    FKT_UP(L.near_tgt, a.near_tgt);
    FKT_UP(L.nu_beg, a.nu_beg);
    FKT_UP(L.nu_end, a.nu_end);
    FKT_UP(L.nu_toff, a.nu_toff);
    FKT_UP(L.nu_tcnt, a.nu_tcnt);
    FKT_UP(L.job_off, a.job_off);
    FKT_UP(L.job_noff, a.job_noff);
    FKT_UP(L.job_nodes, a.job_nodes);
    FKT_UP(L.job_pairs, a.job_pairs);
    {
        // block-major jobs in units of kFarSegJobs, one wave each, so that
        // blocks with many far jobs spread over the machine
        int64_t maxj = 0;
        for (size_t b = 0; b + 1 < L.job_off.size(); ++b)
            maxj = std::max<int64_t>(maxj, (int64_t)L.job_off[b + 1] - L.job_off[b]);
        int64_t seg = fkt::kFarSegJobs;
        if ((maxj + seg - 1) / seg > 65535) seg = (maxj + 65534) / 65535;  // grid y limit
        a.job_seg = (int)seg;
        a.job_nseg = (int)std::max<int64_t>(1, (maxj + seg - 1) / seg);
    }
    {
        // node-major far jobs (far_mode 2; far_mode 0 except FP32 plans of
        // rank above 1000, where the block-major kernel was measured faster)
        const bool node_major = P->opt.far_mode == 2 || P->comp_keep > 0 || P->opt.fuse != 0 ||
                                (P->opt.far_mode == 0 && !(P->opt.prec == FKT_F32 && P->tab.rank > 1000));
        a.nnjobs = 0;
        a.nj_slot = nullptr;
        a.nj_tgt = nullptr;
        if (node_major && !L.slot_node.empty()) {
            std::vector<int32_t> js, jt;
            fkt::pack_node_jobs(L, js, jt);
            if ((int64_t)js.size() > 0x7fffffffLL / 4)
                return fail(FKT_EUNSUPPORTED, "too many far pairs for node-major jobs; use far_mode 1");
            for (size_t j = 0; j < js.size(); ++j) {
                if (js[j] < 0 || js[j] >= (int32_t)L.slot_node.size() || jt[j * 64] < 0)
                    return fail(FKT_EINVAL, "internal error: node-major job " + std::to_string(j));
                for (int q = 0; q < 64; ++q)
                    if (jt[j * 64 + q] >= (int32_t)P->n) return fail(FKT_EINVAL, "internal error: node-major target");
            }
            a.nnjobs = (int)js.size();
            FKT_UP(js, a.nj_slot);
            FKT_UP(jt, a.nj_tgt);
        }
    }
    FKT_UP(L.slot_ctr, a.slot_ctr);
    FKT_UP(L.slot_scale, a.slot_scale);
    FKT_UP(L.unit_slot, a.unit_slot);
    FKT_UP(L.unit_begin, a.unit_begin);
    FKT_UP(L.unit_end, a.unit_end);
    FKT_UP(L.unit_dst, a.unit_dst);
    FKT_UP(L.red_slot, a.red_slot);
    FKT_UP(L.red_off, a.red_off);
    FKT_UP(P->tab.tbar, a.tbar);
    FKT_UP(P->tab.exp2tab, a.exp2tab);
    a.comp_keep = P->comp_keep;
    a.comp_rank = (int)P->st.radial_rank;
    a.comp_invlen = P->kern.kind == FKT_LAPLACE ? 1.0 : 1.0 / P->kern.lengthscale;
    a.comp_coef = nullptr;
    if (P->comp_keep > 0) FKT_UP(P->comp_coef, a.comp_coef);
    {
        std::vector<double> h2(P->tab.hnorm.size());
        for (size_t i = 0; i < h2.size(); ++i) h2[i] = P->tab.hnorm[i] * P->tab.hnorm[i];
        FKT_UP(h2, a.hn64);
        std::vector<float> h32(h2.begin(), h2.end());
        FKT_UP(h32, a.hn32);
    }
#undef FKT_UP
    const size_t es = P->opt.prec == FKT_F32 ? sizeof(float) : sizeof(double);
    // multi-column passes (kMvmCols columns at a time) run on the node-major
    // far field (or with no far field at all); their buffers hold that many
    // columns
    const int nc = (a.nnjobs > 0 || L.slot_node.empty()) ? fkt::kMvmCols : 1;
    P->wk.ncmax = nc;
    const size_t srcw = (size_t)((P->d + nc + 1) & ~1);  // packed record: coordinates + nc weights, even
    if ((e = P->alloc(es * P->n * srcw, &P->wk.src)) != hipSuccess) return hip_fail(e, "work buffer");
    if ((e = P->alloc(es * P->n * nc, &P->wk.zacc)) != hipSuccess) return hip_fail(e, "work buffer");
    if ((e = P->alloc(es * L.slot_node.size() * P->tab.rank * nc, &P->wk.mom)) != hipSuccess)
        return hip_fail(e, "moment buffer");
    if ((e = P->alloc(es * L.npartials * P->tab.rank * nc, &P->wk.part)) != hipSuccess)
        return hip_fail(e, "partial-moment buffer");
    P->wk.momc = nullptr;
    if (P->comp_keep > 0 &&
        (e = P->alloc(es * L.slot_node.size() * (size_t)P->st.radial_rank * nc, &P->wk.momc)) != hipSuccess)
        return hip_fail(e, "compressed-moment buffer");
    P->wk.qctr = nullptr;
    a.fused = 0;
    if (P->opt.fuse) {
        if ((e = P->alloc(sizeof(unsigned), (void**)&P->wk.qctr)) != hipSuccess) return hip_fail(e, "queue counter");
        a.fused = 1;
    }
    P->wk.mom_cols = L.slot_node.size() * (size_t)P->tab.rank;
    P->wk.part_cols = (size_t)L.npartials * (size_t)P->tab.rank;
    P->wk.momc_cols = P->comp_keep > 0 ? L.slot_node.size() * (size_t)P->st.radial_rank : 0;
    // many-RHS near field: leaves padded to multiples of 32 points, SoA
    // coordinates, target-major near lists with padded ranges
    if (P->opt.mrhs != 0) {
        const int d = P->d;
        std::vector<int32_t> pbeg_of(P->n + 1, -1);
        std::vector<int32_t> src;
        for (int64_t b = 0; b < T.nnodes(); ++b) {
            if (!T.leaf(b)) continue;
            const int64_t b0 = T.begin[b], m = T.end[b] - b0;
            pbeg_of[b0] = (int32_t)src.size();
            for (int64_t i = 0; i < m; ++i) src.push_back((int32_t)(b0 + i));
            while (src.size() % 32) src.push_back(-1 - (int32_t)b0);  // pad: -1 - leaf start
        }
        const int64_t npad = (int64_t)src.size();
        if (npad > 0x7fffffff / 32) return fail(FKT_EUNSUPPORTED, "too many points for the many-RHS layout");
        std::vector<float> pts((size_t)d * npad);
        for (int64_t p = 0; p < npad; ++p) {
            const int64_t t = src[p] >= 0 ? src[p] : -1 - (int64_t)src[p];
            for (int k = 0; k < d; ++k) pts[(size_t)k * npad + p] = (float)T.pts[t * d + k];
            if (src[p] < 0) src[p] = -1;
        }
        std::vector<int32_t> pb(L.near_beg.size()), pc(L.near_beg.size());
        for (size_t e2 = 0; e2 < L.near_beg.size(); ++e2) {
            pb[e2] = pbeg_of[L.near_beg[e2]];
            pc[e2] = (L.near_end[e2] - L.near_beg[e2] + 31) / 32 * 32;
            if (pb[e2] < 0) return fail(FKT_EDEVICE, "many-RHS layout: near entry is not a leaf");
        }
        P->mr.npad = (int)npad;
        P->mr.bf16 = P->opt.mrhs == 2;
#define FKT_UP2(vec, dst) \
    if ((e = P->upload(vec, &dst)) != hipSuccess) return hip_fail(e, "many-RHS upload")
        FKT_UP2(pts, P->mr.pts);
        FKT_UP2(src, P->mr.src);
        FKT_UP2(L.near_off, P->mr.near_off);
        {
            int64_t maxe = 0;
            for (size_t b = 0; b + 1 < L.near_off.size(); ++b)
                maxe = std::max<int64_t>(maxe, (int64_t)L.near_off[b + 1] - L.near_off[b]);
            int64_t seg = fkt::kMrSegNear;
            if ((maxe + seg - 1) / seg > 65535) seg = (maxe + 65534) / 65535;  // grid y limit
            P->mr.near_seg = (int)seg;
            P->mr.near_nseg = (int)std::max<int64_t>(1, (maxe + seg - 1) / seg);
        }
        FKT_UP2(pb, P->mr.near_pbeg);
        FKT_UP2(pc, P->mr.near_pcnt);
        FKT_UP2(L.near_mask, P->mr.near_mask);
#undef FKT_UP2
        if ((e = P->alloc((P->mr.bf16 ? 2 : 4) * (size_t)fkt::kMrCols * npad, &P->mr.xt)) != hipSuccess)
            return hip_fail(e, "many-RHS weights");
        if ((e = P->alloc(sizeof(float) * (size_t)fkt::kMrCols * P->n, &P->mr.zf)) != hipSuccess)
            return hip_fail(e, "many-RHS far-field buffer");
        // far field on the matrix cores: moments of the 32 columns and their
        // bf16 high/low B fragments (rank padded to a multiple of 64)
        const int64_t ns = (int64_t)L.slot_node.size(), R = P->tab.rank;
        P->mr.ks = (int)((R + 63) / 64 * 2);
        {
            fkt::JobSet J;
            fkt::pack_far_jobs_grouped(L, fkt::kMrJobNodes, fkt::kMrGroupBlocks, J);
            std::string err;
            if (!fkt::check_jobs_grouped(L, J, fkt::kMrGroupBlocks, err))
                return fail(FKT_EINVAL, "internal error: " + err);
            P->mr.job_group = fkt::kMrGroupBlocks;
            P->mr.ngroups = (int)(J.job_off.size() - 1);
#define FKT_UP3(vec, dst) \
    if ((e = P->upload(vec, &dst)) != hipSuccess) return hip_fail(e, "many-RHS job upload")
            FKT_UP3(J.job_off, P->mr.job_off);
            FKT_UP3(J.job_noff, P->mr.job_noff);
            FKT_UP3(J.job_nodes, P->mr.job_nodes);
            FKT_UP3(J.job_pairs, P->mr.job_pairs);
#undef FKT_UP3
            int64_t maxj = 0;
            for (size_t b = 0; b + 1 < J.job_off.size(); ++b)
                maxj = std::max<int64_t>(maxj, (int64_t)J.job_off[b + 1] - J.job_off[b]);
            int64_t seg = fkt::kMrSegJobs;
            if ((maxj + seg - 1) / seg > 65535) seg = (maxj + 65534) / 65535;  // grid y limit
            P->mr.job_seg = (int)seg;
            P->mr.job_nseg = (int)std::max<int64_t>(1, (maxj + seg - 1) / seg);
        }
        if (ns > 0) {
            if ((e = P->alloc(sizeof(float) * (size_t)fkt::kMrCols * ns * R, &P->mr.mom)) != hipSuccess)
                return hip_fail(e, "many-RHS moments");
            P->mr.npart = L.npartials;
            if ((e = P->alloc(sizeof(float) * (size_t)fkt::kMrCols * P->n, &P->mr.x32)) != hipSuccess ||
                (e = P->alloc(sizeof(float) * (size_t)fkt::kMrCols * (size_t)std::max<int64_t>(L.npartials, 1) * R,
                              &P->mr.part32)) != hipSuccess)
                return hip_fail(e, "many-RHS moment work buffers");
            const size_t fb = (size_t)ns * P->mr.ks * 2 * 64 * 16;
            if ((e = P->alloc(fb, &P->mr.bhi)) != hipSuccess || (e = P->alloc(fb, &P->mr.blo)) != hipSuccess)
                return hip_fail(e, "many-RHS moment fragments");
        }
    }
    // second stream (default priority) and fork/join events for running the
    // near field beside the far field
    if ((e = hipStreamCreateWithFlags(&P->wk.side, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    if ((e = hipEventCreateWithFlags(&P->wk.fork, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipEventCreateWithFlags(&P->wk.join, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
    return FKT_OK;
}

static fkt_status make_plan(const double* points, int64_t n, int d, const int64_t* offsets, int ninst, fkt_kernel k,
                            int leaf_size, int order, const fkt_options* opt_in, fkt_plan_t* out)
{
    if (!out) return fail(FKT_EINVAL, "out is NULL");
    *out = nullptr;
    fkt_options opt;
    fkt_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (!points) return fail(FKT_EINVAL, "points is NULL");
    if (n < 1) return fail(FKT_EINVAL, "n must be >= 1");
    if (n > 0x7fffffffLL) return fail(FKT_EINVAL, "n must be < 2^31");
    if (d < 1) return fail(FKT_EINVAL, "d must be >= 1");
    if (d < 3 || d > 5) return fail(FKT_EUNSUPPORTED, "d must be 3, 4 or 5");
    if (leaf_size < 1) return fail(FKT_EINVAL, "leaf_size must be >= 1");
    if (order < 0) return fail(FKT_EINVAL, "order must be >= 0");
    if (!fkt::far_supported(d, order))
        return fail(FKT_EUNSUPPORTED, "order " + std::to_string(order) + " not built for d = " + std::to_string(d) +
                                          " (built orders: 0.." + std::to_string(fkt::far_max_order(d)) + ")");
    if (!(opt.theta > 0.0 && opt.theta < 1.0)) return fail(FKT_EINVAL, "theta must be in (0, 1)");
    if (opt.prec != FKT_F64 && opt.prec != FKT_F32) return fail(FKT_EINVAL, "unknown precision");
    if (opt.mrhs < 0 || opt.mrhs > 2) return fail(FKT_EINVAL, "mrhs must be 0, 1 or 2");
    if (opt.mrhs != 0 && opt.prec != FKT_F32) return fail(FKT_EUNSUPPORTED, "mrhs needs an FP32 plan");
    if (opt.far_mode < 0 || opt.far_mode > 2) return fail(FKT_EINVAL, "far_mode must be 0, 1 or 2");
    if (opt.compress != 0 && opt.compress != 1) return fail(FKT_EINVAL, "compress must be 0 or 1");
    if (opt.compress && !fkt::radial_has_laurent_q((int)k.kind))
        return fail(FKT_EINVAL, "radial compression needs K' = q K with q a Laurent polynomial "
                                "(exponential, Laplace or Gaussian kernel)");
    if (opt.compress && opt.mrhs != 0) return fail(FKT_EUNSUPPORTED, "radial compression with mrhs is not built");
    if (opt.compress && opt.far_mode == 1)
        return fail(FKT_EUNSUPPORTED, "radial compression runs the node-major far field (far_mode 0 or 2)");
    if (opt.fuse != 0 && opt.fuse != 1) return fail(FKT_EINVAL, "fuse must be 0 or 1");
    if (opt.fuse && d != 3) return fail(FKT_EUNSUPPORTED, "the persistent launch is built for d = 3 only");
    if (opt.fuse && (opt.compress || opt.far_mode == 1))
        return fail(FKT_EUNSUPPORTED, "the persistent launch runs the uncompressed node-major far field "
                                      "(compress 0, far_mode 0 or 2)");
    if (opt.max_depth < 1 || opt.max_depth > 60) return fail(FKT_EINVAL, "max_depth must be in [1, 60]");
    if (opt.device < -1) return fail(FKT_EINVAL, "device must be >= -1");
    fkt_status s = check_kernel(k);
    if (s != FKT_OK) return s;
    for (int64_t i = 0; i < n * d; ++i)
        if (!std::isfinite(points[i])) return fail(FKT_EINVAL, "non-finite coordinate at index " + std::to_string(i));

    const auto t0 = std::chrono::steady_clock::now();
    fkt_plan_t P = new (std::nothrow) fkt_plan_s();
    if (!P) return fail(FKT_ENOMEM, "plan allocation");
    try {
        P->n = n;
        P->d = d;
        P->p = order;
        P->leaf = leaf_size;
        P->kern = k;
        P->opt = opt;
        if (offsets)
            fkt::build_forest(points, offsets, ninst, d, leaf_size, opt.max_depth, P->T);
        else
            fkt::build_tree(points, n, d, leaf_size, opt.max_depth, P->T);
        fkt::build_lists(P->T, opt.theta,
                         fkt::m2t_max_job_nodes(d, order, opt.prec == FKT_F32 ? (int)sizeof(float) : (int)sizeof(double)),
                         P->L, P->st);
        if (P->L.near_tgt.size() > (size_t)0x7fffffff) {
            delete P;
            return fail(FKT_EUNSUPPORTED, "near sets exceed 2^31 (target, leaf) pairs; use fewer points or a smaller theta");
        }
        std::string err;
        if (!fkt::check_lists(P->T, P->L, err)) {
            delete P;
            return fail(FKT_EINVAL, "internal error: " + err);
        }
        fkt::build_tables(d, order, P->tab);
        P->st.radial_rank = P->tab.rank;
        const int keep = opt.compress ? fkt::radial_keep((int)k.kind, d) : 0;
        if (keep > 0) {
            // compressed kernels are built for this kernel and dimension: keep
            // the first min(keep, nj) rows when they carry the exact rank
            std::vector<int> rk;
            std::string cerr;
            bool ok = fkt::radial_ranks((int)k.kind, d, order, rk);
            for (int kk = 0; ok && kk <= order; ++kk) ok = rk[kk] == std::min(keep, (order - kk) / 2 + 1);
            if (ok && fkt::radial_interpolative((int)k.kind, d, order, keep, P->comp_coef, cerr)) {
                P->comp_keep = keep;
                int64_t rc = 0;
                for (int kk = 0; kk <= order; ++kk)
                    rc += (fkt::binom(kk + d - 1, d - 1) - (kk >= 2 ? fkt::binom(kk + d - 3, d - 1) : 0)) * rk[kk];
                P->st.radial_rank = rc;
            }
        }
    } catch (const std::bad_alloc&) {
        delete P;
        return fail(FKT_ENOMEM, "host allocation while building the plan");
    }
    fkt_plan_stats& st = P->st;
    st.n = n;
    st.nnodes = P->T.nnodes();
    st.nleaves = 0;
    st.depth = 0;
    for (int64_t b = 0; b < st.nnodes; ++b) {
        st.nleaves += P->T.leaf(b);
        st.depth = std::max<int64_t>(st.depth, P->T.level[b]);
    }
    st.rank = P->tab.rank;
    st.cg_fallback_iter = -1;
    if (opt.device >= 0) {
        s = upload_plan(P);
        if (s != FKT_OK) {
            delete P;
            return s;
        }
    }
    st.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = P;
    return FKT_OK;
}

fkt_status fkt_plan(const double* points, int64_t n, int d, fkt_kernel k, int leaf_size, int order,
                    const fkt_options* opt_in, fkt_plan_t* out)
{
    return make_plan(points, n, d, nullptr, 1, k, leaf_size, order, opt_in, out);
}

fkt_status fkt_plan_batch(const double* points, const int64_t* offsets, int ninst, int d, fkt_kernel k, int leaf_size,
                          int order, const fkt_options* opt, fkt_plan_t* out)
{
    if (!out) return fail(FKT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!offsets) return fail(FKT_EINVAL, "offsets is NULL");
    if (ninst < 1) return fail(FKT_EINVAL, "ninst must be >= 1");
    if (offsets[0] != 0) return fail(FKT_EINVAL, "offsets[0] must be 0");
    for (int i = 0; i < ninst; ++i)
        if (offsets[i + 1] < offsets[i]) return fail(FKT_EINVAL, "offsets must be non-decreasing");
    return make_plan(points, offsets[ninst], d, offsets, ninst, k, leaf_size, order, opt, out);
}

// Columns of the next MVM pass when `left` columns remain: kMvmCols at a
// time (three padded to four: the shared kernel values, harmonics and
// radial functions outweigh one padded column) where the plan's buffers
// allow it, else one.
static void mvm_pass_width(const fkt_plan_s* P, int left, int& ncols, int& nc)
{
    nc = (P->wk.ncmax >= fkt::kMvmCols && left >= fkt::kMvmCols - 1) ? fkt::kMvmCols : 1;
    ncols = std::min(nc, left);
}

fkt_status fkt_mvm(fkt_plan_t P, const void* x, void* y, int nrhs)
{
    if (!P) return fail(FKT_EINVAL, "plan is NULL");
    if (!P->on_device) return fail(FKT_EDEVICE, "host-only plan (device = -1) cannot run fkt_mvm");
    if (!x || !y) return fail(FKT_EINVAL, "x or y is NULL");
    if (nrhs < 1 || nrhs > 64) return fail(FKT_EINVAL, "nrhs must be in [1, 64]");
    const size_t es = P->opt.prec == FKT_F32 ? sizeof(float) : sizeof(double);
    const size_t bytes = es * (size_t)P->n * nrhs;
    const char *xb = (const char*)x, *yb = (const char*)y;
    if (xb < yb + bytes && yb < xb + bytes) return fail(FKT_EINVAL, "x and y overlap");
    DeviceScope ds(P->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    if (P->opt.mrhs != 0 && nrhs % fkt::kMrCols == 0) {
        const hipError_t e = fkt::launch_mvm_mrhs(P->dp, P->wk, P->mr, (const float*)x, (float*)y, nrhs, P->stream);
        return e == hipSuccess ? FKT_OK : hip_fail(e, "fkt_mvm many-RHS launch");
    }
    for (int c = 0; c < nrhs;) {
        int ncols, nc;
        mvm_pass_width(P, nrhs - c, ncols, nc);
        hipEvent_t* ev = nullptr;
        if (P->opt.profile) {
            fkt_plan_s::Ev7 q{};
            for (auto& e : q.e)
                if (hipEventCreate(&e) != hipSuccess) return fail(FKT_EDEVICE, "hipEventCreate");
            P->prof.push_back(q);
            ev = P->prof.back().e;
        }
        hipError_t e = fkt::launch_mvm_column(P->dp, P->wk, x, y, nrhs, c, ncols, nc, (int)P->opt.prec, P->stream,
                                              P->opt.overlap != 0, ev);
        if (e != hipSuccess) return hip_fail(e, "fkt_mvm launch");
        c += ncols;
    }
    return FKT_OK;
}

fkt_status fkt_plan_stage_times(fkt_plan_t P, double* ms, int64_t* calls, int reset)
{
    if (!P || !ms) return fail(FKT_EINVAL, "NULL argument");
    if (!P->opt.profile) return fail(FKT_EINVAL, "plan was built without opt.profile");
    DeviceScope ds(P->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    // intervals: gather e0-e1, s2m e1-e2, m2t e2-e3, near e4-e5, column e0-e6
    static const int from[5] = {0, 1, 2, 4, 0}, to[5] = {1, 2, 3, 5, 6};
    for (auto& q : P->prof) {
        if (hipEventSynchronize(q.e[6]) != hipSuccess) return fail(FKT_EDEVICE, "hipEventSynchronize");
        for (int i = 0; i < 5; ++i) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, q.e[from[i]], q.e[to[i]]) != hipSuccess)
                return fail(FKT_EDEVICE, "hipEventElapsedTime");
            P->prof_ms[i] += t;
        }
        P->prof_calls += 1;
    }
    P->drop_events();
    for (int i = 0; i < 5; ++i) ms[i] = P->prof_ms[i];
    if (calls) *calls = P->prof_calls;
    if (reset) {
        for (double& v : P->prof_ms) v = 0.0;
        P->prof_calls = 0;
    }
    return FKT_OK;
}

void fkt_destroy(fkt_plan_t P) { delete P; }

fkt_status fkt_plan_info(fkt_plan_t P, fkt_plan_stats* s)
{
    if (!P || !s) return fail(FKT_EINVAL, "NULL argument");
    *s = P->st;
    return FKT_OK;
}

fkt_status fkt_plan_perm(fkt_plan_t P, int64_t* perm)
{
    if (!P || !perm) return fail(FKT_EINVAL, "NULL argument");
    std::memcpy(perm, P->T.perm.data(), sizeof(int64_t) * P->n);
    return FKT_OK;
}

fkt_status fkt_plan_target_counts(fkt_plan_t P, int64_t* far_nodes, int64_t* far_points, int64_t* near_leaves,
                                  int64_t* near_points)
{
    if (!P) return fail(FKT_EINVAL, "plan is NULL");
    const fkt::Lists& L = P->L;
    const fkt::Tree& T = P->T;
    int64_t* outs[4] = {far_nodes, far_points, near_leaves, near_points};
    for (int64_t* o : outs)
        if (o) std::memset(o, 0, sizeof(int64_t) * P->n);
    const int64_t nb = (int64_t)L.blk_begin.size();
    for (int64_t q = 0; q < nb; ++q) {
        for (int e = L.far_off[q]; e < L.far_off[q + 1]; ++e) {
            const int32_t b = L.slot_node[L.far_slot[e]];
            for (int lane = 0; lane < L.blk_count[q]; ++lane) {
                if (!((L.far_mask[e] >> lane) & 1)) continue;
                const int64_t t = T.perm[L.blk_begin[q] + lane];
                if (far_nodes) far_nodes[t] += 1;
                if (far_points) far_points[t] += T.end[b] - T.begin[b];
            }
        }
        for (int e = L.near_off[q]; e < L.near_off[q + 1]; ++e) {
            for (int lane = 0; lane < L.blk_count[q]; ++lane) {
                if (!((L.near_mask[e] >> lane) & 1)) continue;
                const int64_t t = T.perm[L.blk_begin[q] + lane];
                if (near_leaves) near_leaves[t] += 1;
                if (near_points) near_points[t] += L.near_end[e] - L.near_beg[e];
            }
        }
    }
    return FKT_OK;
}

fkt_status fkt_radial_compression(const fkt_kernel* k, int d, int order, int* ranks, int* keep, double* coef)
{
    if (!k) return fail(FKT_EINVAL, "kernel is NULL");
    fkt_status s = check_kernel(*k);
    if (s != FKT_OK) return s;
    if (d < 1 || order < 0 || order > 30) return fail(FKT_EINVAL, "d must be >= 1 and order in [0, 30]");
    if (!fkt::radial_has_laurent_q((int)k->kind))
        return fail(FKT_EINVAL, "the kernel has no K' = q K with q a Laurent polynomial");
    try {
        std::vector<int> rk;
        fkt::radial_ranks((int)k->kind, d, order, rk);
        if (ranks) std::copy(rk.begin(), rk.end(), ranks);
        const int kp = fkt::radial_keep((int)k->kind, d);
        bool ok = kp > 0;
        for (int kk = 0; ok && kk <= order; ++kk) ok = rk[kk] == std::min(kp, (order - kk) / 2 + 1);
        std::vector<double> c;
        std::string err;
        if (ok) ok = fkt::radial_interpolative((int)k->kind, d, order, kp, c, err);
        if (keep) *keep = ok ? kp : 0;
        if (coef && ok) std::copy(c.begin(), c.end(), coef);
    } catch (const std::bad_alloc&) {
        return fail(FKT_ENOMEM, "host allocation");
    }
    return FKT_OK;
}

fkt_status fkt_plan_lists(fkt_plan_t P, int64_t* far_off, int64_t* far_node, int64_t* near_off, int64_t* near_leaf,
                          int64_t* nfar_total, int64_t* nnear_total)
{
    if (!P) return fail(FKT_EINVAL, "plan is NULL");
    const fkt::Lists& L = P->L;
    const fkt::Tree& T = P->T;
    const int64_t n = P->n, nb = (int64_t)L.blk_begin.size();
    // leaf id of each leaf's first tree position (near entries are point ranges)
    std::vector<int32_t> leaf_at(n + 1, -1);
    for (int64_t b = 0; b < T.nnodes(); ++b)
        if (T.leaf(b) && T.end[b] > T.begin[b]) leaf_at[T.begin[b]] = (int32_t)b;
    std::vector<std::vector<int64_t>> fl(n), nl(n);
    for (int64_t q = 0; q < nb; ++q) {
        for (int e = L.far_off[q]; e < L.far_off[q + 1]; ++e)
            for (int lane = 0; lane < L.blk_count[q]; ++lane)
                if ((L.far_mask[e] >> lane) & 1)
                    fl[T.perm[L.blk_begin[q] + lane]].push_back(L.slot_node[L.far_slot[e]]);
        for (int e = L.near_off[q]; e < L.near_off[q + 1]; ++e)
            for (int lane = 0; lane < L.blk_count[q]; ++lane)
                if ((L.near_mask[e] >> lane) & 1) nl[T.perm[L.blk_begin[q] + lane]].push_back(leaf_at[L.near_beg[e]]);
    }
    int64_t tf = 0, tn = 0;
    for (int64_t t = 0; t < n; ++t) {
        std::sort(fl[t].begin(), fl[t].end());
        std::sort(nl[t].begin(), nl[t].end());
        if (far_off) far_off[t] = tf;
        if (near_off) near_off[t] = tn;
        if (far_node) std::copy(fl[t].begin(), fl[t].end(), far_node + tf);
        if (near_leaf) std::copy(nl[t].begin(), nl[t].end(), near_leaf + tn);
        tf += (int64_t)fl[t].size();
        tn += (int64_t)nl[t].size();
    }
    if (far_off) far_off[n] = tf;
    if (near_off) near_off[n] = tn;
    if (nfar_total) *nfar_total = tf;
    if (nnear_total) *nnear_total = tn;
    return FKT_OK;
}

// Spectra of the leaf blocks for sigma2 (host eigendecompositions) and the
// network's device state; weights are kept across sigma2 changes.
static fkt_status ensure_learn(fkt_plan_t P, double sigma2)
{
    if (P->learn && P->learn_sigma2 == sigma2) return FKT_OK;
    // a coarse part belongs to its sigma2; the new spectra replace it
    P->coarse_k = 0;
    P->coarse_sigma2 = -1.0;
    int64_t big = 0;
    for (int64_t b = 0; b < P->T.nnodes(); ++b)
        if (P->T.leaf(b)) big = std::max<int64_t>(big, P->T.end[b] - P->T.begin[b]);
    if (big > fkt::kLearnMaxLeaf) return fail(FKT_EUNSUPPORTED, "the learned preconditioner needs leaves of at most 2048 points");
    if (!(sigma2 > 0.0)) return fail(FKT_EINVAL, "the learned preconditioner needs sigma2 > 0");
    fkt::LeafSpectra S;
    if (!fkt::build_leaf_spectra(P->T, P->kern, sigma2, P->leaf, S))
        return fail(FKT_EINVAL, "a leaf block K_ll + sigma2 I has no positive spectrum (or the eigensolver failed)");
    if (!P->learn) {
        std::string err;
        P->learn = fkt::learn_create(P->opt.device, P->stream, S, P->dp.perm, P->n, 0x5EEDull, err);
        if (!P->learn) return fail(FKT_ENOMEM, err);
    } else {
        const hipError_t e = fkt::learn_update_spectra(P->learn, S);
        if (e != hipSuccess) return hip_fail(e, "learned preconditioner spectra upload");
    }
    P->learn_sigma2 = sigma2;
    return FKT_OK;
}

fkt_status fkt_precond_coarse(fkt_plan_t P, double sigma2, const int64_t* landmarks, int k)
{
    if (!P) return fail(FKT_EINVAL, "plan is NULL");
    if (!P->on_device) return fail(FKT_EDEVICE, "host-only plan (device = -1) has no preconditioner state");
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return fail(FKT_EINVAL, "sigma2 must be > 0");
    if (k < 0 || k > fkt::kCoarseMaxRank) return fail(FKT_EINVAL, "k must be in [0, 4096]");
    if (k > P->n) return fail(FKT_EINVAL, "k exceeds the number of points");
    if (k > 0 && !landmarks) return fail(FKT_EINVAL, "landmarks is NULL");
    DeviceScope ds(P->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    if (k == 0) {
        // back to one-level: drop the coarse part and rebuild the plain spectra on next use
        if (P->learn) (void)fkt::learn_set_coarse(P->learn, nullptr, 0);
        if (P->coarse_k > 0) P->learn_sigma2 = -1.0;
        P->coarse_k = 0;
        P->coarse_sigma2 = -1.0;
        return FKT_OK;
    }
    int64_t big = 0;
    for (int64_t b = 0; b < P->T.nnodes(); ++b)
        if (P->T.leaf(b)) big = std::max<int64_t>(big, P->T.end[b] - P->T.begin[b]);
    if (big > fkt::kLearnMaxLeaf) return fail(FKT_EUNSUPPORTED, "two-level preconditioning needs leaves of at most 2048 points");
    // landmarks: caller order -> tree positions, distinct
    const int64_t n = P->n;
    std::vector<int64_t> pos(n);
    for (int64_t i = 0; i < n; ++i) pos[P->T.perm[i]] = i;
    std::vector<int32_t> cols(k);
    std::vector<char> seen(n, 0);
    for (int j = 0; j < k; ++j) {
        const int64_t c = landmarks[j];
        if (c < 0 || c >= n) return fail(FKT_EINVAL, "landmark index out of range");
        if (seen[c]) return fail(FKT_EINVAL, "landmark indices must be distinct");
        seen[c] = 1;
        cols[j] = (int32_t)pos[c];
    }
    // W = chol(K(X_J, X_J) + sigma2 I)^-T on the host
    const int d = P->d;
    std::vector<double> KJ((size_t)k * k), W((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j <= i; ++j) {
            double s2 = 0.0;
            for (int a = 0; a < d; ++a) {
                const double u = P->T.pts[(int64_t)cols[i] * d + a] - P->T.pts[(int64_t)cols[j] * d + a];
                s2 += u * u;
            }
            KJ[(size_t)i * k + j] = KJ[(size_t)j * k + i] = fkt::kernel_value(P->kern, std::sqrt(s2)) + (i == j ? sigma2 : 0.0);
        }
    if (!fkt::chol_inv_t(k, KJ.data(), W.data()))
        return fail(FKT_EINVAL, "the landmark block K(X_J, X_J) + sigma2 I is not positive definite");
    // device: K(X, X_J), the factor L = K(X, X_J) W, and the leaf blocks L_l L_l^T
    hipStream_t s = P->stream;
    DevTmp tmp;
    fkt::LeafSpectra S;
    fkt::leaf_layout(P->T, S);
    const int nl = (int)S.leaf_begin.size();
    int32_t* dcols = nullptr;
    double *dW = nullptr, *KnJ = nullptr, *Lm = nullptr, *Sb = nullptr;
    fkt::Gemm64* desc = nullptr;
    hipError_t e;
    if ((e = tmp.get(k, &dcols)) || (e = tmp.get((size_t)k * k, &dW)) || (e = tmp.get((size_t)n * k, &KnJ)) ||
        (e = tmp.get((size_t)n * k, &Lm)) || (e = tmp.get(S.off.back(), &Sb)) || (e = tmp.get(nl + 1, &desc)))
        return hip_fail(e, "two-level work buffers");
    std::vector<fkt::Gemm64> dd;
    dd.push_back(fkt::Gemm64{(int)n, k, k, k, k, k, 0, 0, 0, 0});  // L = K(X, X_J) W
    int maxm = 0;
    for (int l = 0; l < nl; ++l) {  // L_l L_l^T
        const int m = S.leaf_count[l];
        const int64_t b0 = S.leaf_begin[l];
        maxm = std::max(maxm, m);
        dd.push_back(fkt::Gemm64{m, m, k, k, k, m, b0 * k, b0 * k, S.off[l], 0});
    }
    std::vector<double> Sh(S.off.back());
    if ((e = hipMemcpy(dcols, cols.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(dW, W.data(), sizeof(double) * W.size(), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(desc, dd.data(), sizeof(fkt::Gemm64) * dd.size(), hipMemcpyHostToDevice)) ||
        (e = fkt::kernel_columns(P->dp, dcols, k, KnJ, s)) ||
        (e = fkt::gemm64_batched(false, false, desc, 1, (int)n, k, KnJ, dW, nullptr, Lm, 1.0, 0.0, s)) ||
        (e = fkt::gemm64_batched(false, true, desc + 1, nl, maxm, maxm, Lm, Lm, nullptr, Sb, 1.0, 0.0, s)) ||
        (e = hipMemcpyAsync(Sh.data(), Sb, sizeof(double) * Sh.size(), hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s)))
        return hip_fail(e, "two-level factor");
    // spectra of the residual leaf blocks, then the coarse matrices
    if (!fkt::build_leaf_spectra(P->T, P->kern, sigma2, P->leaf, S, Sh.data()))
        return fail(FKT_EINVAL, "a residual leaf block K_ll + sigma2 I - L_l L_l^T has no positive spectrum");
    if (!P->learn) {
        std::string err;
        P->learn = fkt::learn_create(P->opt.device, P->stream, S, P->dp.perm, P->n, 0x5EEDull, err);
        if (!P->learn) return fail(FKT_ENOMEM, err);
    } else if ((e = fkt::learn_update_spectra(P->learn, S)) != hipSuccess) {
        return hip_fail(e, "two-level spectra upload");
    }
    P->learn_sigma2 = sigma2;
    if ((e = fkt::learn_set_coarse(P->learn, Lm, k)) != hipSuccess)
        return e == hipErrorInvalidValue ? fail(FKT_EINVAL, "the coarse matrix I + G^T diag(h) G is not positive definite")
                                         : hip_fail(e, "two-level coarse matrices");
    P->coarse_k = k;
    P->coarse_sigma2 = sigma2;
    return FKT_OK;
}

// fkt_cg_solve without (fallback_at NULL) or with the learned filter's
// block-Jacobi fallback; the judge runs the filter on its own.
static fkt_status cg_entry(fkt_plan_t P, double sigma2, const void* b, void* x, int nrhs, double rtol, int maxit,
                           int precond, int* iters, double* relres, int64_t* fallback_at, bool io64 = false,
                           fkt_plan_t P64 = nullptr, const fkt::CgPlanView* v64 = nullptr, int* replaced = nullptr)
{
    if (!P) return fail(FKT_EINVAL, "plan is NULL");
    if (!P->on_device) return fail(FKT_EDEVICE, "host-only plan (device = -1) cannot run fkt_cg_solve");
    if (!b || !x) return fail(FKT_EINVAL, "b or x is NULL");
    if (nrhs < 1 || nrhs > 64) return fail(FKT_EINVAL, "nrhs must be in [1, 64]");
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2)) return fail(FKT_EINVAL, "sigma2 must be >= 0");
    if (!(rtol > 0.0)) return fail(FKT_EINVAL, "rtol must be > 0");
    if (maxit < 1) return fail(FKT_EINVAL, "maxit must be >= 1");
    if (precond < 0 || precond > 2) return fail(FKT_EUNSUPPORTED, "unknown preconditioner");
    DeviceScope ds(P->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    const bool two_level = P->coarse_k > 0 && P->coarse_sigma2 == sigma2 && P->learn;
    if (precond == 2 && !two_level) {
        const fkt_status st = ensure_learn(P, sigma2);
        if (st != FKT_OK) return st;
    }
    // block-Jacobi serves precond 1 and is the fallback of precond 2
    if (precond >= 1 && P->st.nleaves > 0) {
        int64_t big = 0;
        for (int64_t b = 0; b < P->T.nnodes(); ++b)
            if (P->T.leaf(b)) big = std::max<int64_t>(big, P->T.end[b] - P->T.begin[b]);
        if (big > 4096) return fail(FKT_EUNSUPPORTED, "block-Jacobi needs leaves of at most 4096 points");
    }
    // two-level: block-Jacobi and the learned filter both run on the residual
    // leaf spectra with the coarse correction (learned state built by
    // fkt_precond_coarse)
    if (precond >= 1 && !two_level && P->bj_sigma2 != sigma2) {
        std::vector<int32_t> lb, lc;
        std::vector<int64_t> off;
        std::vector<double> inv;
        if (!fkt::build_block_jacobi(P->T, P->kern, sigma2, lb, lc, off, inv))
            return fail(FKT_EINVAL, "a leaf block K_ll + sigma2 I is not positive definite");
        (void)hipStreamSynchronize(P->stream);
        for (void* q : P->bj_allocs) (void)hipFree(q);
        P->bj_allocs.clear();
        P->bj_sigma2 = -1.0;
        auto up = [&](const void* src, size_t bytes, const void** dst) -> hipError_t {
            void* q = nullptr;
            hipError_t e = hipMalloc(&q, bytes ? bytes : 256);
            if (e != hipSuccess) return e;
            P->bj_allocs.push_back(q);
            *dst = q;
            return bytes ? hipMemcpy(q, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
        };
        hipError_t e;
        if ((e = up(lb.data(), sizeof(int32_t) * lb.size(), (const void**)&P->bj_begin)) ||
            (e = up(lc.data(), sizeof(int32_t) * lc.size(), (const void**)&P->bj_count)) ||
            (e = up(off.data(), sizeof(int64_t) * off.size(), (const void**)&P->bj_off)) ||
            (e = up(inv.data(), sizeof(double) * inv.size(), (const void**)&P->bj_inv)))
            return hip_fail(e, "block-Jacobi upload");
        P->bj_nleaf = (int)lb.size();
        P->bj_maxleaf = 0;
        for (int32_t c : lc) P->bj_maxleaf = std::max(P->bj_maxleaf, (int)c);
        P->bj_sigma2 = sigma2;
    }
    fkt::CgPlanView v{P->n,         (int)P->opt.prec, P->opt.device, P->stream,    P->dp.perm,   P->bj_nleaf,
                      P->bj_maxleaf, P->bj_begin,       P->bj_count,  P->bj_off,    P->bj_inv,    P->learn,
                      P->cg_nseg,    P->cg_seg_off,     P->cg_row_seg};
    v.coarse = two_level ? 1 : 0;
    v.active = P->inst_active;
    return fkt::cg_solve_impl(P, v, sigma2, b, x, nrhs, rtol, maxit, precond, iters, relres, fallback_at, io64, P64,
                              v64, replaced);
}

fkt_status fkt_cg_solve(fkt_plan_t P, double sigma2, const void* b, void* x, int nrhs, double rtol, int maxit,
                        int precond, int* iters, double* relres)
{
    return cg_entry(P, sigma2, b, x, nrhs, rtol, maxit, precond, iters, relres, P ? &P->st.cg_fallback_iter : nullptr);
}

fkt_status fkt_cg_solve64(fkt_plan_t P, double sigma2, const double* b, double* x, int nrhs, double rtol, int maxit,
                          int precond, int* iters, double* relres)
{
    return cg_entry(P, sigma2, b, x, nrhs, rtol, maxit, precond, iters, relres, P ? &P->st.cg_fallback_iter : nullptr,
                    true);
}

fkt_status fkt_cg_solve_noalloc(fkt_plan_t P, double sigma2, const void* b, void* x, int nrhs, double rtol, int maxit,
                                int precond, int* iters, double* relres)
{
    if (!P) return fail(FKT_EINVAL, "plan is NULL");
    if (!P->on_device) return fail(FKT_EDEVICE, "host-only plan (device = -1) cannot run fkt_cg_solve_noalloc");
    if (!b || !x) return fail(FKT_EINVAL, "b or x is NULL");
    if (nrhs < 1 || nrhs > 64) return fail(FKT_EINVAL, "nrhs must be in [1, 64]");
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2)) return fail(FKT_EINVAL, "sigma2 must be >= 0");
    if (!(rtol > 0.0)) return fail(FKT_EINVAL, "rtol must be > 0");
    if (maxit < 1) return fail(FKT_EINVAL, "maxit must be >= 1");
    if (precond < 0 || precond > 2) return fail(FKT_EUNSUPPORTED, "unknown preconditioner");
    // preconditioner state is built (and allocated) by fkt_cg_solve or
    // fkt_precond_coarse, never here
    const bool two_level = P->coarse_k > 0 && P->coarse_sigma2 == sigma2 && P->learn;
    if (precond >= 1 && !two_level && P->bj_sigma2 != sigma2)
        return fail(FKT_EINVAL, "block-Jacobi factors for this sigma2 are not built: call fkt_cg_solve with this "
                                "sigma2 and precond 1 or 2 first");
    if (precond == 2 && (!P->learn || P->learn_sigma2 != sigma2))
        return fail(FKT_EINVAL, "the learned preconditioner has no state for this sigma2: call fkt_learn_params or "
                                "fkt_cg_solve with precond 2 and this sigma2 first");
    const size_t es = P->opt.prec == FKT_F32 ? sizeof(float) : sizeof(double);
    const size_t need = fkt::cg_work_bytes_for(P->n, nrhs, P->cg_nseg, es, precond == 2);
    DeviceScope ds(P->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    void* region = nullptr;
    size_t cap = 0;
    const hipError_t e = fkt::cg_scratch(P->opt.device, &region, &cap);
    if (e != hipSuccess) return hip_fail(e, "scratch array address");
    if (need > cap)
        return fail(FKT_EINVAL, "fkt_cg_solve_noalloc needs " + std::to_string(need) + " bytes of work space for n = " +
                                    std::to_string(P->n) + ", nrhs = " + std::to_string(nrhs) + "; its scratch array holds " +
                                    std::to_string(cap));
    fkt::CgPlanView v{P->n,         (int)P->opt.prec, P->opt.device, P->stream,    P->dp.perm,   P->bj_nleaf,
                      P->bj_maxleaf, P->bj_begin,       P->bj_count,  P->bj_off,    P->bj_inv,    P->learn,
                      P->cg_nseg,    P->cg_seg_off,     P->cg_row_seg};
    v.coarse = two_level ? 1 : 0;
    v.active = P->inst_active;
    return fkt::cg_solve_impl(P, v, sigma2, b, x, nrhs, rtol, maxit, precond, iters, relres, &P->st.cg_fallback_iter,
                              false, nullptr, nullptr, nullptr, region, cap);
}

fkt_status fkt_cg_solve_refined(fkt_plan_t P, fkt_plan_t Q, double sigma2, const double* b, double* x, int nrhs,
                                double rtol, int maxit, int precond, int* iters, int* outer, double* relres)
{
    if (!P || !Q) return fail(FKT_EINVAL, "plan is NULL");
    if (!P->on_device || !Q->on_device) return fail(FKT_EDEVICE, "host-only plans cannot run fkt_cg_solve_refined");
    if (P->opt.prec != FKT_F64 || Q->opt.prec != FKT_F32)
        return fail(FKT_EINVAL, "fkt_cg_solve_refined takes an FP64 plan and an FP32 plan");
    if (P->n != Q->n || P->d != Q->d || P->opt.device != Q->opt.device || P->T.inst_begin != Q->T.inst_begin)
        return fail(FKT_EINVAL, "the two plans must cover the same points, instances and device");
    if (!b || !x) return fail(FKT_EINVAL, "b or x is NULL");
    if (nrhs < 1 || nrhs > 64) return fail(FKT_EINVAL, "nrhs must be in [1, 64]");
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2)) return fail(FKT_EINVAL, "sigma2 must be >= 0");
    if (!(rtol > 0.0)) return fail(FKT_EINVAL, "rtol must be > 0");
    if (maxit < 1) return fail(FKT_EINVAL, "maxit must be >= 1");
    if (precond < 0 || precond > 2) return fail(FKT_EUNSUPPORTED, "unknown preconditioner");
    DeviceScope ds(P->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    fkt::CgPlanView v{P->n,         (int)P->opt.prec, P->opt.device, P->stream,    P->dp.perm,   P->bj_nleaf,
                      P->bj_maxleaf, P->bj_begin,       P->bj_count,  P->bj_off,    P->bj_inv,    P->learn,
                      P->cg_nseg,    P->cg_seg_off,     P->cg_row_seg};
    // CG on the FP32 plan with its residual replaced by the FP64 one
    return cg_entry(Q, sigma2, b, x, nrhs, rtol, maxit, precond, iters, relres, &Q->st.cg_fallback_iter, true, P, &v,
                    outer);
}

static fkt_status learn_entry(fkt_plan_t P, double sigma2)
{
    if (!P) return fail(FKT_EINVAL, "plan is NULL");
    if (!P->on_device) return fail(FKT_EDEVICE, "host-only plan (device = -1) has no learned preconditioner");
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return fail(FKT_EINVAL, "sigma2 must be > 0");
    return ensure_learn(P, sigma2);
}

static fkt_status judge_filter(fkt_plan_t P, double sigma2, uint64_t seed, int judge_iters, int* accepted);

int64_t fkt_learn_nparams(void) { return fkt::kLearnParams; }

fkt_status fkt_learn_params(fkt_plan_t P, double sigma2, float* params, int set)
{
    if (!params) return fail(FKT_EINVAL, "params is NULL");
    DeviceScope ds(P ? P->opt.device : 0);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    fkt_status st = learn_entry(P, sigma2);
    if (st != FKT_OK) return st;
    const hipError_t e = fkt::learn_params(P->learn, params, set != 0);
    return e == hipSuccess ? FKT_OK : hip_fail(e, "learned preconditioner parameters");
}

fkt_status fkt_learn_loss_grad(fkt_plan_t P, double sigma2, const double* v, int batch, double* loss, float* grad)
{
    if (!v || !loss) return fail(FKT_EINVAL, "v or loss is NULL");
    if (batch < 1 || batch > 64) return fail(FKT_EINVAL, "batch must be in [1, 64]");
    DeviceScope ds(P ? P->opt.device : 0);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    fkt_status st = learn_entry(P, sigma2);
    if (st != FKT_OK) return st;
    st = fkt::learn_loss_grad(P, P->learn, (int)P->opt.prec, sigma2, v, batch, loss);
    if (st != FKT_OK) return fail(st, "learned preconditioner loss/gradient");
    if (grad) {
        const hipError_t e = fkt::learn_grad(P->learn, grad);
        if (e != hipSuccess) return hip_fail(e, "learned preconditioner gradient copy");
    }
    return FKT_OK;
}

fkt_status fkt_learn_train(fkt_plan_t P, double sigma2, int steps, int batch, double lr, uint64_t seed,
                           double* loss_first, double* loss_last, int judge_iters, int* accepted)
{
    if (steps < 0) return fail(FKT_EINVAL, "steps must be >= 0");
    if (batch < 1 || batch > 64) return fail(FKT_EINVAL, "batch must be in [1, 64]");
    if (!(lr > 0.0) || !std::isfinite(lr)) return fail(FKT_EINVAL, "lr must be > 0");
    if (judge_iters < 0) return fail(FKT_EINVAL, "judge_iters must be >= 0");
    DeviceScope ds(P ? P->opt.device : 0);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    fkt_status st = learn_entry(P, sigma2);
    if (st != FKT_OK) return st;
    st = fkt::learn_train(P, P->learn, (int)P->opt.prec, sigma2, steps, batch, lr, seed, loss_first, loss_last);
    if (st != FKT_OK) return fail(st, "learned preconditioner training");
    return judge_filter(P, sigma2, seed, judge_iters, accepted);
}

fkt_status fkt_learn_cond_grad(fkt_plan_t P, double sigma2, const double* b, int lanczos, double* cond, float* grad)
{
    if (!b || !cond) return fail(FKT_EINVAL, "b or cond is NULL");
    if (lanczos < 2 || lanczos > 1000) return fail(FKT_EINVAL, "lanczos must be in [2, 1000]");
    DeviceScope ds(P ? P->opt.device : 0);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    fkt_status st = learn_entry(P, sigma2);
    if (st != FKT_OK) return st;
    double* r = nullptr;
    hipError_t e = hipMalloc(&r, sizeof(double) * P->n);
    if (e != hipSuccess) return hip_fail(e, "condition-number work vector");
    e = hipMemcpyAsync(r, b, sizeof(double) * P->n, hipMemcpyDeviceToDevice, P->stream);
    st = e == hipSuccess ? fkt::learn_cond_grad(P, P->learn, (int)P->opt.prec, sigma2, r, lanczos, cond) : FKT_EDEVICE;
    (void)hipFree(r);
    if (st != FKT_OK) return fail(st, "condition-number objective (a breakdown or a non-positive Ritz value)");
    if (grad) {
        e = fkt::learn_grad(P->learn, grad);
        if (e != hipSuccess) return hip_fail(e, "learned preconditioner gradient copy");
    }
    return FKT_OK;
}

fkt_status fkt_learn_train_cond(fkt_plan_t P, double sigma2, int steps, int lanczos, double lr, uint64_t seed,
                                double* cond_first, double* cond_last, int judge_iters, int* accepted)
{
    if (steps < 0) return fail(FKT_EINVAL, "steps must be >= 0");
    if (lanczos < 2 || lanczos > 1000) return fail(FKT_EINVAL, "lanczos must be in [2, 1000]");
    if (!(lr > 0.0) || !std::isfinite(lr)) return fail(FKT_EINVAL, "lr must be > 0");
    if (judge_iters < 0) return fail(FKT_EINVAL, "judge_iters must be >= 0");
    DeviceScope ds(P ? P->opt.device : 0);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    fkt_status st = learn_entry(P, sigma2);
    if (st != FKT_OK) return st;
    st = fkt::learn_train_cond(P, P->learn, (int)P->opt.prec, sigma2, steps, lanczos, lr, seed, cond_first, cond_last);
    if (st != FKT_OK) return fail(st, "learned preconditioner training (condition number)");
    return judge_filter(P, sigma2, seed, judge_iters, accepted);
}

// Block-Jacobi judges a trained filter: judge_iters CG iterations on a
// Gaussian right-hand side with each preconditioner; if the learned filter
// ends with the larger residual, its last layer is zeroed, which is
// block-Jacobi exactly.
static fkt_status judge_filter(fkt_plan_t P, double sigma2, uint64_t seed, int judge_iters, int* accepted)
{
    fkt_status st = FKT_OK;
    if (accepted) *accepted = 1;
    if (judge_iters == 0) return FKT_OK;
    const size_t es = P->opt.prec == FKT_F32 ? sizeof(float) : sizeof(double);
    void *b = nullptr, *x = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&b, es * P->n)) != hipSuccess || (e = hipMalloc(&x, es * P->n)) != hipSuccess) {
        if (b) (void)hipFree(b);
        return hip_fail(e, "judge buffers");
    }
    double rr[2] = {0.0, 0.0};
    if ((e = fkt::learn_randn(P->learn, b, P->n, P->opt.prec == FKT_F32, seed ^ 0x4A554447ull)) != hipSuccess)
        st = hip_fail(e, "judge right-hand side");
    for (int pc = 1; pc <= 2 && st == FKT_OK; ++pc) {
        if ((e = hipMemsetAsync(x, 0, es * P->n, P->stream)) != hipSuccess) {
            st = hip_fail(e, "judge initial guess");
            break;
        }
        int it = 0;
        const fkt_status s2 = cg_entry(P, sigma2, b, x, 1, 1e-300, judge_iters, pc, &it, &rr[pc - 1], nullptr);
        if (s2 != FKT_OK && s2 != FKT_ENOTCONV) st = s2;
    }
    (void)hipFree(b);
    (void)hipFree(x);
    if (st != FKT_OK) return st;
    if (!(rr[1] < rr[0])) {
        std::vector<float> w(fkt::kLearnParams);
        if ((e = fkt::learn_params(P->learn, w.data(), false)) != hipSuccess) return hip_fail(e, "judge reset");
        for (int i = fkt::kLearnParams - fkt::kLearnHidden - 1; i < fkt::kLearnParams; ++i) w[i] = 0.f;
        if ((e = fkt::learn_params(P->learn, w.data(), true)) != hipSuccess) return hip_fail(e, "judge reset");
        if (accepted) *accepted = 0;
    }
    return FKT_OK;
}

struct fkt_graph_s {
    fkt_plan_t plan = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~fkt_graph_s()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

fkt_status fkt_graph_create(fkt_plan_t P, const void* x, void* y, int nrhs, fkt_graph_t* out)
{
    if (!out) return fail(FKT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!P) return fail(FKT_EINVAL, "plan is NULL");
    if (!P->on_device) return fail(FKT_EDEVICE, "host-only plan (device = -1) cannot run fkt_mvm");
    if (!x || !y) return fail(FKT_EINVAL, "x or y is NULL");
    if (nrhs < 1 || nrhs > 64) return fail(FKT_EINVAL, "nrhs must be in [1, 64]");
    DeviceScope ds(P->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    fkt_graph_s* G = new (std::nothrow) fkt_graph_s();
    if (!G) {
        (void)hipStreamDestroy(cap);
        return fail(FKT_ENOMEM, "graph allocation");
    }
    G->plan = P;
    // the whole MVM as fkt_mvm enqueues it (no memset nodes: the
    // accumulators are cleared by the gather kernel); with opt.overlap the
    // near field's branch on the plan's second stream joins the capture
    // through the fork event and returns through the join event, so the
    // graph keeps the near/far concurrency of eager launches
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipSuccess;
        if (P->opt.mrhs != 0 && nrhs % fkt::kMrCols == 0)
            le = fkt::launch_mvm_mrhs(P->dp, P->wk, P->mr, (const float*)x, (float*)y, nrhs, cap);
        else
            for (int c = 0; c < nrhs && le == hipSuccess;) {
                int ncols, nc;
                mvm_pass_width(P, nrhs - c, ncols, nc);
                le = fkt::launch_mvm_column(P->dp, P->wk, x, y, nrhs, c, ncols, nc, (int)P->opt.prec, cap,
                                            P->opt.overlap != 0, nullptr);
                c += ncols;
            }
        e = hipStreamEndCapture(cap, &G->graph);
        if (e == hipSuccess && le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        delete G;
        return hip_fail(e, "graph capture");
    }
    *out = G;
    return FKT_OK;
}

fkt_status fkt_graph_launch(fkt_graph_t G)
{
    if (!G) return fail(FKT_EINVAL, "graph is NULL");
    DeviceScope ds(G->plan->opt.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    const hipError_t e = hipGraphLaunch(G->exec, G->plan->stream);
    return e == hipSuccess ? FKT_OK : hip_fail(e, "graph launch");
}

void fkt_graph_destroy(fkt_graph_t G) { delete G; }

fkt_status fkt_autotune(const double* points, const int64_t* offsets, int ninst, int64_t n, int d, fkt_kernel k,
                        int order, const fkt_options* opt, const int* leaves, int nleaf, const int* far_modes,
                        int nmodes, int nrhs, int reps, int* best_leaf, int* best_mode, double* ms)
{
    if (!leaves || nleaf < 1 || !far_modes || nmodes < 1 || !best_leaf)
        return fail(FKT_EINVAL, "candidates, counts or best_leaf invalid");
    if (nrhs < 1 || nrhs > 64 || reps < 1) return fail(FKT_EINVAL, "nrhs must be in [1, 64] and reps >= 1");
    for (int m = 0; m < nmodes; ++m)
        if (far_modes[m] < 0 || far_modes[m] > 2) return fail(FKT_EINVAL, "far_modes entries must be 0, 1 or 2");
    fkt_options o;
    fkt_default_options(&o);
    if (opt) o = *opt;
    if (o.device < 0) return fail(FKT_EINVAL, "autotuning needs a device");
    o.profile = 0;
    const int64_t ntot = offsets ? offsets[ninst] : n;
    const size_t bytes = (o.prec == FKT_F32 ? sizeof(float) : sizeof(double)) * (size_t)ntot * nrhs;
    DeviceScope ds(o.device);
    if (!ds.ok) return fail(FKT_EDEVICE, "cannot select HIP device");
    void *x = nullptr, *y = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he;
    if ((he = hipMalloc(&x, bytes)) || (he = hipMalloc(&y, bytes)) || (he = hipMemset(x, 0, bytes)) ||
        (he = hipEventCreate(&e0)) || (he = hipEventCreate(&e1))) {
        if (x) (void)hipFree(x);
        if (y) (void)hipFree(y);
        return hip_fail(he, "autotune buffers");
    }
    fkt_status st = FKT_OK;
    double best_ms = 0.0;
    *best_leaf = -1;
    if (best_mode) *best_mode = -1;
    for (int c = 0; c < nleaf && st == FKT_OK; ++c) {
        for (int m = 0; m < nmodes && st == FKT_OK; ++m) {
            o.far_mode = far_modes[m];
            fkt_plan_t P = nullptr;
            st = offsets ? fkt_plan_batch(points, offsets, ninst, d, k, leaves[c], order, &o, &P)
                         : fkt_plan(points, n, d, k, leaves[c], order, &o, &P);
            if (st != FKT_OK) break;
            // one untimed pass, then reps timed passes bracketed by events
            st = fkt_mvm(P, x, y, nrhs);
            if (st == FKT_OK && hipEventRecord(e0, P->stream) != hipSuccess) st = fail(FKT_EDEVICE, "event record");
            for (int r = 0; r < reps && st == FKT_OK; ++r) st = fkt_mvm(P, x, y, nrhs);
            float t = 0.f;
            if (st == FKT_OK && (hipEventRecord(e1, P->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                st = fail(FKT_EDEVICE, "autotune timing");
            fkt_destroy(P);
            if (st != FKT_OK) break;
            const double per = (double)t / reps;
            if (ms) ms[(size_t)c * nmodes + m] = per;
            if (*best_leaf < 0 || per < best_ms) {
                best_ms = per;
                *best_leaf = leaves[c];
                if (best_mode) *best_mode = far_modes[m];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(y);
    return st;
}

fkt_status fkt_autotune_leaf(const double* points, const int64_t* offsets, int ninst, int64_t n, int d, fkt_kernel k,
                             int order, const fkt_options* opt, const int* candidates, int ncand, int nrhs, int reps,
                             int* best, double* ms)
{
    fkt_options o;
    fkt_default_options(&o);
    if (opt) o = *opt;
    const int mode = o.far_mode;
    return fkt_autotune(points, offsets, ninst, n, d, k, order, &o, candidates, ncand, &mode, 1, nrhs, reps, best,
                        nullptr, ms);
}

}  // extern "C"

namespace fkt {
fkt_status mvm_masked(fkt_plan_t P, const void* x, void* y, int nrhs)
{
    P->dp.inst_active = P->inst_active;
    const fkt_status st = fkt_mvm(P, x, y, nrhs);
    P->dp.inst_active = nullptr;
    return st;
}
}  // namespace fkt
