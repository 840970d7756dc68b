// Host plan builder: space-partition tree, per-target near/far partition
// gathered into 64-target blocks, and the expansion's constant tables.
//
// Built with -ffp-contract=off: the far test of eq. (accparam) must give the
// same answer as any other FP64 evaluation of the same predicate (summed in
// axis order, multiply then add, no fused multiply-add).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "fkt_host.h"

namespace fkt {

void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& fn)
{
    if (n <= 0) return;
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nthreads = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 16));
    if (n <= grain || nthreads == 1) { fn(0, n); return; }
    std::atomic<int64_t> next(0);
    auto worker = [&]() {
        for (;;) {
            int64_t b = next.fetch_add(grain);
            if (b >= n) break;
            fn(b, std::min(n, b + grain));
        }
    };
    std::vector<std::thread> pool;
    for (int64_t t = 1; t < nthreads; ++t) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
}

int64_t binom(int64_t a, int64_t b)
{
    if (b < 0 || a < 0 || b > a) return 0;
    int64_t r = 1;
    for (int64_t i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return r;
}

// ---------------------------------------------------------------- tree

namespace {
struct Pending {
    int64_t begin, end;
    int32_t parent, level, which;
    double lo[8], side[8];
};
}  // namespace

// Orders a leaf's points by continued midplane halving of the longest side
// (down to groups of kLeafGroup points) so that every 64-target block is a
// compact piece of space. Only the order inside the leaf changes: leaf
// membership, and so the partition, is untouched.
constexpr int64_t kLeafGroup = 16;
static void order_leaf(const double* X, int d, const double* lo_in, const double* side_in, int64_t* idx,
                       int64_t cnt, int64_t* scratch, int depth = 0)
{
    if (cnt <= kLeafGroup || depth >= 64) return;
    double lo[8] = {0}, side[8] = {0};
    for (int a = 0; a < d; ++a) { lo[a] = lo_in[a]; side[a] = side_in[a]; }
    int axis = 0;
    for (int a = 1; a < d; ++a) if (side[a] > side[axis]) axis = a;
    if (!(side[axis] > 0.0)) return;
    const double mid = lo[axis] + 0.5 * side[axis];
    int64_t w = 0, r = 0;
    for (int64_t i = 0; i < cnt; ++i) {
        if (X[idx[i] * d + axis] < mid) idx[w++] = idx[i]; else scratch[r++] = idx[i];
    }
    std::memcpy(idx + w, scratch, sizeof(int64_t) * r);
    side[axis] *= 0.5;
    order_leaf(X, d, lo, side, idx, w, scratch, depth + 1);
    lo[axis] = mid;
    order_leaf(X, d, lo, side, idx + w, cnt - w, scratch, depth + 1);
}

// Sec. 3.1: hypercube root; each split halves one of the longest sides of the
// node (so the aspect ratio stays <= 2), choosing among those the axis that
// splits the points most evenly (lowest axis on ties); a node with at most
// leaf_size points (or at the depth cap) is a leaf. Children keep the stable
// order of their points; empty children are not created; ids are preorder.
void build_tree(const double* X, int64_t n, int d, int leaf_size, int max_depth, Tree& T)
{
    T = Tree();
    T.d = d;
    T.n = n;
    T.perm.resize(n);
    std::iota(T.perm.begin(), T.perm.end(), int64_t(0));
    std::vector<int64_t> scratch(n);

    Pending root{};
    root.begin = 0; root.end = n; root.parent = -1; root.level = 0; root.which = -1;
    double extent = 0.0;
    for (int a = 0; a < d; ++a) {
        double mn = X[a], mx = X[a];
        for (int64_t i = 1; i < n; ++i) {
            double v = X[i * d + a];
            mn = v < mn ? v : mn;
            mx = v > mx ? v : mx;
        }
        root.lo[a] = mn;
        extent = std::max(extent, mx - mn);
    }
    for (int a = 0; a < d; ++a) root.side[a] = extent;

    std::vector<Pending> stack{root};
    while (!stack.empty()) {
        Pending P = stack.back();
        stack.pop_back();
        const int32_t id = (int32_t)T.rho2.size();
        for (int a = 0; a < d; ++a) {
            T.lo.push_back(P.lo[a]);
            T.side.push_back(P.side[a]);
            T.ctr.push_back(P.lo[a] + 0.5 * P.side[a]);
        }
        T.rho2.push_back(0.0);
        T.begin.push_back(P.begin);
        T.end.push_back(P.end);
        T.kid0.push_back(-1);
        T.kid1.push_back(-1);
        T.parent.push_back(P.parent);
        T.level.push_back(P.level);
        if (P.parent >= 0) (P.which == 0 ? T.kid0 : T.kid1)[P.parent] = id;

        const int64_t cnt = P.end - P.begin;
        if (cnt <= leaf_size || P.level >= max_depth) {
            order_leaf(X, d, P.lo, P.side, T.perm.data() + P.begin, cnt, scratch.data());
            continue;
        }

        double smax = 0.0;
        for (int a = 0; a < d; ++a) smax = std::max(smax, P.side[a]);
        int axis = -1;
        int64_t best = 0, nl_best = 0;
        double mid_best = 0.0;
        for (int a = 0; a < d; ++a) {
            if (P.side[a] != smax) continue;
            const double mid = P.lo[a] + 0.5 * P.side[a];
            int64_t nl = 0;
            for (int64_t i = P.begin; i < P.end; ++i) nl += X[T.perm[i] * d + a] < mid;
            const int64_t score = std::llabs(2 * nl - cnt);
            if (axis < 0 || score < best) { axis = a; best = score; nl_best = nl; mid_best = mid; }
        }
        // stable partition of perm[begin, end) into {< mid} then {>= mid}
        int64_t w = P.begin, r = 0;
        for (int64_t i = P.begin; i < P.end; ++i) {
            const int64_t q = T.perm[i];
            if (X[q * d + axis] < mid_best) T.perm[w++] = q; else scratch[r++] = q;
        }
        std::memcpy(T.perm.data() + w, scratch.data(), sizeof(int64_t) * r);

        Pending L = P, R = P;
        L.parent = R.parent = id;
        L.level = R.level = P.level + 1;
        L.which = 0; R.which = 1;
        L.side[axis] = R.side[axis] = 0.5 * P.side[axis];
        R.lo[axis] = mid_best;
        L.end = P.begin + nl_best;
        R.begin = P.begin + nl_best;
        // LIFO: the left child is taken (and numbered) first
        if (R.end > R.begin) stack.push_back(R);
        if (L.end > L.begin) stack.push_back(L);
    }

    T.pts.resize((size_t)n * d);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a) T.pts[i * d + a] = X[T.perm[i] * d + a];
    T.inst_begin = {0, n};
    T.inst_root = {0};

    const int64_t nn = T.nnodes();
    parallel_for(nn, 64, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            double m = 0.0;
            for (int64_t i = T.begin[b]; i < T.end[b]; ++i) {
                double s = 0.0;
                for (int a = 0; a < d; ++a) {
                    const double u = T.pts[i * d + a] - T.ctr[b * d + a];
                    s = s + u * u;
                }
                m = s > m ? s : m;
            }
            T.rho2[b] = m;
        }
    });
}

void build_forest(const double* X, const int64_t* offsets, int ninst, int d, int leaf_size, int max_depth, Tree& T)
{
    T = Tree();
    T.d = d;
    T.n = offsets[ninst];
    T.inst_begin.assign(offsets, offsets + ninst + 1);
    T.inst_root.assign(ninst, -1);
    Tree Ti;
    for (int i = 0; i < ninst; ++i) {
        const int64_t po = offsets[i], ni = offsets[i + 1] - po;
        if (ni <= 0) continue;
        build_tree(X + po * d, ni, d, leaf_size, max_depth, Ti);
        const int32_t no = (int32_t)T.nnodes();
        T.inst_root[i] = no;
        for (int64_t q : Ti.perm) T.perm.push_back(q + po);
        T.pts.insert(T.pts.end(), Ti.pts.begin(), Ti.pts.end());
        T.lo.insert(T.lo.end(), Ti.lo.begin(), Ti.lo.end());
        T.side.insert(T.side.end(), Ti.side.begin(), Ti.side.end());
        T.ctr.insert(T.ctr.end(), Ti.ctr.begin(), Ti.ctr.end());
        T.rho2.insert(T.rho2.end(), Ti.rho2.begin(), Ti.rho2.end());
        for (int64_t b = 0; b < Ti.nnodes(); ++b) {
            T.begin.push_back(Ti.begin[b] + po);
            T.end.push_back(Ti.end[b] + po);
            T.kid0.push_back(Ti.kid0[b] >= 0 ? Ti.kid0[b] + no : -1);
            T.kid1.push_back(Ti.kid1[b] >= 0 ? Ti.kid1[b] + no : -1);
            T.parent.push_back(Ti.parent[b] >= 0 ? Ti.parent[b] + no : -1);
            T.level.push_back(Ti.level[b]);
        }
    }
}

// ------------------------------------------------------------- partition

// Pack each block's far pairs into jobs of 64 lanes, in list order (so a
// node's lanes are adjacent), starting a new job when 64 pairs or max_nodes
// distinct nodes are reached.
void pack_far_jobs(const Lists& L, int max_nodes, JobSet& J)
{
    const int64_t nb = (int64_t)L.blk_begin.size();
    J = JobSet();
    J.max_nodes = max_nodes;
    J.job_off.assign(nb + 1, 0);
    J.job_noff.assign(1, 0);
    for (int64_t q = 0; q < nb; ++q) {
        int in_job = kBlock, nodes_in_job = max_nodes;  // forces a new job
        for (int e = L.far_off[q]; e < L.far_off[q + 1]; ++e) {
            uint64_t m = L.far_mask[e];
            bool node_open = false;
            while (m) {
                if (in_job == kBlock || (!node_open && nodes_in_job == max_nodes)) {
                    J.job_pairs.resize(J.job_pairs.size() + kBlock, (uint16_t)0xffff);
                    J.job_noff.push_back(J.job_noff.back());
                    in_job = 0;
                    nodes_in_job = 0;
                    node_open = false;
                }
                if (!node_open) {
                    J.job_nodes.push_back(L.far_slot[e]);
                    J.job_noff.back() += 1;
                    ++nodes_in_job;
                    node_open = true;
                }
                const int lane = __builtin_ctzll(m);
                m &= m - 1;
                J.job_pairs[J.job_pairs.size() - kBlock + in_job] = (uint16_t)(lane | ((nodes_in_job - 1) << 6));
                ++in_job;
            }
        }
        J.job_off[q + 1] = (int32_t)(J.job_noff.size() - 1);
    }
}

void pack_far_jobs_grouped(const Lists& L, int max_nodes, int group, JobSet& J)
{
    const int64_t nb = (int64_t)L.blk_begin.size(), ng = (nb + group - 1) / group;
    J = JobSet();
    J.max_nodes = max_nodes;
    J.job_off.assign(ng + 1, 0);
    J.job_noff.assign(1, 0);
    struct Ent {
        int32_t slot, bg, e;
    };
    std::vector<Ent> ent;
    for (int64_t g = 0; g < ng; ++g) {
        ent.clear();
        const int64_t q0 = g * group, q1 = std::min<int64_t>(nb, q0 + group);
        for (int64_t q = q0; q < q1; ++q)
            for (int e = L.far_off[q]; e < L.far_off[q + 1]; ++e) ent.push_back({L.far_slot[e], (int32_t)(q - q0), e});
        std::stable_sort(ent.begin(), ent.end(), [](const Ent& u, const Ent& v) { return u.slot < v.slot; });
        int in_job = kBlock, nodes_in_job = max_nodes;  // forces a new job
        int32_t open_slot = -1;                          // node whose lanes the current job is filling
        for (const Ent& en : ent) {
            uint64_t m = L.far_mask[en.e];
            while (m) {
                if (in_job == kBlock || (open_slot != en.slot && nodes_in_job == max_nodes)) {
                    J.job_pairs.resize(J.job_pairs.size() + kBlock, (uint16_t)0xffff);
                    J.job_noff.push_back(J.job_noff.back());
                    in_job = 0;
                    nodes_in_job = 0;
                    open_slot = -1;
                }
                if (open_slot != en.slot) {
                    J.job_nodes.push_back(en.slot);
                    J.job_noff.back() += 1;
                    ++nodes_in_job;
                    open_slot = en.slot;
                }
                const int lane = __builtin_ctzll(m);
                m &= m - 1;
                J.job_pairs[J.job_pairs.size() - kBlock + in_job] =
                    (uint16_t)(lane | (en.bg << 6) | ((nodes_in_job - 1) << 12));
                ++in_job;
            }
        }
        J.job_off[g + 1] = (int32_t)(J.job_noff.size() - 1);
    }
}

void pack_node_jobs(const Lists& L, std::vector<int32_t>& job_slot, std::vector<int32_t>& job_tgt)
{
    const int64_t nb = (int64_t)L.blk_begin.size(), ns = (int64_t)L.slot_node.size();
    std::vector<int64_t> cnt(ns + 1, 0);
    for (int64_t q = 0; q < nb; ++q)
        for (int e = L.far_off[q]; e < L.far_off[q + 1]; ++e) cnt[L.far_slot[e] + 1] += __builtin_popcountll(L.far_mask[e]);
    // first job of each slot
    std::vector<int64_t> jb(ns + 1, 0);
    for (int64_t s2 = 0; s2 < ns; ++s2) jb[s2 + 1] = jb[s2] + (cnt[s2 + 1] + kBlock - 1) / kBlock;
    job_slot.assign(jb[ns], 0);
    job_tgt.assign((size_t)jb[ns] * kBlock, -1);
    for (int64_t s2 = 0; s2 < ns; ++s2)
        for (int64_t j = jb[s2]; j < jb[s2 + 1]; ++j) job_slot[j] = (int32_t)s2;
    // blocks in order, so every slot's targets come out ascending
    std::vector<int64_t> fill(ns, 0);
    for (int64_t q = 0; q < nb; ++q)
        for (int e = L.far_off[q]; e < L.far_off[q + 1]; ++e) {
            const int32_t s2 = L.far_slot[e];
            for (uint64_t m = L.far_mask[e]; m; m &= m - 1) {
                const int lane = __builtin_ctzll(m);
                job_tgt[(size_t)jb[s2] * kBlock + fill[s2]++] = L.blk_begin[q] + lane;
            }
        }
}

namespace {
struct BlockLists {
    std::vector<int32_t> near_node, far_node;
    std::vector<uint64_t> near_mask, far_mask;
};
}  // namespace

// For every target t, walking from the root: t is in F_b when b is the first
// node on the path with rho_b^2 < theta^2 |t - c_b|^2 (eq. accparam), and in
// N_l for each leaf l reached without such a node (Sec. 3.2). Done for 64
// targets at once with a mask of the targets still walking.
void build_lists(const Tree& T, double theta, int max_job_nodes, Lists& L, fkt_plan_stats& st)
{
    const int d = T.d;
    const int64_t nn = T.nnodes();
    const double theta2 = theta * theta;
    L = Lists();

    // 64 consecutive tree positions per block (blocks may span leaves: tree
    // order keeps them spatially compact, and full blocks keep lanes busy)
    for (int64_t o = 0; o < T.n; o += kBlock) {
        L.blk_begin.push_back((int32_t)o);
        L.blk_count.push_back((int32_t)std::min<int64_t>(kBlock, T.n - o));
    }
    const int64_t nb = (int64_t)L.blk_begin.size();
    std::vector<BlockLists> per(nb);

    parallel_for(nb, 16, [&](int64_t q0, int64_t q1) {
        std::vector<std::pair<int32_t, uint64_t>> stack;
        for (int64_t q = q0; q < q1; ++q) {
            const int64_t tb = L.blk_begin[q];
            const int cnt = L.blk_count[q];
            BlockLists& out = per[q];
            stack.clear();
            // one walk per instance the block's targets belong to, from its root
            int64_t i = std::upper_bound(T.inst_begin.begin(), T.inst_begin.end(), tb) - T.inst_begin.begin() - 1;
            for (; i + 1 < (int64_t)T.inst_begin.size() && T.inst_begin[i] < tb + cnt; ++i) {
                if (T.inst_root[i] < 0) continue;
                const int64_t l0 = std::max<int64_t>(T.inst_begin[i], tb) - tb;
                const int64_t l1 = std::min<int64_t>(T.inst_begin[i + 1], tb + cnt) - tb;
                if (l1 <= l0) continue;
                const uint64_t hi = l1 == 64 ? ~uint64_t(0) : ((uint64_t(1) << l1) - 1);
                const uint64_t lo = (uint64_t(1) << l0) - 1;
                stack.emplace_back(T.inst_root[i], hi & ~lo);
            }
            while (!stack.empty()) {
                auto [b, active] = stack.back();
                stack.pop_back();
                uint64_t far = 0;
                for (int lane = 0; lane < cnt; ++lane) {
                    if (!((active >> lane) & 1)) continue;
                    const double* t = &T.pts[(tb + lane) * d];
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) {
                        const double u = t[a] - T.ctr[b * d + a];
                        s = s + u * u;
                    }
                    if (T.rho2[b] < theta2 * s) far |= uint64_t(1) << lane;
                }
                if (far) { out.far_node.push_back(b); out.far_mask.push_back(far); }
                active &= ~far;
                if (!active) continue;
                if (T.leaf(b)) { out.near_node.push_back(b); out.near_mask.push_back(active); continue; }
                if (T.kid1[b] >= 0) stack.emplace_back(T.kid1[b], active);
                if (T.kid0[b] >= 0) stack.emplace_back(T.kid0[b], active);
            }
        }
    });

    // far-node slots, in node order
    std::vector<int32_t> slot_of(nn, -1);
    for (const auto& bl : per)
        for (int32_t b : bl.far_node) slot_of[b] = 1;
    for (int64_t b = 0; b < nn; ++b)
        if (slot_of[b] >= 0) { slot_of[b] = (int32_t)L.slot_node.size(); L.slot_node.push_back((int32_t)b); }

    L.near_off.assign(nb + 1, 0);
    L.far_off.assign(nb + 1, 0);
    for (int64_t q = 0; q < nb; ++q) {
        L.near_off[q + 1] = L.near_off[q] + (int32_t)per[q].near_node.size();
        L.far_off[q + 1] = L.far_off[q] + (int32_t)per[q].far_node.size();
    }
    int64_t near_pairs = 0, near_lane = 0, far_pairs = 0, far_lane = 0;
    std::vector<int64_t> ncount(nn + 1, 0);  // |N_l| per leaf
    for (int64_t q = 0; q < nb; ++q) {
        for (size_t e = 0; e < per[q].near_node.size(); ++e) {
            const int32_t b = per[q].near_node[e];
            L.near_beg.push_back((int32_t)T.begin[b]);
            L.near_end.push_back((int32_t)T.end[b]);
            L.near_mask.push_back(per[q].near_mask[e]);
            const int c = __builtin_popcountll(per[q].near_mask[e]);
            near_pairs += (int64_t)c * (T.end[b] - T.begin[b]);
            ncount[b + 1] += c;
        }
        for (size_t e = 0; e < per[q].far_node.size(); ++e) {
            L.far_slot.push_back(slot_of[per[q].far_node[e]]);
            L.far_mask.push_back(per[q].far_mask[e]);
            far_pairs += __builtin_popcountll(per[q].far_mask[e]);
        }
    }

    {
        JobSet J;
        pack_far_jobs(L, max_job_nodes, J);
        L.max_job_nodes = max_job_nodes;
        L.job_off = std::move(J.job_off);
        L.job_noff = std::move(J.job_noff);
        L.job_nodes = std::move(J.job_nodes);
        L.job_pairs = std::move(J.job_pairs);
    }
    far_lane = (int64_t)(L.job_noff.size() - 1) * kBlock;

    // N_l for every leaf l: the targets whose walk ends in l, in target order
    // (blocks and lanes are visited in tree order)
    for (int64_t b = 0; b < nn; ++b) ncount[b + 1] += ncount[b];
    L.near_tgt.resize(ncount[nn]);
    {
        std::vector<int64_t> fill(ncount.begin(), ncount.end() - 1);
        for (int64_t q = 0; q < nb; ++q)
            for (size_t e = 0; e < per[q].near_node.size(); ++e) {
                uint64_t m = per[q].near_mask[e];
                const int32_t b = per[q].near_node[e];
                while (m) {
                    const int lane = __builtin_ctzll(m);
                    m &= m - 1;
                    L.near_tgt[fill[b]++] = L.blk_begin[q] + lane;
                }
            }
    }
    for (int64_t b = 0; b < nn; ++b) {
        if (!T.leaf(b)) continue;
        for (int64_t o = ncount[b]; o < ncount[b + 1]; o += kNearUnitTargets) {
            const int64_t c = std::min<int64_t>(kNearUnitTargets, ncount[b + 1] - o);
            L.nu_beg.push_back((int32_t)T.begin[b]);
            L.nu_end.push_back((int32_t)T.end[b]);
            L.nu_toff.push_back((int32_t)o);
            L.nu_tcnt.push_back((int32_t)c);
            near_lane += ((c + kBlock - 1) / kBlock) * kBlock * (T.end[b] - T.begin[b]);
        }
    }

    const int64_t ns = (int64_t)L.slot_node.size();
    L.slot_ctr.resize(ns * d);
    L.slot_scale.resize(ns);
    int64_t s2m_terms = 0;
    for (int64_t s = 0; s < ns; ++s) {
        const int32_t b = L.slot_node[s];
        for (int a = 0; a < d; ++a) L.slot_ctr[s * d + a] = T.ctr[b * d + a];
        L.slot_scale[s] = T.rho2[b] > 0.0 ? std::sqrt(T.rho2[b]) : 1.0;
        const int64_t beg = T.begin[b], end = T.end[b];
        s2m_terms += end - beg;
        const int64_t nunits = (end - beg + kUnitPoints - 1) / kUnitPoints;
        if (nunits > 1) {
            L.red_slot.push_back((int32_t)s);
            L.red_off.push_back((int32_t)L.npartials);
        }
        for (int64_t u = 0; u < nunits; ++u) {
            L.unit_slot.push_back((int32_t)s);
            L.unit_begin.push_back((int32_t)(beg + u * kUnitPoints));
            L.unit_end.push_back((int32_t)std::min(end, beg + (u + 1) * kUnitPoints));
            L.unit_dst.push_back(nunits == 1 ? (int32_t)s : (int32_t)(-1 - L.npartials++));
        }
    }
    L.red_off.push_back((int32_t)L.npartials);

    st.nblocks = nb;
    st.far_nodes = ns;
    st.near_entries = (int64_t)L.near_beg.size();
    st.far_entries = (int64_t)L.far_slot.size();
    st.near_pairs = near_pairs;
    st.near_lane_pairs = near_lane;
    st.far_pairs = far_pairs;
    st.far_lane_pairs = far_lane;
    st.s2m_terms = s2m_terms;
}

// ----------------------------------------------------------------- tables

namespace {
using ld = long double;

ld fact(int n) { ld r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }
ld dfact(int n) { ld r = 1; for (int i = n; i > 1; i -= 2) r *= i; return r; }  // (-1)!! = 0!! = 1
ld rising(ld a, int n) { ld r = 1; for (int i = 0; i < n; ++i) r *= a + i; return r; }

// cos^i = sum_k A(k,i) C_k^alpha(cos), Appendix A.2 eq. (coschange), with the
// half-integer (i-k)/2 in the denominator read as a factorial.
ld coef_A(int k, int i, ld alpha)
{
    if (k > i || ((i - k) & 1)) return 0;
    return fact(i) * (alpha + k) / (std::pow((ld)2, (ld)i) * fact((i - k) / 2) * rising(alpha, (i + k) / 2 + 1));
}

// d^n/de^n K(r sqrt(1+e)) at e = 0 = sum_m B(n,m) K^(m)(r) r^m (Lemma A.2).
ld coef_B(int n, int m)
{
    if (m < 1 || m > n) return 0;
    const ld sgn = ((n + m) & 1) ? -1 : 1;
    return sgn * dfact(2 * n - 2 * m - 1) * (ld)binom(2 * n - m - 1, m - 1) / std::pow((ld)2, (ld)n);
}
}  // namespace

void build_tables(int d, int p, Tables& tab)
{
    tab.d = d;
    tab.p = p;
    const ld alpha = (ld)d / 2 - 1;
    const int P1 = p + 1;
    tab.exp2tab.resize(kExpTab);
    for (int j = 0; j < kExpTab; ++j) tab.exp2tab[j] = (double)std::exp2((ld)j / kExpTab);
    tab.tbar.assign((size_t)P1 * P1 * P1, 0.0);
    // Tbar_{k,j,m} = sum_n A_{k,2n-j} (-2)^{2n-j} C(n, 2n-j) B_{n,m} / n!  (the
    // binomial of the binomial expansion of eps^n is kept).
    for (int k = 0; k <= p; ++k)
        for (int j = k; j <= p; j += 2)
            for (int m = 1; m <= j; ++m) {
                ld s = 0;
                for (int n = std::max((j + k) / 2, m); n <= j; ++n) {
                    const int i = 2 * n - j;
                    s += coef_A(k, i, alpha) * std::pow((ld)-2, (ld)i) * (ld)binom(n, i) * coef_B(n, m) / fact(n);
                }
                tab.tbar[((size_t)k * P1 + j) * P1 + m] = (double)s;
            }

    // Orthonormal solid harmonics built one dimension at a time: a degree-k
    // harmonic in e dimensions is |x|^(k-mu) C_{k-mu}^{mu+(e-2)/2}(x_e/|x|)
    // times a degree-mu harmonic of the first e-1 coordinates. hnorm holds
    // the factor that makes each level orthonormal on its sphere, and at the
    // top level also sqrt(Z_k) of the addition theorem, so that
    //   sum_h Yhat_kh(u) Yhat_kh(v) = C_k^alpha(u . v)   (|u| = |v| = 1).
    tab.hnorm.assign((size_t)std::max(1, d - 2) * P1 * P1, 0.0);
    const ld pi = 3.14159265358979323846264338327950288L;
    const ld area = 2 * std::pow(pi, (ld)d / 2) / std::tgamma((ld)d / 2);
    for (int e = 3; e <= d; ++e)
        for (int mu = 0; mu <= p; ++mu)
            for (int n = 0; mu + n <= p; ++n) {
                const ld lam = mu + (ld)(e - 2) / 2;
                const ld logh = std::log(pi) + (1 - 2 * lam) * std::log((ld)2) + std::lgamma(n + 2 * lam) -
                                std::lgamma((ld)n + 1) - std::log(n + lam) - 2 * std::lgamma(lam);
                ld v = std::exp(-0.5L * logh);
                if (e == d) {
                    const int k = mu + n;
                    v *= std::sqrt(alpha * area / (k + alpha));
                }
                tab.hnorm[((size_t)(e - 3) * P1 + mu) * P1 + n] = (double)v;
            }
    tab.rank = binom(p + d, d);
}

// ------------------------------------------------------- block Jacobi

double kernel_value(const fkt_kernel& k, double r)
{
    const double l = k.lengthscale, s2 = k.variance;
    switch (k.kind) {
    case FKT_GAUSSIAN: return s2 * std::exp(-r * r / (2.0 * l * l));
    case FKT_EXPONENTIAL: return s2 * std::exp(-r / l);
    case FKT_MATERN32: { const double a = std::sqrt(3.0) * r / l; return s2 * (1.0 + a) * std::exp(-a); }
    case FKT_MATERN52: { const double a = std::sqrt(5.0) * r / l; return s2 * (1.0 + a + a * a / 3.0) * std::exp(-a); }
    case FKT_RATQUAD: return s2 * std::pow(1.0 + r * r / (2.0 * k.alpha * l * l), -k.alpha);
    case FKT_CAUCHY: return s2 / (1.0 + r * r / (l * l));
    case FKT_LAPLACE: return r > 0.0 ? s2 / r : 0.0;
    }
    return 0.0;
}

bool build_block_jacobi(const Tree& T, const fkt_kernel& k, double sigma2, std::vector<int32_t>& leaf_begin,
                        std::vector<int32_t>& leaf_count, std::vector<int64_t>& off, std::vector<double>& inv)
{
    const int d = T.d;
    leaf_begin.clear();
    leaf_count.clear();
    off.assign(1, 0);
    for (int64_t b = 0; b < T.nnodes(); ++b) {
        if (!T.leaf(b)) continue;
        const int64_t m = T.end[b] - T.begin[b];
        leaf_begin.push_back((int32_t)T.begin[b]);
        leaf_count.push_back((int32_t)m);
        off.push_back(off.back() + m * m);
    }
    inv.assign(off.back(), 0.0);
    std::atomic<bool> ok(true);
    parallel_for((int64_t)leaf_begin.size(), 1, [&](int64_t l0, int64_t l1) {
        std::vector<double> L, Wt;
        for (int64_t l = l0; l < l1; ++l) {
            const int m = leaf_count[l];
            const int64_t b0 = leaf_begin[l];
            L.assign((size_t)m * m, 0.0);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j <= i; ++j) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) {
                        const double u = T.pts[(b0 + i) * d + a] - T.pts[(b0 + j) * d + a];
                        s += u * u;
                    }
                    L[(size_t)i * m + j] = kernel_value(k, std::sqrt(s)) + (i == j ? sigma2 : 0.0);
                }
            // in-place Cholesky A = L L^T (lower triangle)
            for (int j = 0; j < m; ++j) {
                double dj = L[(size_t)j * m + j];
                for (int q = 0; q < j; ++q) dj -= L[(size_t)j * m + q] * L[(size_t)j * m + q];
                if (!(dj > 0.0)) { ok = false; return; }
                dj = std::sqrt(dj);
                L[(size_t)j * m + j] = dj;
                for (int i = j + 1; i < m; ++i) {
                    double s = L[(size_t)i * m + j];
                    for (int q = 0; q < j; ++q) s -= L[(size_t)i * m + q] * L[(size_t)j * m + q];
                    L[(size_t)i * m + j] = s / dj;
                }
            }
            // Wt = (L^-1)^T (upper triangular, rows contiguous), A^-1 = W^T W
            Wt.assign((size_t)m * m, 0.0);
            for (int j = 0; j < m; ++j) {
                double* wj = Wt.data() + (size_t)j * m;
                wj[j] = 1.0 / L[(size_t)j * m + j];
                for (int i = j + 1; i < m; ++i) {
                    const double* li = L.data() + (size_t)i * m;
                    double s = 0.0;
                    for (int q = j; q < i; ++q) s += li[q] * wj[q];
                    wj[i] = -s / li[i];
                }
            }
            double* out = inv.data() + off[l];
            for (int i = 0; i < m; ++i)
                for (int j = 0; j <= i; ++j) {
                    const double *wi = Wt.data() + (size_t)i * m, *wj = Wt.data() + (size_t)j * m;
                    double s = 0.0;
                    for (int q = i; q < m; ++q) s += wi[q] * wj[q];
                    out[(size_t)i * m + j] = s;
                    out[(size_t)j * m + i] = s;
                }
        }
    });
    return ok;
}

// Every index a device kernel derives from the work lists, checked against
// the sizes of the buffers it reads (a plan that fails is never launched).
bool check_lists(const Tree& T, const Lists& L, std::string& err)
{
    const int64_t n = T.n, nb = (int64_t)L.blk_begin.size(), ns = (int64_t)L.slot_node.size();
    auto bad = [&](const std::string& what, int64_t i) {
        err = "plan check: " + what + " at " + std::to_string(i);
        return false;
    };
    if ((int64_t)L.blk_count.size() != nb) return bad("block arrays", 0);
    // list offsets are 32-bit on the device
    constexpr int64_t kMax32 = 0x7fffffff;
    if ((int64_t)L.near_tgt.size() > kMax32 || (int64_t)L.far_slot.size() > kMax32 ||
        (int64_t)L.job_nodes.size() > kMax32 || (int64_t)L.job_noff.size() > kMax32 || L.npartials > kMax32) {
        err = "plan check: more list entries than 32-bit offsets hold (too many points for one plan)";
        return false;
    }
    for (int64_t q = 0; q < nb; ++q)
        if (L.blk_count[q] < 1 || L.blk_count[q] > kBlock || L.blk_begin[q] < 0 || L.blk_begin[q] + L.blk_count[q] > n)
            return bad("block range", q);
    // near units (source-major near field)
    const int64_t nu = (int64_t)L.nu_beg.size();
    if ((int64_t)L.nu_end.size() != nu || (int64_t)L.nu_toff.size() != nu || (int64_t)L.nu_tcnt.size() != nu)
        return bad("near-unit arrays", 0);
    for (int64_t u = 0; u < nu; ++u) {
        if (L.nu_beg[u] < 0 || L.nu_beg[u] > L.nu_end[u] || L.nu_end[u] > n) return bad("near-unit sources", u);
        if (L.nu_tcnt[u] < 1 || L.nu_tcnt[u] > kNearUnitTargets || L.nu_toff[u] < 0 ||
            (int64_t)L.nu_toff[u] + L.nu_tcnt[u] > (int64_t)L.near_tgt.size())
            return bad("near-unit targets", u);
    }
    for (size_t i = 0; i < L.near_tgt.size(); ++i)
        if (L.near_tgt[i] < 0 || L.near_tgt[i] >= n) return bad("near target", (int64_t)i);
    // target-major near lists (many-RHS near field)
    if ((int64_t)L.near_off.size() != nb + 1 || L.near_off[0] != 0 || L.near_off[nb] != (int64_t)L.near_beg.size())
        return bad("near list offsets", 0);
    for (int64_t q = 0; q < nb; ++q)
        if (L.near_off[q + 1] < L.near_off[q]) return bad("near list offsets", q);
    for (size_t e = 0; e < L.near_beg.size(); ++e)
        if (L.near_beg[e] < 0 || L.near_beg[e] > L.near_end[e] || L.near_end[e] > n) return bad("near entry", (int64_t)e);
    // far-field jobs
    if (!check_jobs(L, L.job_off, L.job_noff, L.job_nodes, L.job_pairs, L.max_job_nodes, err)) return false;
    if ((int64_t)L.slot_ctr.size() != ns * T.d || (int64_t)L.slot_scale.size() != ns) return bad("slot arrays", 0);
    // s2m units and partial sums
    for (size_t u = 0; u < L.unit_slot.size(); ++u) {
        if (L.unit_slot[u] < 0 || L.unit_slot[u] >= ns) return bad("s2m unit slot", (int64_t)u);
        if (L.unit_begin[u] < 0 || L.unit_begin[u] >= L.unit_end[u] || L.unit_end[u] > n ||
            L.unit_end[u] - L.unit_begin[u] > kUnitPoints)
            return bad("s2m unit range", (int64_t)u);
        const int32_t dst = L.unit_dst[u];
        if (dst >= 0 ? dst >= ns : (int64_t)(-1 - (int64_t)dst) >= L.npartials) return bad("s2m unit target", (int64_t)u);
    }
    if (L.red_off.size() != L.red_slot.size() + 1 || L.red_off.back() != L.npartials) return bad("partial lists", 0);
    for (size_t r = 0; r < L.red_slot.size(); ++r)
        if (L.red_slot[r] < 0 || L.red_slot[r] >= ns || L.red_off[r + 1] < L.red_off[r]) return bad("partial list", (int64_t)r);
    return true;
}

bool check_jobs_grouped(const Lists& L, const JobSet& J, int group, std::string& err)
{
    const int64_t nb = (int64_t)L.blk_begin.size(), ns = (int64_t)L.slot_node.size();
    const int64_t ng = (nb + group - 1) / group, njobs = (int64_t)J.job_noff.size() - 1;
    auto bad = [&](const std::string& what, int64_t i) {
        err = "plan check: " + what + " at " + std::to_string(i);
        return false;
    };
    if (group < 1 || group > 64 || J.max_nodes < 1 || J.max_nodes > 4) return bad("job grouping", group);
    if ((int64_t)J.job_off.size() != ng + 1 || J.job_off[0] != 0 || J.job_off[ng] != njobs)
        return bad("grouped job offsets", 0);
    if (J.job_noff[0] != 0 || J.job_noff[njobs] != (int64_t)J.job_nodes.size() ||
        (int64_t)J.job_pairs.size() != njobs * kBlock)
        return bad("grouped job arrays", 0);
    for (int64_t g = 0; g < ng; ++g) {
        if (J.job_off[g + 1] < J.job_off[g]) return bad("grouped job offsets", g);
        for (int64_t j = J.job_off[g]; j < J.job_off[g + 1]; ++j) {
            const int nn = J.job_noff[j + 1] - J.job_noff[j];
            if (nn < 1 || nn > J.max_nodes) return bad("grouped job node count", j);
            for (int k = 0; k < nn; ++k) {
                const int32_t sl = J.job_nodes[J.job_noff[j] + k];
                if (sl < 0 || sl >= ns) return bad("grouped job node slot", j);
            }
            int prev = 0;
            for (int lane = 0; lane < kBlock; ++lane) {
                const uint16_t pw = J.job_pairs[(size_t)j * kBlock + lane];
                if (pw == 0xffffu) continue;
                const int bg = (pw >> 6) & 63, node = pw >> 12;
                const int64_t q = g * group + bg;
                if (bg >= group || q >= nb || (pw & 63) >= L.blk_count[q] || node >= nn || node < prev)
                    return bad("grouped job pair", j);
                prev = node;  // lanes grouped by node, in node order
            }
        }
    }
    return true;
}

bool check_jobs(const Lists& L, const std::vector<int32_t>& job_off, const std::vector<int32_t>& job_noff,
                const std::vector<int32_t>& job_nodes, const std::vector<uint16_t>& job_pairs, int max_nodes,
                std::string& err)
{
    const int64_t nb = (int64_t)L.blk_begin.size(), ns = (int64_t)L.slot_node.size();
    const int64_t njobs = (int64_t)job_noff.size() - 1;
    struct {
        const std::vector<int32_t>& job_off;
        const std::vector<int32_t>& job_noff;
        const std::vector<int32_t>& job_nodes;
        const std::vector<uint16_t>& job_pairs;
        int max_nodes;
    } J{job_off, job_noff, job_nodes, job_pairs, max_nodes};
    auto bad = [&](const std::string& what, int64_t i) {
        err = "plan check: " + what + " at " + std::to_string(i);
        return false;
    };
    if ((int64_t)J.job_off.size() != nb + 1 || J.job_off[0] != 0 || J.job_off[nb] != njobs)
        return bad("job offsets", 0);
    if (J.job_noff[0] != 0 || J.job_noff[njobs] != (int64_t)J.job_nodes.size() ||
        (int64_t)J.job_pairs.size() != njobs * kBlock)
        return bad("job arrays", 0);
    for (int64_t q = 0; q < nb; ++q) {
        if (J.job_off[q + 1] < J.job_off[q]) return bad("job offsets", q);
        for (int64_t j = J.job_off[q]; j < J.job_off[q + 1]; ++j) {
            const int nn = J.job_noff[j + 1] - J.job_noff[j];
            if (nn < 1 || nn > J.max_nodes) return bad("job node count", j);
            for (int k = 0; k < nn; ++k) {
                const int32_t sl = J.job_nodes[J.job_noff[j] + k];
                if (sl < 0 || sl >= ns) return bad("job node slot", j);
            }
            int prev = 0;
            for (int lane = 0; lane < kBlock; ++lane) {
                const uint16_t pw = J.job_pairs[(size_t)j * kBlock + lane];
                if (pw == 0xffffu) continue;
                if ((pw & 63) >= L.blk_count[q] || (pw >> 6) >= nn || (int)(pw >> 6) < prev)
                    return bad("job pair", j);
                prev = pw >> 6;  // lanes grouped by node, in node order
            }
        }
    }
    return true;
}

}  // namespace fkt
