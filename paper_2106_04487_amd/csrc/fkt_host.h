// Host-side plan data of the FKT library: tree, interaction lists, tables.
//
// Everything here is built once per plan on the CPU and uploaded to the
// device; the device kernels only read it.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/fkt.h"

namespace fkt {

// Targets are processed in blocks of up to 64 consecutive tree positions
// inside one leaf: one block is one wavefront, one lane per target.
constexpr int kBlock = 64;
// s2m work units: at most this many consecutive points of one node.
constexpr int kUnitPoints = 1024;
// near-field work units: one source leaf and at most this many of its targets.
constexpr int kNearUnitTargets = 256;

// Binary space-partition tree (paper Sec. 3.1), nodes in preorder.
struct Tree {
    int d = 0;
    int64_t n = 0;
    std::vector<int64_t> perm;   // tree position -> original index
    std::vector<double> pts;     // [n][d] coordinates in tree order
    std::vector<double> lo, side, ctr;  // [nnodes][d] box corner, side lengths, centre
    std::vector<double> rho2;    // squared radius: max over the node's points of |x - ctr|^2
    std::vector<int64_t> begin, end;    // point range [begin, end) in tree order
    std::vector<int32_t> kid0, kid1, parent, level;
    // independent instances (a forest): instance i owns tree positions
    // [inst_begin[i], inst_begin[i + 1]) and the tree rooted at inst_root[i]
    // (-1 for an empty instance); one instance for a plain plan
    std::vector<int64_t> inst_begin;
    std::vector<int32_t> inst_root;
    int64_t nnodes() const { return (int64_t)rho2.size(); }
    bool leaf(int64_t b) const { return kid0[b] < 0 && kid1[b] < 0; }
};

// Far pairs of the 64-target blocks packed into 64-lane jobs: every
// (target, far node) pair of a block gets a lane; a job holds the pairs of at
// most max_nodes nodes, lanes grouped by node.
struct JobSet {
    std::vector<int32_t> job_off;     // [nblocks + 1] jobs of each block
    std::vector<int32_t> job_noff;    // [njobs + 1] into job_nodes
    std::vector<int32_t> job_nodes;   // far-node slots of each job
    std::vector<uint16_t> job_pairs;  // [njobs][64]: lane | node index << 6 (0xffff: empty)
    int max_nodes = 0;
};

// Near/far interaction lists per 64-target block, with lane masks: bit i of
// a mask is set when target (block begin + i) has that entry in its own
// near or far set (paper eq. accparam, per target). The far lists drive the
// multipole-to-target kernel; the near lists are transposed into the
// source-major near sets N_l (Sec. 3.2) that drive the near-field kernel.
struct Lists {
    std::vector<int32_t> blk_begin, blk_count;
    std::vector<int32_t> near_off, near_beg, near_end;  // near_off: [nblocks + 1] (host only)
    std::vector<uint64_t> near_mask;                    // (host only)
    std::vector<int32_t> near_tgt;                      // N_l: target positions, by leaf
    std::vector<int32_t> nu_beg, nu_end;                // near units: source leaf range
    std::vector<int32_t> nu_toff, nu_tcnt;              //   and their slice of near_tgt
    std::vector<int32_t> far_off, far_slot;             // far_off: [nblocks + 1] (host only)
    std::vector<uint64_t> far_mask;                     // (host only)
    // far field packed into 64-lane jobs: every (target, far node) pair of a
    // block gets its own lane; a job holds pairs of at most max_job_nodes nodes
    std::vector<int32_t> job_off;                       // [nblocks + 1] jobs of each block
    std::vector<int32_t> job_noff, job_nodes;           // [njobs + 1] node slots of each job
    std::vector<uint16_t> job_pairs;                    // [njobs][64]: lane | node index << 6
    int max_job_nodes = 0;
    std::vector<int32_t> slot_node;                     // far-node slot -> node id
    std::vector<double> slot_ctr, slot_scale;           // [nslots][d], [nslots]
    // s2m work units (node slot, point range) and the moment/partial they fill
    std::vector<int32_t> unit_slot, unit_begin, unit_end, unit_dst;
    // slots whose moments are the sum of several partials: slot, partial range
    std::vector<int32_t> red_slot, red_off;
    int64_t npartials = 0;
};

// Dimension/order-only constants (paper Appendix A.2; harmonics normalisation).
struct Tables {
    int d = 0, p = 0;
    int64_t rank = 0;
    std::vector<double> tbar;   // [(k*(p+1) + j)*(p+1) + m]
    std::vector<double> hnorm;  // [((e-3)*(p+1) + mu)*(p+1) + n], e = 3..d
    std::vector<double> exp2tab;  // [kExpTab] 2^(j / kExpTab), rounded to nearest
};

constexpr int kExpTab = 256;

void build_tree(const double* X, int64_t n, int d, int leaf_size, int max_depth, Tree& T);
// One tree per instance (points of instance i: rows offsets[i] .. offsets[i+1]
// of X), concatenated in instance order; no interaction crosses instances.
void build_forest(const double* X, const int64_t* offsets, int ninst, int d, int leaf_size, int max_depth, Tree& T);
void build_lists(const Tree& T, double theta, int max_job_nodes, Lists& L, fkt_plan_stats& st);
// pack L's far lists (far_off / far_slot / far_mask) into jobs
void pack_far_jobs(const Lists& L, int max_nodes, JobSet& J);
// far jobs over groups of `group` consecutive blocks (group <= 64): a far
// node's pairs from all blocks of a group are packed together, so a job's
// moment fragments serve more rows. job_off has one entry per group; a pair
// word is lane | (block - first block of the group) << 6 | node index << 12
// (0xffff: empty lane; max_nodes <= 4).
void pack_far_jobs_grouped(const Lists& L, int max_nodes, int group, JobSet& J);
bool check_jobs_grouped(const Lists& L, const JobSet& J, int group, std::string& err);
// node-major far jobs: for every far-node slot, its far targets (tree
// positions, ascending) in jobs of 64 lanes (-1 pads a slot's last job)
void pack_node_jobs(const Lists& L, std::vector<int32_t>& job_slot, std::vector<int32_t>& job_tgt);

void build_tables(int d, int p, Tables& tab);
// Bounds of every index the kernels derive from the lists (false + err).
bool check_lists(const Tree& T, const Lists& L, std::string& err);
bool check_jobs(const Lists& L, const std::vector<int32_t>& job_off, const std::vector<int32_t>& job_noff,
                const std::vector<int32_t>& job_nodes, const std::vector<uint16_t>& job_pairs, int max_nodes,
                std::string& err);

// K(r) for a kernel (K(0) = 0 for the singular 1/r), FP64, host side.
double kernel_value(const fkt_kernel& k, double r);

// Block-Jacobi preconditioner: for every leaf l, (K_ll + sigma2 I)^-1 as a
// dense symmetric matrix, from a Cholesky factorisation (FP64). inv holds
// the blocks back to back; off[l] is block l's first entry. Returns false if
// a block is not numerically positive definite.
bool build_block_jacobi(const Tree& T, const fkt_kernel& k, double sigma2, std::vector<int32_t>& leaf_begin,
                        std::vector<int32_t>& leaf_count, std::vector<int64_t>& off, std::vector<double>& inv);
int64_t binom(int64_t a, int64_t b);

// Radial compression (Appendix A.4, radial_host.cpp). Whether the kernel
// satisfies K' = q K with q a Laurent polynomial (exponential, 1/r, Gaussian).
bool radial_has_laurent_q(int kind);
// Exact R_k, k = 0..p, of eq. (f_g); false for a kernel without such a q.
bool radial_ranks(int kind, int d, int p, std::vector<int>& rank);
// Interpolative coefficients keeping the first min(keep, nj) radial rows of
// every degree: coef[(k * mj + jj) * mj + i] (mj = p / 2 + 1) with
// L_{k+2jj} = sum_i coef L_{k+2i}; false (+ err) when those rows do not
// span all rows or are dependent.
bool radial_interpolative(int kind, int d, int p, int keep, std::vector<double>& coef, std::string& err);

// Simple parallel-for over [0, n) on host threads.
void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& fn);

// Symmetric eigendecomposition of the n x n row-major matrix a (overwritten):
// on return w holds the eigenvalues in ascending order and row i of a the
// unit eigenvector of w[i]. False if the QR iteration does not converge.
bool sym_eig(int n, double* a, double* w);

// Spectra of the leaves' near-field diagonal blocks K(X_l, X_l) + sigma2 I
// (tree order) and the network's features, one row per eigenvalue.
constexpr int kLearnFeat = 4;
struct LeafSpectra {
    std::vector<int32_t> leaf_begin, leaf_count;
    std::vector<int64_t> off;   // [nleaves + 1] into vecs
    std::vector<double> vecs;   // per leaf m x m, row i = eigenvector i
    std::vector<double> vals;   // [n] eigenvalues, ascending within each leaf
    std::vector<float> feat;    // [n][kLearnFeat]
    int max_leaf = 0;
};
// Eigendecompositions of the leaf blocks K_ll + sigma2 I, or, with sub (one
// m x m block per leaf at the offsets of leaf_layout), of K_ll + sigma2 I -
// sub_l (symmetrised).
bool build_leaf_spectra(const Tree& T, const fkt_kernel& k, double sigma2, int leaf_cap, LeafSpectra& S,
                        const double* sub = nullptr);
// Leaf layout of the spectra (leaf_begin, leaf_count, off) without the
// eigendecompositions.
void leaf_layout(const Tree& T, LeafSpectra& S);

}  // namespace fkt
