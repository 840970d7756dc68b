// Host side of the learned per-leaf preconditioner: the spectra of the
// near-field diagonal blocks A_l = K(X_l, X_l) + sigma2 I of the leaves, and
// the per-eigenvalue features the network reads.
//
// Symmetric eigendecomposition: Householder reduction to tridiagonal form,
// then implicit symmetric QR steps with the Wilkinson shift and deflation
// (Golub & Van Loan, Matrix Computations, Algorithms 8.3.1 and 8.3.3). The
// transformations are accumulated in U = Q^T, whose rows are rotated in
// place, so every update touches contiguous memory.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

#include "fkt_host.h"

namespace fkt {

bool sym_eig(int n, double* a, double* w)
{
    if (n <= 0) return true;
    std::vector<double> U((size_t)n * n, 0.0), v(n), p(n), t(n), e(n > 1 ? n - 1 : 1, 0.0);
    for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
    auto A = [&](int i, int j) -> double& { return a[(size_t)i * n + j]; };

    // 1. A = Q T Q^T with T tridiagonal; reflector k zeroes column k below
    //    the subdiagonal: H = I - beta v v^T, v supported on k+1..n-1.
    for (int k = 0; k + 2 < n; ++k) {
        double nrm2 = 0.0;
        for (int i = k + 1; i < n; ++i) nrm2 += A(i, k) * A(i, k);
        const double nrm = std::sqrt(nrm2);
        if (nrm == 0.0) continue;
        const double alpha = A(k + 1, k) > 0.0 ? -nrm : nrm;
        double vv = 0.0;
        for (int i = k + 1; i < n; ++i) {
            v[i] = A(i, k) - (i == k + 1 ? alpha : 0.0);
            vv += v[i] * v[i];
        }
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        // S <- H S H on the trailing block: p = beta S v, w = p - (beta/2)(v.p) v,
        // S -= v w^T + w v^T
        double vp = 0.0;
        for (int i = k + 1; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += A(i, j) * v[j];
            p[i] = beta * s;
            vp += v[i] * p[i];
        }
        const double K = 0.5 * beta * vp;
        for (int i = k + 1; i < n; ++i) p[i] -= K * v[i];
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) A(i, j) -= v[i] * p[j] + p[i] * v[j];
        A(k + 1, k) = alpha;
        A(k, k + 1) = alpha;
        for (int i = k + 2; i < n; ++i) A(i, k) = A(k, i) = 0.0;
        // Q <- Q H, i.e. U <- H U: rows k+1..n-1 of U minus beta v (v^T U)
        std::fill(t.begin(), t.end(), 0.0);
        for (int i = k + 1; i < n; ++i) {
            const double* ui = U.data() + (size_t)i * n;
            for (int c = 0; c < n; ++c) t[c] += v[i] * ui[c];
        }
        for (int i = k + 1; i < n; ++i) {
            double* ui = U.data() + (size_t)i * n;
            const double f = beta * v[i];
            for (int c = 0; c < n; ++c) ui[c] -= f * t[c];
        }
    }
    for (int i = 0; i < n; ++i) w[i] = A(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);

    // 2. Implicit QR on the tridiagonal (w, e): each step chases the bulge
    //    of a rotation R of rows/columns (k, k+1), T <- R T R^T, U <- R U.
    const double eps = std::numeric_limits<double>::epsilon();
    long steps = 0;
    const long max_steps = 64L * n + 64;
    for (;;) {
        for (int i = 0; i + 1 < n; ++i)
            if (std::fabs(e[i]) <= eps * (std::fabs(w[i]) + std::fabs(w[i + 1]))) e[i] = 0.0;
        int hi = n - 1;
        while (hi > 0 && e[hi - 1] == 0.0) --hi;
        if (hi == 0) break;
        int lo = hi - 1;
        while (lo > 0 && e[lo - 1] != 0.0) --lo;
        if (++steps > max_steps) return false;
        // Wilkinson shift: the eigenvalue of the trailing 2x2 closer to w[hi]
        const double dd = 0.5 * (w[hi - 1] - w[hi]), b = e[hi - 1];
        const double mu = w[hi] - b * b / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::hypot(dd, b));
        double x = w[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : z / r;
            if (k > lo) e[k - 1] = r;
            const double ak = w[k], bk = e[k], ck = w[k + 1];
            w[k] = c * c * ak + 2.0 * c * s * bk + s * s * ck;
            w[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ck;
            e[k] = c * s * (ck - ak) + (c * c - s * s) * bk;
            if (k + 1 < hi) {
                z = s * e[k + 1];
                e[k + 1] *= c;
            }
            x = e[k];
            double* u0 = U.data() + (size_t)k * n;
            double* u1 = u0 + n;
            for (int q = 0; q < n; ++q) {
                const double f0 = u0[q], f1 = u1[q];
                u0[q] = c * f0 + s * f1;
                u1[q] = c * f1 - s * f0;
            }
        }
    }

    // 3. ascending order; row i of a <- eigenvector of w[i]
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) { return w[i] < w[j]; });
    std::vector<double> ws(w, w + n);
    for (int i = 0; i < n; ++i) {
        w[i] = ws[ord[i]];
        std::copy(U.begin() + (size_t)ord[i] * n, U.begin() + (size_t)(ord[i] + 1) * n, a + (size_t)i * n);
    }
    return true;
}

void leaf_layout(const Tree& T, LeafSpectra& S)
{
    S.leaf_begin.clear();
    S.leaf_count.clear();
    S.off.assign(1, 0);
    for (int64_t b = 0; b < T.nnodes(); ++b) {
        if (!T.leaf(b)) continue;
        const int64_t m = T.end[b] - T.begin[b];
        S.leaf_begin.push_back((int32_t)T.begin[b]);
        S.leaf_count.push_back((int32_t)m);
        S.off.push_back(S.off.back() + m * m);
    }
}

bool build_leaf_spectra(const Tree& T, const fkt_kernel& k, double sigma2, int leaf_cap, LeafSpectra& S,
                        const double* sub)
{
    const int d = T.d;
    leaf_layout(T, S);
    const int64_t nl = (int64_t)S.leaf_begin.size();
    S.vecs.assign(S.off.back(), 0.0);
    S.vals.assign(T.n, 0.0);
    S.feat.assign((size_t)T.n * kLearnFeat, 0.f);
    S.max_leaf = 0;
    for (int32_t m : S.leaf_count) S.max_leaf = std::max(S.max_leaf, (int)m);
    std::atomic<bool> ok(true);
    parallel_for(nl, 1, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1 && ok; ++l) {
            const int m = S.leaf_count[l];
            const int64_t b0 = S.leaf_begin[l];
            double* A = S.vecs.data() + S.off[l];
            for (int i = 0; i < m; ++i)
                for (int j = 0; j <= i; ++j) {
                    double s = 0.0;
                    for (int c = 0; c < d; ++c) {
                        const double u = T.pts[(b0 + i) * d + c] - T.pts[(b0 + j) * d + c];
                        s += u * u;
                    }
                    double kv = kernel_value(k, std::sqrt(s)) + (i == j ? sigma2 : 0.0);
                    // two-level: the residual block, less the coarse part L_l L_l^T
                    if (sub) kv -= 0.5 * (sub[S.off[l] + (size_t)i * m + j] + sub[S.off[l] + (size_t)j * m + i]);
                    A[(size_t)i * m + j] = A[(size_t)j * m + i] = kv;
                }
            double* lam = S.vals.data() + b0;
            if (!sym_eig(m, A, lam) || !(lam[0] > 0.0)) {
                ok = false;
                return;
            }
            // features of eigenvalue i of leaf l (all O(1)):
            //   log(lam_i / sigma2) / 8, log(lam_max / sigma2) / 8,
            //   m / leaf_cap, (i + 1/2) / m
            const double lmax = lam[m - 1];
            for (int i = 0; i < m; ++i) {
                float* f = S.feat.data() + (size_t)(b0 + i) * kLearnFeat;
                f[0] = (float)(std::log(lam[i] / sigma2) / 8.0);
                f[1] = (float)(std::log(lmax / sigma2) / 8.0);
                f[2] = (float)((double)m / leaf_cap);
                f[3] = (float)((i + 0.5) / m);
            }
        }
    });
    return ok;
}

}  // namespace fkt
