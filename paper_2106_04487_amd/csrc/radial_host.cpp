// Compression of the radial expansion (Appendix A.4, eq. f_g), host side.
//
// For a kernel with K' = q K and q a Laurent polynomial (the exponential,
// 1/r and the Gaussian here), K^(m) = K P_m with P_0 = 1 and
// P_{m+1} = P_m' + q P_m, so the radial function of harmonic degree k,
// truncated at order p, is
//     sum_j r'^j F_kj(r),   F_kj = K(u) L_j(u),
//     L_j(u) = u^-j ([j = 0] + sum_{m=1..j} Tbar_kjm P_m(u) u^m),
// j = k, k+2, ..., <= p, in the kernel's scaled distance u = r / l (u = r
// for 1/r). The L_j have rational coefficients; their rank R_k over the
// rationals is the number of separable terms eq. (f_g) needs.
//
// Exactness: every coefficient is carried twice, as its residue modulo the
// prime 2^61 - 1 (exact; a rational whose numerator the prime divides would
// read as zero, which for these small-integer quantities does not happen)
// and as a long double (its value). Ranks, independence and the zero test of
// every reconstruction residual use the residues; the coefficients handed
// to the device are the long double values rounded to FP64.
//
// The decomposition kept is interpolative: the first n = R_k of the L_j
// (j = k, k+2, ...) are kept as the F_ki, and every other row is written as
// L_j = sum_i c_ji L_{k+2i}; the moments then combine as
//     M'_i = M_i + sum_{j > n} c_ji sigma^(j - (k+2i)) M_j,  sigma = s / l,
// for a node of scale s (moments normalised by s^j).
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "fkt_host.h"

namespace fkt {
namespace {

using u64 = unsigned long long;
constexpr u64 kPrime = (1ULL << 61) - 1;

u64 mred(unsigned __int128 z)
{
    const u64 lo = (u64)(z & kPrime), hi = (u64)(z >> 61);
    const u64 r = lo + hi;
    return r >= kPrime ? r - kPrime : r;
}
u64 mmul(u64 a, u64 b) { return mred((unsigned __int128)a * b); }
u64 madd(u64 a, u64 b)
{
    const u64 r = a + b;
    return r >= kPrime ? r - kPrime : r;
}
u64 mneg(u64 a) { return a ? kPrime - a : 0; }
u64 mpow(u64 a, u64 e)
{
    u64 r = 1;
    while (e) {
        if (e & 1) r = mmul(r, a);
        a = mmul(a, a);
        e >>= 1;
    }
    return r;
}
u64 minv(u64 a) { return mpow(a, kPrime - 2); }

// a rational: residue mod kPrime and value
struct Q {
    u64 m = 0;
    long double f = 0.0L;
};
Q qi(long long v)
{
    long long r = v % (long long)kPrime;
    if (r < 0) r += (long long)kPrime;
    return {(u64)r, (long double)v};
}
Q operator+(Q a, Q b) { return {madd(a.m, b.m), a.f + b.f}; }
Q operator-(Q a, Q b) { return {madd(a.m, mneg(b.m)), a.f - b.f}; }
Q operator*(Q a, Q b) { return {mmul(a.m, b.m), a.f * b.f}; }
Q operator/(Q a, Q b) { return {mmul(a.m, minv(b.m)), a.f / b.f}; }
bool is_zero(const Q& a) { return a.m == 0; }

Q qfact(int n)
{
    Q r = qi(1);
    for (int t = 2; t <= n; ++t) r = r * qi(t);
    return r;
}
Q qbinom(int n, int k)
{
    if (k < 0 || k > n) return qi(0);
    Q r = qi(1);
    for (int t = 1; t <= k; ++t) r = r * qi(n - k + t) / qi(t);
    return r;
}
Q qdfact(int n)  // n!! with (-1)!! = 1
{
    Q r = qi(1);
    for (int t = n; t > 1; t -= 2) r = r * qi(t);
    return r;
}

// cos^i = sum_k A(k, i) C_k^alpha, alpha = (d - 2) / 2 (Appendix A.2)
Q coef_A(int k, int i, int d)
{
    if (k > i || ((i - k) & 1)) return qi(0);
    const Q alpha = qi(d - 2) / qi(2);
    Q rise = qi(1);
    for (int t = 0; t < (i + k) / 2 + 1; ++t) rise = rise * (alpha + qi(t));
    return qfact(i) * (alpha + qi(k)) / (qi(1LL << i) * qfact((i - k) / 2) * rise);
}
// derivative coefficients of Lemma A.2
Q coef_B(int n, int m)
{
    if (m < 1 || m > n) return qi(0);
    const Q s = ((n + m) & 1) ? qi(-1) : qi(1);
    return s * qdfact(2 * n - 2 * m - 1) * qbinom(2 * n - m - 1, m - 1) / qi(1LL << n);
}
Q coef_tbar(int d, int k, int j, int m)
{
    Q s = qi(0);
    const int n0 = std::max((j + k) / 2, m);
    for (int n = n0; n <= j; ++n) {
        const int i = 2 * n - j;
        const Q pw = (i & 1) ? qi(-(1LL << i)) : qi(1LL << i);  // (-2)^i
        s = s + coef_A(k, i, d) * pw * qbinom(n, i) * coef_B(n, m) / qfact(n);
    }
    return s;
}

using Laurent = std::map<int, Q>;

void lacc(Laurent& a, int e, const Q& v)
{
    auto it = a.find(e);
    if (it == a.end())
        a[e] = v;
    else
        it->second = it->second + v;
}

// q of K' = q K in the scaled distance, or false
bool laurent_q(int kind, Laurent& q)
{
    q.clear();
    switch (kind) {
    case FKT_LAPLACE: q[-1] = qi(-1); return true;      // 1/u
    case FKT_EXPONENTIAL: q[0] = qi(-1); return true;   // e^-u
    case FKT_GAUSSIAN: q[1] = qi(-1); return true;      // e^(-u^2/2)
    default: return false;
    }
}

// rows L_j (j = k, k+2, ..., <= p) of harmonic degree k
std::vector<Laurent> radial_rows(const Laurent& q, int d, int k, int p)
{
    std::vector<Laurent> P(1);
    P[0][0] = qi(1);
    for (int m = 0; m < p; ++m) {
        Laurent nx;
        for (const auto& [e, v] : P[m]) {
            if (e != 0) lacc(nx, e - 1, v * qi(e));
            for (const auto& [f, w] : q) lacc(nx, e + f, v * w);
        }
        P.push_back(nx);
    }
    std::vector<Laurent> rows;
    for (int j = k; j <= p; j += 2) {
        Laurent L;
        if (j == 0) L[0] = qi(1);
        for (int m = 1; m <= j; ++m) {
            const Q t = coef_tbar(d, k, j, m);
            if (is_zero(t)) continue;
            for (const auto& [e, v] : P[m]) lacc(L, e + m - j, v * t);
        }
        rows.push_back(L);
    }
    return rows;
}

// residue matrix (rows x columns over the union of powers), the columns' powers
std::vector<std::vector<u64>> residues(const std::vector<Laurent>& rows, std::vector<int>& cols)
{
    std::map<int, int> idx;
    for (const auto& r : rows)
        for (const auto& [e, v] : r) idx[e] = 0;
    cols.clear();
    for (auto& [e, i] : idx) {
        i = (int)cols.size();
        cols.push_back(e);
    }
    std::vector<std::vector<u64>> M(rows.size(), std::vector<u64>(cols.size(), 0));
    for (size_t i = 0; i < rows.size(); ++i)
        for (const auto& [e, v] : rows[i]) M[i][idx[e]] = v.m;
    return M;
}

int rank_mod(std::vector<std::vector<u64>> M)
{
    int rk = 0;
    const int nr = (int)M.size(), nc = nr ? (int)M[0].size() : 0;
    for (int c = 0; c < nc && rk < nr; ++c) {
        int piv = -1;
        for (int i = rk; i < nr; ++i)
            if (M[i][c]) { piv = i; break; }
        if (piv < 0) continue;
        std::swap(M[rk], M[piv]);
        const u64 inv = minv(M[rk][c]);
        for (int i = 0; i < nr; ++i) {
            if (i == rk || !M[i][c]) continue;
            const u64 f = mmul(M[i][c], inv);
            for (int cc = 0; cc < nc; ++cc) M[i][cc] = madd(M[i][cc], mneg(mmul(f, M[rk][cc])));
        }
        ++rk;
    }
    return rk;
}

}  // namespace

bool radial_has_laurent_q(int kind)
{
    Laurent q;
    return laurent_q(kind, q);
}

bool radial_ranks(int kind, int d, int p, std::vector<int>& rank)
{
    Laurent q;
    if (!laurent_q(kind, q)) return false;
    rank.assign(p + 1, 0);
    for (int k = 0; k <= p; ++k) {
        std::vector<int> cols;
        rank[k] = rank_mod(residues(radial_rows(q, d, k, p), cols));
    }
    return true;
}

bool radial_interpolative(int kind, int d, int p, int keep, std::vector<double>& coef, std::string& err)
{
    Laurent q;
    if (!laurent_q(kind, q)) {
        err = "the kernel has no K' = q K with a Laurent polynomial q";
        return false;
    }
    const int mj = p / 2 + 1;
    coef.assign((size_t)(p + 1) * mj * mj, 0.0);
    for (int k = 0; k <= p; ++k) {
        const std::vector<Laurent> rows = radial_rows(q, d, k, p);
        const int nj = (int)rows.size();
        const int n = std::min(keep, nj);
        std::vector<int> cols;
        const std::vector<std::vector<u64>> M = residues(rows, cols);
        std::vector<std::vector<u64>> lead(M.begin(), M.begin() + n);
        if (rank_mod(M) != n || rank_mod(lead) != n) {
            err = "degree " + std::to_string(k) + ": the first " + std::to_string(n) +
                  " radial rows do not span the expansion";
            return false;
        }
        // n columns on which the leading rows are independent
        std::vector<int> chosen;
        for (int c = 0; c < (int)cols.size() && (int)chosen.size() < n; ++c) {
            std::vector<std::vector<u64>> sub(n);
            for (int i = 0; i < n; ++i) {
                for (int cc : chosen) sub[i].push_back(M[i][cc]);
                sub[i].push_back(M[i][c]);
            }
            if (rank_mod(sub) == (int)chosen.size() + 1) chosen.push_back(c);
        }
        auto val = [&](int row, int c) -> Q {
            auto it = rows[row].find(cols[c]);
            return it == rows[row].end() ? qi(0) : it->second;
        };
        for (int jj = 0; jj < nj; ++jj) {
            // A c = b on the chosen columns: A[r][i] = L_i[col_r], b[r] = L_jj[col_r]
            std::vector<std::vector<Q>> A(n, std::vector<Q>(n + 1));
            for (int r = 0; r < n; ++r) {
                for (int i = 0; i < n; ++i) A[r][i] = val(i, chosen[r]);
                A[r][n] = val(jj, chosen[r]);
            }
            for (int c = 0; c < n; ++c) {
                int piv = -1;
                for (int r = c; r < n; ++r)
                    if (!is_zero(A[r][c]) && (piv < 0 || fabsl(A[r][c].f) > fabsl(A[piv][c].f))) piv = r;
                if (piv < 0) {
                    err = "internal error: singular radial system";
                    return false;
                }
                std::swap(A[c], A[piv]);
                for (int r = 0; r < n; ++r) {
                    if (r == c || is_zero(A[r][c])) continue;
                    const Q f = A[r][c] / A[c][c];
                    for (int cc = c; cc <= n; ++cc) A[r][cc] = A[r][cc] - f * A[c][cc];
                }
            }
            std::vector<Q> cvec(n);
            for (int i = 0; i < n; ++i) cvec[i] = A[i][n] / A[i][i];
            // exact check on every column: L_jj - sum_i c_i L_i = 0
            for (int c = 0; c < (int)cols.size(); ++c) {
                Q r = val(jj, c);
                for (int i = 0; i < n; ++i) r = r - cvec[i] * val(i, c);
                if (!is_zero(r)) {
                    err = "internal error: radial row " + std::to_string(jj) + " of degree " + std::to_string(k) +
                          " is not reproduced";
                    return false;
                }
            }
            for (int i = 0; i < n; ++i)
                coef[((size_t)k * mj + jj) * mj + i] = is_zero(cvec[i]) ? 0.0 : (double)cvec[i].f;
        }
    }
    return true;
}

}  // namespace fkt
