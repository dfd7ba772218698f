// Planner of the discrete Laplace transform (Sect. 3, Def. 3.2, Algorithm 1):
// parameters, dyadic blocks of the frequencies and bands of the nodes, the
// Chebyshev tables and the kernel blocks K^{Y_m,Omega_l}.  Host, FP64.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "flt.h"
#include "laplace.h"

namespace flt {

// Index i of the dyadic interval holding v >= 0: (v1 2^-i, v1 2^(1-i)] for
// i < L, [0, v1 2^(1-L)] for i = L (Def. 3.2); exact compares after a guess.
static int lap_level(double v, double v1, int L)
{
    if (L == 1 || v <= std::ldexp(v1, 1 - L)) return L;
    int i = (int)std::floor(std::log2(v1 / v)) + 1;
    i = std::max(1, std::min(L - 1, i));
    while (i > 1 && v > std::ldexp(v1, 1 - i)) --i;
    while (i < L - 1 && v <= std::ldexp(v1, -i)) ++i;
    return i;
}

// Chebyshev nodes of [a, b]: centre + half-width cos((2r+1) pi / (2q)) (Sect. 2).
static void cheb_nodes(double a, double b, int q, double* out)
{
    for (int r = 0; r < q; ++r) out[r] = 0.5 * (a + b) + 0.5 * (b - a) * std::cos((2 * r + 1) * M_PI / (2.0 * q));
}

// Rank of a general kernel kappa(y, xi) = g(y xi) (Thm 3.3): the smallest q
// whose tensor Chebyshev interpolant is within (eps / 2) max(1, max |kappa|)
// of kappa on every block Y_m x Omega_l, m, l < L (absolute eps / 2 where the
// kernel is at most 1, as in the theorem's proof; relative to its size on the
// blocks near the origin, where a singular kernel exceeds 1 / eps and no
// floating-point evaluation, direct sums included, is absolutely that close).  With y = a u, xi = b v (a = y_1 2^-m, b = xi_1 2^-l,
// u, v in [1, 2]) the block's kappa is g(P u v), P = a b = y_1 xi_1 2^-(m+l),
// so the 2L - 3 values of m + l cover every block.  The error is taken on a
// 33 x 33 grid of [1, 2]^2 (endpoints included).  0 if no q <= LAP_MAX_Q does.
template <class G> static int lap_rank_general(double y1, double xi1, int L, double eps, G g)
{
    constexpr int NG = 33;
    double ug[NG];
    for (int i = 0; i < NG; ++i) ug[i] = 1.0 + (double)i / (NG - 1);
    for (int q = 2; q <= LAP_MAX_Q; ++q) {
        std::vector<double> tau(q), lam(q), Lu((size_t)NG * q), Gm((size_t)q * q), T1((size_t)NG * q);
        cheb_nodes(1.0, 2.0, q, tau.data());
        for (int r = 0; r < q; ++r) lam[r] = ((r & 1) ? -1.0 : 1.0) * std::sin((2 * r + 1) * M_PI / (2.0 * q));
        for (int i = 0; i < NG; ++i) {   // Lagrange basis at the grid, barycentric form (Sect. 2)
            int hit = -1;
            double den = 0.0;
            for (int r = 0; r < q; ++r) {
                if (ug[i] == tau[r]) hit = r;
                else den += lam[r] / (ug[i] - tau[r]);
            }
            for (int r = 0; r < q; ++r)
                Lu[(size_t)i * q + r] = hit >= 0 ? (r == hit ? 1.0 : 0.0) : lam[r] / (ug[i] - tau[r]) / den;
        }
        double worst = 0.0;
        for (int k = 2; k <= 2 * L - 2 && worst <= 0.5 * eps; ++k) {
            const double P = std::ldexp(y1 * xi1, -k);
            for (int s = 0; s < q; ++s)
                for (int r = 0; r < q; ++r) Gm[(size_t)s * q + r] = g(P * tau[s] * tau[r]);
            for (int i = 0; i < NG; ++i)   // T1 = Lu G
                for (int r = 0; r < q; ++r) {
                    double a = 0.0;
                    for (int s = 0; s < q; ++s) a += Lu[(size_t)i * q + s] * Gm[(size_t)s * q + r];
                    T1[(size_t)i * q + r] = a;
                }
            double err = 0.0, big = 1.0;
            for (int i = 0; i < NG; ++i)
                for (int j = 0; j < NG; ++j) {
                    double a = 0.0;
                    for (int r = 0; r < q; ++r) a += T1[(size_t)i * q + r] * Lu[(size_t)j * q + r];
                    const double gv = g(P * ug[i] * ug[j]);
                    err = std::max(err, std::fabs(a - gv));
                    big = std::max(big, std::fabs(gv));
                }
            worst = std::max(worst, err / big);
        }
        if (worst <= 0.5 * eps) return q;
    }
    return 0;
}

int build_laplace_plan(LapHost& hp, int64_t N, const double* xi, int64_t M, const double* y, double eps,
                       int dtype, int kernel)
{
    if (kernel != LAP_KERNEL_EXP && kernel != LAP_KERNEL_K12) return FLT_EINVAL;
    const bool general = kernel != LAP_KERNEL_EXP;
    if (!xi || !y || N < 1 || M < 1) return FLT_EINVAL;
    if (dtype != FLT_C64 && dtype != FLT_C128) return FLT_EINVAL;
    if (!(eps > 0.0 && eps < 1.0)) return FLT_EDOMAIN;
    if (eps < (dtype == FLT_C64 ? 1e-6 : 1e-14)) return FLT_EPRECISION;
    if (N > (int64_t)INT32_MAX || M > (int64_t)INT32_MAX) return FLT_ERANGE;
    double xi1 = 0.0, y1 = 0.0;
    for (int64_t k = 0; k < N; ++k) {
        if (!(xi[k] > 0.0) || !std::isfinite(xi[k])) return FLT_EDOMAIN;   // xi_k > 0 (Thm A.3)
        xi1 = std::max(xi1, xi[k]);
    }
    for (int64_t j = 0; j < M; ++j) {
        if (!(y[j] >= 0.0) || !std::isfinite(y[j])) return FLT_EDOMAIN;    // y_j >= 0
        if (general && !(y[j] > 0.0)) return FLT_EDOMAIN;                  // K_{1/2} is singular at 0
        y1 = std::max(y1, y[j]);
    }
    hp = LapHost();
    hp.N = N;
    hp.M = M;
    hp.dtype = dtype;
    hp.eps = eps;
    hp.xi1 = xi1;
    hp.y1 = y1;
    hp.kernel = kernel;
    if (!general) {
        hp.q = (int)std::ceil(0.5 + std::log(1.0 / eps) / std::log(4.0));
        // levels (the paper's M); all nodes at 0: one level, every block "kernel = 1"
        hp.L = y1 > 0.0 ? (int)std::ceil(std::log2(y1 * xi1 / eps)) + 1 : 1;
    } else {
        // Thm 3.3: M = ceil(log2(y_1 xi_1 N / eps)) + 1 (at least one interpolated level)
        hp.L = std::max(2, (int)std::ceil(std::log2(y1 * xi1 * (double)N / eps)) + 1);
        if (hp.L > 1000) return FLT_ERANGE;
        hp.q = lap_rank_general(y1, xi1, hp.L, eps, [](double x) { return lap_kernel_k12(x); });
        if (hp.q == 0) return FLT_EPRECISION;
    }
    if (hp.q > LAP_MAX_Q) return FLT_EPRECISION;
    const int q = hp.q;
    hp.L = std::max(hp.L, 1);
    if (hp.L > 1000) return FLT_ERANGE;
    const int L = hp.L;
    // frequencies grouped by block, caller order kept inside a block (a
    // counting sort): neighbouring lanes then gather nearby coefficients
    std::vector<int32_t> blk(N);
    std::vector<int64_t> first((size_t)L + 2, 0);
    for (int64_t k = 0; k < N; ++k) {
        blk[k] = lap_level(xi[k], xi1, L);
        first[blk[k] + 1]++;
    }
    for (int l = 1; l <= L + 1; ++l) first[l] += first[l - 1];
    std::vector<int32_t> ord(N);
    hp.near0 = first[L];   // Omega_L, the last block in the sorted order
    hp.nnear = N - first[L];
    for (int64_t k = 0; k < N; ++k) ord[first[blk[k]]++] = (int32_t)k;
    hp.xs.resize(N);
    hp.kperm.resize(N);
    for (int64_t i = 0; i < N; ++i) {
        hp.xs[i] = xi[ord[i]];
        hp.kperm[i] = ord[i];
    }
    for (int64_t i = 0; i < N;) {   // items: chunks of one block
        int64_t e = i;
        while (e < N && blk[ord[e]] == blk[ord[i]] && e - i < LAP_CHUNK) ++e;
        hp.items.push_back(LapItem{blk[ord[i]], (int32_t)(e - i), i});
        i = e;
    }
    if (hp.items.size() > (size_t)INT32_MAX / 2) return FLT_ERANGE;
    hp.bitem.assign((size_t)L + 1, 0);   // items of block l: bitem[l - 1] .. bitem[l] - 1
    for (const LapItem& it : hp.items) hp.bitem[it.blk]++;
    for (int l = 1; l <= L; ++l) hp.bitem[l] += hp.bitem[l - 1];
    // Chebyshev nodes, centres and inverse half-widths of the blocks l < L and
    // bands m < L (closures of the intervals)
    const size_t nl = (size_t)std::max(L - 1, 1);
    std::vector<double> bnodes(nl * q, 0.0), ynodes(nl * q, 0.0);
    hp.bcw.assign(2 * nl, 0.0);
    hp.ycw.assign(2 * (size_t)L, 0.0);   // band L: t = 0
    for (int l = 1; l < L; ++l) {
        const double a = std::ldexp(xi1, -l), b = std::ldexp(xi1, 1 - l);
        cheb_nodes(a, b, q, &bnodes[(size_t)(l - 1) * q]);
        hp.bcw[2 * (l - 1)] = 0.5 * (a + b);
        hp.bcw[2 * (l - 1) + 1] = 2.0 / (b - a);
    }
    for (int m = 1; m < L; ++m) {
        const double a = std::ldexp(y1, -m), b = std::ldexp(y1, 1 - m);
        cheb_nodes(a, b, q, &ynodes[(size_t)(m - 1) * q]);
        hp.ycw[2 * (m - 1)] = 0.5 * (a + b);
        hp.ycw[2 * (m - 1) + 1] = 2.0 / (b - a);
    }
    // C[p][r] = a_p T_p(tau_r) = a_p cos(p (2r+1) pi / (2q)), a_0 = 1/q, a_p = 2/q
    std::vector<double> C((size_t)q * q);
    for (int p = 0; p < q; ++p)
        for (int r = 0; r < q; ++r)
            C[(size_t)p * q + r] = (p ? 2.0 : 1.0) / q * std::cos(p * (2 * r + 1) * M_PI / (2.0 * q));
    // l_m, L_m (Def. 3.2; natural log inside l_m) and, per (m, l), C K C^T with
    // K^{Y_m,Omega_l}[s][r] = exp(-y_s xi_r)
    const double lg = L > 1 ? std::log2(y1 * xi1) - std::log2(std::log(1.0 / eps)) : 0.0;
    std::vector<double> K((size_t)q * q), KC((size_t)q * q);
    for (int m = 1; m < L; ++m) {
        // general kernels: every block l < L (the kernel is neither ~0 nor ~1 on any)
        const int lm = general ? 1 : std::max(1, (int)std::floor(lg - m) + 1);
        const int Lm = general ? L - 1 : L - m;
        hp.lm.push_back(lm);
        hp.Lm.push_back(Lm);
        hp.koff.push_back((int64_t)hp.K.size());
        for (int l = lm; l <= Lm; ++l) {
            for (int s = 0; s < q; ++s)
                for (int r = 0; r < q; ++r)
                {
                    const double yx = ynodes[(size_t)(m - 1) * q + s] * bnodes[(size_t)(l - 1) * q + r];
                    K[(size_t)s * q + r] = general ? lap_kernel_k12(yx) : std::exp(-yx);
                }
            for (int s = 0; s < q; ++s)   // KC = K C^T
                for (int p = 0; p < q; ++p) {
                    double a = 0.0;
                    for (int r = 0; r < q; ++r) a += K[(size_t)s * q + r] * C[(size_t)p * q + r];
                    KC[(size_t)s * q + p] = a;
                }
            for (int pp = 0; pp < q; ++pp)   // C KC
                for (int p = 0; p < q; ++p) {
                    double a = 0.0;
                    for (int s = 0; s < q; ++s) a += C[(size_t)pp * q + s] * KC[(size_t)s * q + p];
                    hp.K.push_back(a);
                }
        }
    }
    if (hp.lm.empty()) {   // keep every table non-empty
        hp.lm.push_back(1);
        hp.Lm.push_back(0);
        hp.koff.push_back(0);
    }
    if (hp.K.empty()) hp.K.push_back(0.0);
    hp.y.assign(y, y + M);
    hp.band.resize(M);
    for (int64_t j = 0; j < M; ++j) hp.band[j] = lap_level(y[j], y1, L);
    return FLT_OK;
}

}  // namespace flt
