// Host planner of the real-exponent transform (see xi_plan.h).
#include "xi_plan.h"

#include <math.h>

#include <algorithm>
#include <numeric>

#include "flt.h"

namespace flt {

static const double PI = 3.14159265358979323846;
// Smallest frequency density sigma a band is given: each band picks the
// smallest power-of-two frequency count its integer sum fits with sigma >=
// XI_SIG_MIN, sigma capped at 2; the window half-width is chosen for this
// worst case.
static const double XI_SIG_MIN = 1.9;

double kb_bound(int m, double sigma)
{
    const double s = sqrt(1.0 - 1.0 / sigma);
    return 4.0 * PI * (sqrt((double)m) + m) * sqrt(s) * exp(-2.0 * PI * m * s);
}

// ceil(log2 xi) for xi >= 1: the exponent of the dyadic block (2^(c-1), 2^c]
// that holds xi (the device computes it the same way).
static int ceil_log2_real(double xi)
{
    int e;
    const double f = frexp(xi, &e);   // xi = f 2^e, f in [1/2, 1)
    return f == 0.5 ? e - 1 : e;
}

int build_xi_plan(XiHost& hp, int64_t N, const double* xi, int64_t M, const double* z, double eps, int dtype)
{
    if (!xi || !z || N < 1 || M < 1 || (dtype != FLT_C64 && dtype != FLT_C128)) return FLT_EINVAL;
    if (!(eps > 0.0 && eps < 1.0)) return FLT_EDOMAIN;
    if (N > ((int64_t)1 << 30) || M > ((int64_t)1 << 31) - 1) return FLT_ERANGE;
    double xmax = 0.0;
    for (int64_t k = 0; k < N; ++k) {
        if (!(xi[k] >= 1.0) || !isfinite(xi[k])) return FLT_EDOMAIN;
        xmax = std::max(xmax, xi[k]);
    }
    if (xmax > ldexp(1.0, 29)) return FLT_ERANGE;
    hp = XiHost();
    hp.N = N;
    hp.M = M;
    hp.dtype = dtype;
    hp.eps = eps;

    // ---- the Laplace side: the integer plan's partition for exponents up to
    // ceil(max xi) (direct sums off: every band is an NFFT band)
    const int64_t Nint = (int64_t)ceil(xmax) + 1;
    int rc = build_host_plan(hp.outer, Nint, M, z, eps, dtype, FLT_FLAG_NFFT_ONLY);
    if (rc != FLT_OK) return rc;
    const HostPlan& op = hp.outer;

    // ---- exponents, ascending
    hp.xi_perm.resize(N);
    std::iota(hp.xi_perm.begin(), hp.xi_perm.end(), 0);
    std::stable_sort(hp.xi_perm.begin(), hp.xi_perm.end(), [&](int32_t a, int32_t b) { return xi[a] < xi[b]; });
    hp.xi.resize(N);
    for (int64_t k = 0; k < N; ++k) hp.xi[k] = xi[hp.xi_perm[k]];
    hp.xp.resize(M);
    for (int64_t j = 0; j < M; ++j) hp.xp[j] = op.nx[j] > 0.5 ? op.nx[j] - 1.0 : op.nx[j];

    // ---- Fourier side: eps/6 for the frequency window, eps/6 for the inner
    // integer sums after the window's amplification (Lemma 4.1 leaves eps/3
    // to the Fourier factor)
    hp.eps_w = eps / 6.0;
    hp.mw1 = 2;
    while (kb_bound(hp.mw1, XI_SIG_MIN) > hp.eps_w) ++hp.mw1;
    if (hp.mw1 > MAX_MW) return FLT_EPRECISION;
    const int m = hp.mw1;

    const int nb = (int)op.bands.size();
    hp.bands.resize(nb);
    hp.sig_min = 2.0;
    hp.amp = 1.0;
    int64_t cin = 0, hout = 0;
    for (int b = 0; b < nb; ++b) {
        const BandDesc& B = op.bands[b];
        XiBand& X = hp.bands[b];
        X = XiBand();
        X.node_start = B.node_start;
        X.node_count = B.node_count;
        if (B.q == 0) continue;
        // exponents in the band's support (e^{-xi y} < eps_K beyond it)
        const double xi_hi = (double)B.kmax;
        const int64_t k_end = std::upper_bound(hp.xi.begin(), hp.xi.end(), xi_hi) - hp.xi.begin();
        if (k_end == 0) continue;   // nothing reaches these nodes: f = 0 there
        X.q = B.q;
        X.ell_lo = B.ell_lo;
        X.ell_hi = B.ell_hi;
        X.n_xi = B.n_xi;
        X.coef_off = B.coef_off;
        X.ycheb_off = B.ycheb_off;
        X.k_end = k_end;
        const double lo = hp.xi[0], hi = hp.xi[k_end - 1], width = hi - lo;
        double sig = 2.0;
        if (width > 0.0) {
            int p = 1;
            while ((ldexp(1.0, p) - 2.0 * m - 2.0) / width < XI_SIG_MIN) ++p;
            sig = std::min(2.0, (ldexp(1.0, p) - 2.0 * m - 2.0) / width);
        }
        X.sig = sig;
        X.kb_b = PI * (2.0 - 1.0 / sig);
        // window taps of xi: the integers l with u = sigma xi - l in (-m, m]
        X.l_lo = (int64_t)ceil(sig * lo - m);
        const int64_t l_hi = (int64_t)ceil(sig * hi + m) - 1;
        X.l_count = l_hi - X.l_lo + 1;
        X.cin_off = cin;
        X.hout_off = hout;
        cin += (int64_t)X.q * X.l_count;
        hout += (int64_t)X.q * X.node_count;
        hp.sig_min = std::min(hp.sig_min, sig);
        const double bb = X.kb_b, w = PI / sig;   // |2 pi x / sigma| <= pi / sigma
        hp.amp = std::max(hp.amp, bessel_i0(m * bb) / bessel_i0(m * sqrt(bb * bb - w * w)));
        for (int s = 0; s < X.q; ++s) {
            hp.in_N.push_back(X.l_count);
            hp.in_M.push_back(X.node_count);
            for (int64_t j = 0; j < X.node_count; ++j) {
                hp.in_z.push_back(hp.xp[X.node_start + j] / sig);
                hp.in_z.push_back(0.0);
            }
        }
    }
    hp.cin_elems = cin;
    hp.hout_elems = hout;
    hp.eps_in = hp.eps_w / hp.amp;

    // ---- work items
    auto blocks_of = [&](const XiBand& X, int64_t k_lo, int64_t k_hi, XiItem& it) {
        it.blk_lo = 0;
        it.nblk = 0;
        if (k_lo >= k_hi || X.ell_hi < X.ell_lo) return;
        // ell = n_xi + 1 - ceil(log2 xi) decreases with xi
        const int e_hi = std::min(X.ell_hi, X.n_xi + 1 - ceil_log2_real(hp.xi[k_lo]));
        const int e_lo = std::max(X.ell_lo, X.n_xi + 1 - ceil_log2_real(hp.xi[k_hi - 1]));
        if (e_hi < e_lo) return;
        it.blk_lo = e_lo - X.ell_lo;
        it.nblk = e_hi - e_lo + 1 <= XI_NBLK ? e_hi - e_lo + 1 : -1;
    };
    for (int b = 0; b < nb; ++b) {
        const XiBand& X = hp.bands[b];
        for (int64_t s = 0; s < X.node_count; s += GATHER_THREADS)
            hp.nodes.push_back(NodeItem{b, (int32_t)std::min<int64_t>(GATHER_THREADS, X.node_count - s),
                                        X.node_start + s});
        if (X.q == 0) continue;
        for (int64_t li = 0; li < X.l_count; li += XI_THREADS) {
            XiItem it;
            it.band = b;
            it.count = (int32_t)std::min<int64_t>(XI_THREADS, X.l_count - li);
            it.first = li;
            const double l_first = (double)(X.l_lo + li), l_last = (double)(X.l_lo + li + it.count - 1);
            // exponents with sigma xi - l in (-m, m] for some l of the run
            it.k_lo = std::partition_point(hp.xi.begin(), hp.xi.begin() + X.k_end,
                                           [&](double v) { return !(X.sig * v - l_first > -m); }) -
                      hp.xi.begin();
            it.k_hi = std::partition_point(hp.xi.begin(), hp.xi.begin() + X.k_end,
                                           [&](double v) { return X.sig * v - l_last <= m; }) -
                      hp.xi.begin();
            blocks_of(X, it.k_lo, it.k_hi, it);
            hp.spread.push_back(it);
        }
        for (int64_t k0 = 0; k0 < X.k_end; k0 += XI_THREADS) {
            XiItem it;
            it.band = b;
            it.count = (int32_t)std::min<int64_t>(XI_THREADS, X.k_end - k0);
            it.first = k0;
            it.k_lo = k0;
            it.k_hi = k0 + it.count;
            blocks_of(X, it.k_lo, it.k_hi, it);
            hp.gather.push_back(it);
        }
    }
    return FLT_OK;
}

}  // namespace flt
