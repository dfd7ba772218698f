// Host planner for the fast Fourier-Laplace transform (Kunis & Melzer,
// Algorithm 2).  FP64 throughout; see plan_host.h.
#include "plan_host.h"

#include <math.h>

#include <algorithm>
#include <atomic>
#include <exception>
#include <map>
#include <numeric>
#include <system_error>
#include <thread>

#include "flt.h"

namespace flt {

static const double PI = 3.14159265358979323846264338327950288;

double bessel_i0(double x)
{
    // sum_j ((x/2)^2)^j / (j!)^2: all terms positive, no cancellation
    const double h = 0.25 * x * x;
    double t = 1.0, s = 1.0;
    for (int j = 1; j < 1000; ++j) {
        t *= h / ((double)j * (double)j);
        s += t;
        if (t < s * 1e-17) break;
    }
    return s;
}

// Kaiser-Bessel NFFT error bound relative to the coefficient 1-norm, oversampling 2
// (Potts & Steidl): 4 pi (sqrt(m) + m) (1 - 1/sigma)^(1/4) e^{-2 pi m sqrt(1 - 1/sigma)}.
static double kb_error_bound(int m)
{
    const double s = sqrt(0.5);
    return 4.0 * PI * (sqrt((double)m) + m) * sqrt(s) * exp(-2.0 * PI * m * s);
}

static int log2_exact(int64_t v)
{
    int r = 0;
    while (((int64_t)1 << r) < v) ++r;
    return r;
}

// Direct-sum policy: a band whose grids cost more HBM time than summing its
// nodes directly is evaluated exactly (nodes x N terms) instead of by NFFT.
static const double POLICY_HBM_BYTES_PER_S = 4.0e12;
static const double POLICY_TERMS_PER_S_C64 = 2.0e12;
static const double POLICY_TERMS_PER_S_C128 = 1.5e12;

// One instance, everything but the launch groups and the workspace layout.
static int build_one(HostPlan& hp, int64_t N, int64_t M, const double* z, double eps, int dtype, uint32_t flags,
                     PlanShape shape)
{
    const double direct_scale = shape.direct_scale;
    if (!z || N < 1 || M < 1 || (dtype != FLT_C64 && dtype != FLT_C128)) return FLT_EINVAL;
    if (!(eps > 0.0 && eps < 1.0)) return FLT_EDOMAIN;
    if (!(flags & PLAN_FLAG_NO_FLOOR) && eps < (dtype == FLT_C64 ? 1e-6 : 1e-14)) return FLT_EPRECISION;
    if (N - 1 > ((int64_t)1 << 21)) return FLT_ERANGE;
    if (M > (int64_t)INT32_MAX) return FLT_ERANGE;
    for (int64_t j = 0; j < M; ++j) {
        const double re = z[2 * j], im = z[2 * j + 1];
        if (!isfinite(re) || isnan(im) || im < 0.0) return FLT_EDOMAIN;
    }

    hp = HostPlan();
    hp.flags = flags;
    hp.direct_scale = direct_scale;
    hp.N = N;
    hp.M = M;
    hp.dtype = dtype;
    hp.eps = eps;
    // Lemma 4.1: split the target between the Laplace and Fourier factors
    hp.eps_K = eps / 3.0;
    hp.eps_A = eps / 3.0;
    // Def. 3.2 / Alg. 2 with y_1 = ln(1/eps_K) and xi_1 = 2^n_xi >= N - 1
    hp.q = (int)ceil(0.5 + log(1.0 / hp.eps_K) / log(4.0));
    if (hp.q > MAX_Q) return FLT_EPRECISION;
    hp.y1 = log(1.0 / hp.eps_K);
    hp.n_xi = log2_exact(std::max<int64_t>(N - 1, 1));
    const double xi1 = ldexp(1.0, hp.n_xi);
    hp.D = (int)ceil(log2(hp.y1 * xi1 / hp.eps_K)) + 1;
    hp.mw = 2;
    while (kb_error_bound(hp.mw) > hp.eps_A) ++hp.mw;
    if (hp.mw > MAX_MW) return FLT_EPRECISION;
    hp.kb_b = PI * (2.0 - 1.0 / 2.0);
    const int q = hp.q, D = hp.D;

    // ---- node partition: Z^0 (y > y_1), Y_m = (y_1 2^-m, y_1 2^(1-m)], Y_D = [0, y_1 2^(1-D)]
    std::vector<double> xs(M), ys(M);
    hp.node_band.resize(M);
    std::vector<int64_t> count(D + 1, 0);
    for (int64_t j = 0; j < M; ++j) {
        const double re = z[2 * j], im = z[2 * j + 1];
        double x = re - floor(re);
        if (x >= 1.0) x = 0.0;
        const double y = isinf(im) ? INFINITY : 2.0 * PI * im;
        xs[j] = x;
        ys[j] = y;
        int m;
        if (y > hp.y1) m = 0;
        else if (y == 0.0) m = D;
        else {
            m = (int)floor(log2(hp.y1 / y)) + 1;
            m = std::min(std::max(m, 1), D);
            while (m < D && !(y > ldexp(hp.y1, -m))) ++m;
            while (m > 1 && y > ldexp(hp.y1, 1 - m)) --m;
        }
        hp.node_band[j] = m;
        count[m]++;
    }
    hp.nodes_z0 = count[0];

    // ---- bands
    const int LOG2P = dtype == FLT_C64 ? Sizes<float>::LOG2P : Sizes<double>::LOG2P;
    std::vector<int> band_of_m(D + 1, -1);
    int64_t n_const = count[0];
    for (int m = 1; m <= D; ++m) {
        if (count[m] == 0) continue;
        if (N == 1) { n_const += count[m]; continue; }      // only c_0: every node is constant
        BandDesc B{};
        const int64_t K = (int64_t)1 << (m < D ? std::min(m, hp.n_xi) : hp.n_xi);
        B.q = m < D ? q : 1;
        B.ell_lo = m < D ? std::max(1, hp.n_xi - m + 1) : 1;
        B.ell_hi = m < D ? D - m : 0;
        B.n_xi = hp.n_xi;
        B.kmax = std::min<int64_t>(K, N - 1);
        B.k0 = K / 2;
        B.log2n = std::max(log2_exact(2 * K), std::max(4, log2_exact(2 * hp.mw)));
        if (B.log2n <= LOG2P) {
            B.log2n1 = B.log2n;
            B.log2n2 = B.log2b = B.log2B = 0;
        } else {
            B.log2n1 = (B.log2n + 1) / 2;
            B.log2n2 = B.log2n - B.log2n1;
            B.log2b = LOG2P - B.log2n1;     // a full LDS tile of sub-transforms per workgroup
            B.log2B = LOG2P - B.log2n2;
            if (B.log2b > B.log2n2 || B.log2B > B.log2n1) return FLT_ERANGE;
        }
        band_of_m[m] = (int)hp.bands.size();
        hp.bands.push_back(B);
        hp.band_m.push_back(m);
    }
    int const_band = -1;
    if (n_const > 0) {
        BandDesc B{};
        B.q = 0;
        const_band = (int)hp.bands.size();
        hp.bands.push_back(B);
        hp.band_m.push_back(0);
    }
    const int nb = (int)hp.bands.size();
    // one column's coefficients of every block of a band are staged in LDS,
    // q padded to whole 16-byte vectors; a band has at most D - n_xi blocks
    {
        const int cv = dtype == FLT_C64 ? 4 : 2;
        const int qp = (q + cv - 1) / cv * cv;
        if ((int64_t)(D - hp.n_xi) * qp > (dtype == FLT_C64 ? Sizes<float>::COEF : Sizes<double>::COEF))
            return FLT_EPRECISION;
    }

    // ---- per-band choice: NFFT (Alg. 2) or the exact direct sum for sparsely filled bands
    {
        const double S = dtype == FLT_C64 ? 8.0 : 16.0;
        // direct_scale: factor on the assumed direct-sum rate (a tuned plan's
        // choice among candidates; 0 keeps every band on the NFFT path)
        const double rate = (dtype == FLT_C64 ? POLICY_TERMS_PER_S_C64 : POLICY_TERMS_PER_S_C128) * direct_scale;
        for (int b = 0; b < nb; ++b) {
            BandDesc& B = hp.bands[b];
            if (B.q == 0 || (flags & FLT_FLAG_NFFT_ONLY) || !(direct_scale > 0.0)) continue;
            const double n = ldexp(1.0, B.log2n);
            const double passes = B.log2n > LOG2P ? 4.0 : 2.0;
            const double t_nfft = (passes * B.q * n * S + (double)B.kmax * S) / POLICY_HBM_BYTES_PER_S;
            const double t_direct = (double)count[hp.band_m[b]] * (double)N / rate;
            B.direct = t_direct < t_nfft ? 1 : 0;
        }
    }

    // ---- sort nodes by (band, grid cell)
    std::vector<int> nb_of(M);
    std::vector<int64_t> cell(M);
    for (int64_t j = 0; j < M; ++j) {
        const int m = hp.node_band[j];
        const int b = (m == 0 || band_of_m[m] < 0) ? const_band : band_of_m[m];
        nb_of[j] = b;
        cell[j] = hp.bands[b].q ? (int64_t)floor(ldexp(xs[j], hp.bands[b].log2n)) : 0;
    }
    std::vector<int32_t> idx(M);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
        if (nb_of[a] != nb_of[b]) return nb_of[a] < nb_of[b];
        return cell[a] < cell[b];
    });
    hp.perm = idx;
    hp.nx.resize(M);
    hp.ny.resize(M);
    for (int64_t i = 0; i < M; ++i) {
        hp.nx[i] = xs[idx[i]];
        hp.ny[i] = ys[idx[i]];
    }
    {
        int64_t pos = 0;
        for (int b = 0; b < nb; ++b) {
            int64_t cnt = 0;
            while (pos + cnt < M && nb_of[idx[pos + cnt]] == b) ++cnt;
            hp.bands[b].node_start = pos;
            hp.bands[b].node_count = cnt;
            pos += cnt;
        }
    }

    // ---- tables
    std::vector<double> t(q), lam(q), theta(q);
    for (int s = 0; s < q; ++s) {
        theta[s] = (2.0 * s + 1.0) * PI / (2.0 * q);
        t[s] = cos(theta[s]);                                   // Sect. 2: zeros of T_q
        lam[s] = ((s & 1) ? -1.0 : 1.0) * sin(theta[s]);        // barycentric weights
    }
    // Chebyshev coefficients of xi -> sum_r K[s,r] L_r^{Omega_l}(xi) (Lemma A.1 with
    // the barycentric L_r of Sect. 2 written in the Chebyshev basis).  The block
    // (Omega_l, Y_m) is the pair (2^d (1,2], y_1 (1,2]) scaled by powers of two,
    // d = n_xi - l - m, and e^{-y x} depends only on the product, so one table
    // over d = -1, -2, ..., n_xi - D serves every band (a band's blocks
    // l_lo..l_hi are consecutive entries), a[d][s][i].
    for (int d = -1; d >= hp.n_xi - D; --d) {
        const double xlo = ldexp(1.0, d), xhi = ldexp(1.0, d + 1);
        const double ylo = hp.y1, yhi = 2.0 * hp.y1;
        for (int s = 0; s < q; ++s) {
            const double ysn = 0.5 * (ylo + yhi) + 0.5 * (yhi - ylo) * t[s];
            for (int i = 0; i < q; ++i) {
                double a = 0.0;
                for (int r = 0; r < q; ++r) {
                    const double xr = 0.5 * (xlo + xhi) + 0.5 * (xhi - xlo) * t[r];
                    a += exp(-ysn * xr) * cos(i * theta[r]);   // K[s,r] T_i(t_r)
                }
                hp.coef.push_back(a * (i == 0 ? 1.0 : 2.0) / q);
            }
        }
    }
    std::map<int, int> deconv_of;
    for (int b = 0; b < nb; ++b) {
        BandDesc& B = hp.bands[b];
        const int m = hp.band_m[b];
        if (B.q == 0 || B.direct) continue;
        // y interpolation nodes (Y_m) and weights
        B.ycheb_off = (int32_t)(hp.ycheb.size() / 2);
        if (m < D) {
            const double lo = ldexp(hp.y1, -m), hi = ldexp(hp.y1, 1 - m);
            for (int s = 0; s < q; ++s) {
                hp.ycheb.push_back(0.5 * (lo + hi) + 0.5 * (hi - lo) * t[s]);
                hp.ycheb.push_back(lam[s]);
            }
        } else {
            hp.ycheb.push_back(0.5 * ldexp(hp.y1, 1 - D));
            hp.ycheb.push_back(1.0);
        }
        B.coef_off = m < D ? (int32_t)((-1 - (hp.n_xi - B.ell_lo - m)) * q * q) : 0;
        // deconvolution 1 / (n phi_hat(k')) = 1 / I_0(mw sqrt(b^2 - (2 pi k'/n)^2)), |k'| <= n/4
        auto it = deconv_of.find(B.log2n);
        if (it == deconv_of.end()) {
            const int off = (int)hp.deconv.size();
            const int64_t n = (int64_t)1 << B.log2n;
            for (int64_t kp = 0; kp <= n / 4; ++kp) {
                const double w = 2.0 * PI * (double)kp / (double)n;
                hp.deconv.push_back(1.0 / bessel_i0(hp.mw * sqrt(hp.kb_b * hp.kb_b - w * w)));
            }
            it = deconv_of.emplace(B.log2n, off).first;
        }
        B.deconv_off = it->second;
    }
    const int TWN = 1 << TW_STAGE_LOG2;
    hp.tw_stage.resize(2 * TWN);
    for (int i = 0; i < TWN; ++i) {
        const double a = 2.0 * PI * (double)i / TWN;
        hp.tw_stage[2 * i] = cos(a);
        hp.tw_stage[2 * i + 1] = -sin(a);
    }
    const int H = 1 << TW2_HALF;
    hp.tw_lo.resize(2 * H);
    hp.tw_hi.resize(2 * H);
    for (int i = 0; i < H; ++i) {
        const double a = 2.0 * PI * (double)i / ldexp(1.0, TW2_LOG2);
        const double bb = 2.0 * PI * (double)i / ldexp(1.0, TW2_LOG2 - TW2_HALF);
        hp.tw_lo[2 * i] = cos(a);
        hp.tw_lo[2 * i + 1] = -sin(a);
        hp.tw_hi[2 * i] = cos(bb);
        hp.tw_hi[2 * i + 1] = -sin(bb);
    }

    // ---- workspace layout and work lists
    int64_t goff = 0, soff = 0, boff = 0;
    for (int b = 0; b < nb; ++b) {
        BandDesc& B = hp.bands[b];
        if (B.q == 0 || B.direct) continue;
        const int64_t n = (int64_t)1 << B.log2n;
        B.grid_off = goff;
        goff += (int64_t)B.q * n;
        // cell-start table: first sorted node with cell >= c, c = 0..n
        B.cs_off = (int64_t)hp.cstart.size();
        {
            int64_t jn = B.node_start;
            const int64_t end = B.node_start + B.node_count;
            for (int64_t cc = 0; cc <= n; ++cc) {
                while (jn < end && cell[idx[jn]] < cc) ++jn;
                hp.cstart.push_back((int32_t)jn);
            }
        }
        // cells some node's window reads: [l0 - mw + 1, l0 + mw] (mod n) around
        // each node's cell l0 = floor(n x); a two-pass band keeps them as a bit
        // mask over grid addresses, so pass B stores (and, for the adjoint,
        // loads) only those cells
        {
            std::vector<uint8_t> hit((size_t)n, 0);
            for (int64_t j = B.node_start; j < B.node_start + B.node_count; ++j)
                for (int t = 0; t < 2 * hp.mw; ++t) hit[(size_t)((cell[idx[j]] - hp.mw + 1 + t) & (n - 1))] = 1;
            B.cells = 0;
            for (int64_t l = 0; l < n; ++l) B.cells += hit[(size_t)l];
            if (B.log2n2 > 0) {
                B.mask_off = (int64_t)hp.mask.size();
                hp.mask.resize(hp.mask.size() + (size_t)(n >> 5), 0u);
                uint32_t* mk = hp.mask.data() + B.mask_off;
                for (int64_t l = 0; l < n; ++l)
                    if (hit[(size_t)l]) {
                        const int64_t a = grid_addr(B, l);
                        mk[a >> 5] |= 1u << (a & 31);
                    }
            }
            // adjoint grid side: groups of 2^lt threads per cell, sized so that a
            // thread handles about CELL_TARGET of a cell's contributions.  A
            // one-pass band gets every cell (its adjoint FFT reads whole columns);
            // a two-pass band whose windows leave cells untouched gets only the
            // touched ones, listed in clist (pass B loads only those)
            const bool listed = B.log2n2 > 0 && B.cells < n;
            const double span = listed ? (double)B.cells : (double)n;
            const double contrib = 2.0 * hp.mw * (double)B.node_count / span;
            int lt = 0;
            while (lt < 8 && (double)(1 << lt) * CELL_TARGET < contrib) ++lt;
            const int per = GATHER_THREADS >> lt;
            if (listed) {
                const int64_t first = (int64_t)hp.clist.size();
                for (int64_t l = 0; l < n; ++l)
                    if (hit[(size_t)l]) hp.clist.push_back((int32_t)l);
                while ((hp.clist.size() - (size_t)first) % (size_t)per) hp.clist.push_back(-1);
                for (int64_t c0 = first; c0 < (int64_t)hp.clist.size(); c0 += per)
                    hp.cells.push_back(CellItem{b, (int32_t)c0, lt, 1});
            } else {
                for (int64_t c0 = 0; c0 < n; c0 += per) hp.cells.push_back(CellItem{b, (int32_t)c0, lt, 0});
            }
        }
        if (B.log2n2 > 0) {
            B.scratch_off = soff;
            soff += (int64_t)B.q * n;
            if (dtype == FLT_C128) {   // the FP64 pass A keeps its bases in the workspace
                B.base_off = boff;
                boff += n;
            }
            const int nA = 1 << (B.log2n2 - B.log2b), nB = 1 << (B.log2n1 - B.log2B);
            for (int k = 0; k < nA; ++k) hp.passA_fwd.push_back(FftItem{b, 0, B.q, k});
            for (int s = 0; s < B.q; ++s)
                for (int k = 0; k < nB; ++k) hp.passB.push_back(FftItem{b, s, 1, k});
            for (int s = 0; s < 2 * B.q; ++s)
                for (int k = 0; k < nB; ++k) hp.passB_fused.push_back(FftItem{b, s, 1, k});
            for (int k = 0; k < nA; ++k) hp.passA_adj.push_back(FftItem{b, 0, B.q, k});
        } else {
            const int ns = std::max(1, std::min(B.q, std::min(MAX_Q, 1 << (LOG2P - B.log2n))));
            for (int s0 = 0; s0 < B.q; s0 += ns) {
                hp.onepass_fwd.push_back(FftItem{b, s0, std::min(ns, B.q - s0), 0});
                hp.onepass_adj.push_back(FftItem{b, s0, std::min(ns, B.q - s0), 0});
            }
            const int ns2 = std::max(1, std::min(2 * B.q, std::min(MAX_Q, 1 << (LOG2P - B.log2n))));
            for (int s0 = 0; s0 < 2 * B.q; s0 += ns2)
                hp.onepass_fused.push_back(FftItem{b, s0, std::min(ns2, 2 * B.q - s0), 0});
        }
        hp.qs = std::max(hp.qs, B.q);
    }
    for (int b = 0; b < nb; ++b) {
        const BandDesc& B = hp.bands[b];
        if (B.direct) {
            for (int64_t s = 0; s < B.node_count; ++s) hp.dlist.push_back((int32_t)(B.node_start + s));
            continue;
        }
        for (int64_t s = 0; s < B.node_count; s += GATHER_THREADS) {
            const NodeItem it{b, (int32_t)std::min<int64_t>(GATHER_THREADS, B.node_count - s), B.node_start + s};
            if (B.q > 0) hp.nfft_nodes.push_back(it);
            // the cells the item's windows read, as the gather computes them
            // (first and last sorted node)
            const int64_t lf = (int64_t)floor(ldexp(hp.nx[it.start], B.log2n));
            const int64_t ll = (int64_t)floor(ldexp(hp.nx[it.start + it.count - 1], B.log2n));
            if (B.q > 0 && ll - lf + 2 * hp.mw <= GATHER_STAGE) hp.gather_st.push_back(it);
            else hp.gather_ln.push_back(it);
        }
    }
    if (!hp.dlist.empty()) {
        const int64_t nd = (int64_t)hp.dlist.size();
        const int64_t fchunks = (N + (int64_t)256 * DIRECT_TPT - 1) / ((int64_t)256 * DIRECT_TPT);
        const int cpw = direct_cpw(dtype == FLT_C64 ? 4 : 8);
        // short sums (fewer 32-term pieces than threads): a workgroup splits into
        // groups of 2^lt threads, one per piece, each group with its own nodes
        const int64_t pieces = (N + DIRECT_TPT - 1) / DIRECT_TPT;
        int lt = 3;   // at least 8 threads per group: at most 256 / 8 = DIRECT_GMAX groups
        while (lt < 8 && ((int64_t)1 << lt) < pieces) ++lt;
        if (lt < 8) {
            const int64_t ng = 256 >> lt;
            const int64_t per = DIRECT_NG * ng;
            for (int64_t g = 0; g < nd; g += per)
                hp.direct_short.push_back(DirectItem{(int32_t)g, (int16_t)std::min<int64_t>(per, nd - g), 1, 0, 0, lt});
        } else {
            for (int64_t g = 0; g < nd; g += DIRECT_NG)
                for (int64_t ch = 0; ch < fchunks; ch += cpw)
                    hp.direct_fwd.push_back(DirectItem{(int32_t)g, (int16_t)std::min<int64_t>(DIRECT_NG, nd - g),
                                                       (int16_t)std::min<int64_t>(cpw, fchunks - ch), (int32_t)ch,
                                                       0, 8});
        }
        const int64_t aspan = (int64_t)256 * direct_atpt(dtype == FLT_C64 ? 4 : 8);   // adjoint workgroup
        const int64_t achunks = (N + aspan - 1) / aspan;
        for (int64_t g = 0; g < nd; g += DIRECT_ANG)
            for (int64_t ch = 0; ch < achunks; ++ch)
                hp.direct_adj.push_back(DirectItem{(int32_t)g, (int16_t)std::min<int64_t>(DIRECT_ANG, nd - g), 1,
                                                   (int32_t)ch, 0, 8});
    }
    hp.grid_elems = goff;
    hp.scratch_elems = soff;
    hp.base_elems = boff;
    hp.inst.push_back(InstDesc{0, N, 0, M});
    for (int64_t s0 = 0; s0 < M; s0 += (int64_t)256 * SUMG_PER_THREAD) hp.sum_items.push_back(SumItem{0, 0, s0});
    const size_t S = hp.elem_bytes();

    // ---- algorithmic model of one forward: c read once per band; a one-pass
    // band's grid written once; a two-pass band's pass-A output written and
    // read once, its grid written only at the cells the windows read; the
    // gather reads those cells (at most 2 mw per node and column); node
    // records and results once
    double bytes = (double)M * (16.0 + 4.0 + S);
    double flops = 0;
    for (int b = 0; b < nb; ++b) {
        const BandDesc& B = hp.bands[b];
        if (B.q == 0) continue;
        if (B.direct) {                                       // c read once per node group
            bytes += (double)N * S * (double)((B.node_count + DIRECT_NG - 1) / DIRECT_NG);
            flops += 16.0 * (double)N * (double)B.node_count;
            continue;
        }
        const double n = ldexp(1.0, B.log2n);
        const double cells = std::min((double)B.cells, (double)B.node_count * 2 * hp.mw);
        bytes += (double)B.kmax * S + B.q * cells * S;
        bytes += (B.log2n2 > 0 ? 2.0 * B.q * n + B.q * (double)B.cells : B.q * n) * S;
        flops += 2.0 * B.q * B.q * (double)B.kmax + 8.0 * B.q * (double)B.kmax;   // contraction, scaling
        flops += 5.0 * B.q * n * B.log2n;                                          // FFT
        flops += (double)B.node_count * (8.0 * B.q * 2 * hp.mw + 4.0 * B.q);       // gather, weighting
    }
    hp.bytes_forward = bytes;
    hp.flops_forward = flops;
    return FLT_OK;
}

// Workgroups are handed to the 8 XCDs of the GPU in turn (launch slot i on XCD
// i mod 8), each XCD with an L2 of its own.  Neighbouring pass-A items of a
// band (consecutive j2 blocks) share the cache lines of c (and, adjoint, of the
// accumulator) when a block holds fewer j2 than a 128-byte line holds
// elements: g = 128 / (b S) items per line.  Within every run of 8 g slots of
// one band, slot i takes item x g + i / 8 (x = i mod 8), so that the g items
// sharing lines run on one XCD.
static constexpr int NUM_XCD = 8;
static void xcd_order(const HostPlan& hp, std::vector<FftItem>& v)
{
    const int S = (int)hp.elem_bytes();
    std::vector<FftItem> out(v);
    size_t i = 0;
    while (i < v.size()) {
        const BandDesc& B = hp.bands[v[i].band];
        const int g = std::max(1, 128 / (S << B.log2b));
        const size_t run = (size_t)NUM_XCD * g;
        bool same = g > 1 && i + run <= v.size() && i % NUM_XCD == 0;
        for (size_t u = 1; same && u < run; ++u) same = v[i + u].band == v[i].band && v[i + u].blk == v[i].blk + (int)u;
        if (!same) {
            ++i;
            continue;
        }
        for (size_t u = 0; u < run; ++u) out[i + u] = v[i + (u % NUM_XCD) * g + u / NUM_XCD];
        i += run;
    }
    v.swap(out);
}

// Launch groups (FFT lists sorted by transform length, one compile-time kernel
// instance per length) and the workspace layout.
static void finish(HostPlan& hp)
{
    auto group = [&](std::vector<FftItem>& v, std::vector<LaunchGroup>& g, int which) {
        auto len = [&](const FftItem& it) {
            const BandDesc& B = hp.bands[it.band];
            return which == 0 ? B.log2n : (which == 1 ? B.log2n1 : B.log2n2);
        };
        std::stable_sort(v.begin(), v.end(), [&](const FftItem& a, const FftItem& b) { return len(a) < len(b); });
        g.clear();
        for (size_t i = 0; i < v.size(); ++i) {
            if (g.empty() || g.back().log2 != len(v[i])) g.push_back(LaunchGroup{len(v[i]), (int32_t)i, 0, 0});
            g.back().count++;
        }
    };
    group(hp.onepass_fwd, hp.g_onepass_fwd, 0);
    group(hp.onepass_adj, hp.g_onepass_adj, 0);
    group(hp.passA_fwd, hp.g_passA_fwd, 0);   // pass A instances are per grid length
    group(hp.passA_adj, hp.g_passA_adj, 0);
    xcd_order(hp, hp.passA_fwd);
    xcd_order(hp, hp.passA_adj);
    group(hp.passB, hp.g_passB, 2);
    group(hp.onepass_fused, hp.g_onepass_fused, 0);
    group(hp.passB_fused, hp.g_passB_fused, 2);
    if (hp.cstart.empty()) hp.cstart.push_back(0);
    if (hp.clist.empty()) hp.clist.push_back(-1);
    if (hp.mask.empty()) hp.mask.push_back(0u);
    if (hp.coef.empty()) hp.coef.push_back(0.0);
    if (hp.deconv.empty()) hp.deconv.push_back(0.0);
    if (hp.ycheb.empty()) { hp.ycheb.push_back(0.0); hp.ycheb.push_back(0.0); }
    const size_t S = hp.elem_bytes();
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    hp.off_grid = 0;
    // grids and pass-A output for 2q columns per band: the size the fused
    // forward + derivative call needs (the other calls use the first halves)
    hp.off_scratch = al(hp.off_grid + (size_t)hp.grid_elems * 2 * S);
    hp.off_acc = al(hp.off_scratch + (size_t)hp.scratch_elems * 2 * S);
    hp.qs = (hp.qs + 1) & ~1;   // even: the adjoint moves column values in pairs
    hp.off_U = al(hp.off_acc + (size_t)hp.N * 16);
    hp.off_phi = al(hp.off_U + (size_t)hp.M * hp.qs * S);
    hp.off_l0 = al(hp.off_phi + (size_t)hp.M * 2 * hp.mw * (S / 2));
    hp.off_dacc = al(hp.off_l0 + (size_t)hp.M * 4);
    hp.off_base = al(hp.off_dacc + (size_t)hp.M * 16);
    hp.ws_bytes = al(hp.off_base + (size_t)hp.base_elems * S);
    hp.fwd_off_scratch = al((size_t)hp.grid_elems * S);
    hp.fwd_off_dacc = al(hp.fwd_off_scratch + (size_t)hp.scratch_elems * S);
    hp.fwd_off_base = al(hp.fwd_off_dacc + (size_t)hp.M * 16);
    hp.fwd_ws_bytes = al(hp.fwd_off_base + (size_t)hp.base_elems * S);
}

int build_host_plan(HostPlan& hp, int64_t N, int64_t M, const double* z, double eps, int dtype, uint32_t flags,
                    PlanShape shape)
{
    const int rc = build_one(hp, N, M, z, eps, dtype, flags, shape);
    if (rc != FLT_OK) return rc;
    finish(hp);
    return FLT_OK;
}

int build_batch_plan(HostPlan& out, int32_t count, const int64_t* N, const int64_t* M, const double* z, double eps,
                     int dtype, uint32_t flags, PlanShape shape)
{
    if (count < 1 || !N || !M || !z) return FLT_EINVAL;
    out = HostPlan();
    std::vector<int64_t> zoff(count, 0);          // first node of each member in z
    for (int32_t i = 1; i < count; ++i) zoff[i] = zoff[i - 1] + M[i - 1];
    std::map<int, int> deconv_at;                 // log2 n -> offset in the merged deconvolution table
    std::map<int, int> ycheb_at;                  // m (or -D for Y_D) -> pair offset in the merged ycheb table
    // The members are independent: they are planned on several host threads,
    // CHUNK at a time (bounding the memory held at once), and merged in order.
    const int32_t CHUNK = 64;
    const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    for (int32_t c0 = 0; c0 < count; c0 += CHUNK) {
        const int32_t c1 = std::min(count, c0 + CHUNK);
        std::vector<HostPlan> members(c1 - c0);
        std::vector<int> rcs(c1 - c0, FLT_OK);
        std::atomic<int32_t> next(c0);
        auto work = [&]() {
            for (int32_t i = next.fetch_add(1); i < c1; i = next.fetch_add(1)) {
                try {
                    rcs[i - c0] = build_one(members[i - c0], N[i], M[i], z + 2 * zoff[i], eps, dtype, flags, shape);
                } catch (const std::exception&) {   // allocation failures (no exception may leave a thread)
                    rcs[i - c0] = FLT_ENOMEM;
                }
            }
        };
        std::vector<std::thread> pool;
        try {
            for (int t = 1; t < std::min(nth, (int)(c1 - c0)); ++t) pool.emplace_back(work);
        } catch (const std::system_error&) {   // fewer threads: the calling one does the rest
        }
        work();
        for (std::thread& t : pool) t.join();
        for (int32_t i = c0; i < c1; ++i) {
            if (rcs[i - c0] != FLT_OK) return rcs[i - c0];
            HostPlan p = std::move(members[i - c0]);
            if (i == 0) {
                out.dtype = p.dtype;
                out.eps = p.eps;
                out.eps_K = p.eps_K;
                out.eps_A = p.eps_A;
                out.y1 = p.y1;
                out.q = p.q;
                out.mw = p.mw;
                out.kb_b = p.kb_b;
                out.flags = p.flags;
                out.direct_scale = p.direct_scale;
                out.tw_stage = p.tw_stage;
                out.tw_lo = p.tw_lo;
                out.tw_hi = p.tw_hi;
            }
            // the coefficient table depends on q, y_1 and D - n_xi only (see build_one):
            // share it, appending when a member's table differs (never for one eps)
            int32_t coef_shift = 0;
            if (out.coef.empty()) out.coef = p.coef;
            else if (p.coef.size() > out.coef.size() ||
                     !std::equal(p.coef.begin(), p.coef.end(), out.coef.begin())) {
                coef_shift = (int32_t)out.coef.size();
                out.coef.insert(out.coef.end(), p.coef.begin(), p.coef.end());
            }
            const int32_t bo = (int32_t)out.bands.size();
            const int64_t no = out.M;                    // sorted-node (and caller-index) offset
            const int64_t co = out.N;                    // coefficient offset
            const int64_t dlo = (int64_t)out.dlist.size();
            const int64_t cso = (int64_t)out.cstart.size(), mko = (int64_t)out.mask.size();
            for (size_t b = 0; b < p.bands.size(); ++b) {
                BandDesc B = p.bands[b];
                const int m = p.band_m[b];
                B.c_off = co;
                B.node_start += no;
                if (B.q > 0 && !B.direct) {
                    B.coef_off += coef_shift;
                    B.grid_off += out.grid_elems;
                    B.scratch_off += out.scratch_elems;
                    B.cs_off += cso;
                    B.mask_off += mko;
                    B.base_off += out.base_elems;
                    auto dt = deconv_at.find(B.log2n);
                    if (dt == deconv_at.end()) {
                        const int64_t len = ((int64_t)1 << B.log2n) / 4 + 1;
                        dt = deconv_at.emplace(B.log2n, (int)out.deconv.size()).first;
                        out.deconv.insert(out.deconv.end(), p.deconv.begin() + B.deconv_off,
                                          p.deconv.begin() + B.deconv_off + len);
                    }
                    B.deconv_off = dt->second;
                    const int key = m < p.D ? m : -p.D;
                    auto yt = ycheb_at.find(key);
                    if (yt == ycheb_at.end()) {
                        yt = ycheb_at.emplace(key, (int)(out.ycheb.size() / 2)).first;
                        out.ycheb.insert(out.ycheb.end(), p.ycheb.begin() + 2 * B.ycheb_off,
                                         p.ycheb.begin() + 2 * (B.ycheb_off + B.q));
                    }
                    B.ycheb_off = yt->second;
                }
                out.bands.push_back(B);
                out.band_m.push_back(m);
            }
            out.node_band.insert(out.node_band.end(), p.node_band.begin(), p.node_band.end());
            out.nx.insert(out.nx.end(), p.nx.begin(), p.nx.end());
            out.ny.insert(out.ny.end(), p.ny.begin(), p.ny.end());
            for (int32_t v : p.perm) out.perm.push_back((int32_t)(v + no));
            auto shift_fft = [&](std::vector<FftItem>& dst, const std::vector<FftItem>& src) {
                for (FftItem it : src) { it.band += bo; dst.push_back(it); }
            };
            shift_fft(out.onepass_fwd, p.onepass_fwd);
            shift_fft(out.passA_fwd, p.passA_fwd);
            shift_fft(out.passB, p.passB);
            shift_fft(out.onepass_adj, p.onepass_adj);
            shift_fft(out.passA_adj, p.passA_adj);
            shift_fft(out.onepass_fused, p.onepass_fused);
            shift_fft(out.passB_fused, p.passB_fused);
            const int32_t clo = (int32_t)out.clist.size();
            for (CellItem it : p.cells) {
                it.band += bo;
                if (it.listed) it.cell0 += clo;
                out.cells.push_back(it);
            }
            out.clist.insert(out.clist.end(), p.clist.begin(), p.clist.end());
            auto shift_nodes = [&](std::vector<NodeItem>& dst, const std::vector<NodeItem>& src) {
                for (NodeItem it : src) { it.band += bo; it.start += no; dst.push_back(it); }
            };
            shift_nodes(out.gather_st, p.gather_st);
            shift_nodes(out.gather_ln, p.gather_ln);
            shift_nodes(out.nfft_nodes, p.nfft_nodes);
            for (int32_t v : p.dlist) out.dlist.push_back((int32_t)(v + no));
            for (DirectItem it : p.direct_fwd) { it.first += (int32_t)dlo; it.inst = i; out.direct_fwd.push_back(it); }
            for (DirectItem it : p.direct_short) { it.first += (int32_t)dlo; it.inst = i; out.direct_short.push_back(it); }
            for (DirectItem it : p.direct_adj) { it.first += (int32_t)dlo; it.inst = i; out.direct_adj.push_back(it); }
            for (int32_t v : p.cstart) out.cstart.push_back((int32_t)(v + no));
            out.mask.insert(out.mask.end(), p.mask.begin(), p.mask.end());
            out.inst.push_back(InstDesc{co, p.N, no, p.M});
            for (SumItem it : p.sum_items) { it.inst = i; it.start += no; out.sum_items.push_back(it); }
            out.qs = std::max(out.qs, p.qs);
            out.D = std::max(out.D, p.D);
            out.n_xi = std::max(out.n_xi, p.n_xi);
            out.nodes_z0 += p.nodes_z0;
            out.grid_elems += p.grid_elems;
            out.scratch_elems += p.scratch_elems;
            out.base_elems += p.base_elems;
            out.bytes_forward += p.bytes_forward;
            out.flops_forward += p.flops_forward;
            out.N += p.N;
            out.M += p.M;
        }
    }
    if (out.M > (int64_t)INT32_MAX) return FLT_ERANGE;
    finish(out);
    return FLT_OK;
}

}  // namespace flt
