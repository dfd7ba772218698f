// Kernel bodies of the real-exponent transform (device and CPU build alike):
// the frequency-side window spread and gather of the NNFFT, and the node-side
// weighting around the inner integer sums.  See xi_plan.h for the scheme.
#pragma once
#include "kernels_impl.h"
#include "xi_plan.h"

namespace flt {

// ceil(log2 xi) for a finite xi >= 1, from the bits (host and device alike).
FLT_HD int ceil_log2_real(double xi)
{
    uint64_t bits;
    __builtin_memcpy(&bits, &xi, 8);
    const int e = (int)((bits >> 52) & 0x7ff) - 1022;   // xi = f 2^e, f in [1/2, 1)
    return (bits & 0xfffffffffffffull) == 0 ? e - 1 : e;
}

// The truncated Kaiser-Bessel window rho(u) = sinh(b v) / (pi v), v = sqrt(m^2 - u^2),
// |u| <= m (b / pi at v = 0).
template <typename T> FLT_HD T kb_rho(T u, int m, T b)
{
    const T v2 = T(m * m) - u * u;
    if (!(v2 > T(0))) return b * T(0.31830988618379067153776752674503);
    if constexpr (sizeof(T) == 4) {
        const float v = sqrt_f32(v2);
        const float e = exp2_f32(b * 1.4426950408889634f * v);
        return (e - rcp_f32(e)) * (0.5f * 0.31830988618379067154f) * rcp_f32(v);
    } else {
        const double v = sqrt(v2);
        return sinh(b * v) / v * 0.31830988618379067153776752674503;
    }
}

// 1 / rho_hat(t), rho_hat(t) = I_0(m sqrt(b^2 - (2 pi t)^2)) (|2 pi t| < b),
// FP64 power series of I_0.
FLT_HD double kb_inv_rho_hat(double t, int m, double b)
{
    const double w = 6.283185307179586476925286766559 * t;
    const double a = m * sqrt(b * b - w * w);
    const double q = 0.25 * a * a;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return 1.0 / sum;
}

// e^{2 pi i l x} for an integer l and a real x: the phase reduced in FP64 with
// the error-free product, its sine and cosine in the working type.
template <typename T> FLT_HD void int_phase(double l, double x, double* cs, double* sn)
{
    const double p = l * x;
    const double e = fma(l, x, -p);
    const double ph = (p - rint(p)) + e;
    if constexpr (sizeof(T) == 4) {
        float s, c;
        sincos_rev_f32((float)ph, &s, &c);
        *cs = c;
        *sn = s;
    } else {
        sincos(6.283185307179586476925286766559 * ph, sn, cs);
    }
}

// Stage the item's interpolated blocks (q x q coefficients each, a[s][i] of
// block ell_lo + blk_lo + b at lc[(b q + s) q + i]).
template <class Ctx, typename T>
FLT_HD void xi_stage_blocks(const Ctx& ctx, const XiView<T>& xv, const XiBand& X, const XiItem& it, T* lc)
{
    if (it.nblk <= 0) return;
    const int qq = X.q * X.q, n = it.nblk * qq;
    const T* src = xv.coef + X.coef_off + (int64_t)it.blk_lo * qq;
    for (int i = ctx.tid(); i < n; i += ctx.ntid()) lc[i] = src[i];
}

// t_s(xi) = the band's interpolant of e^{-y_s xi} at exponent xi for every
// column s < q (1 on the blocks where the kernel is ~1): the Chebyshev
// polynomials T_i(u) of the block's variable u = xi 2^(2-c) - 3, then the
// rows of coefficients (from LDS when staged).
template <typename T, int QM>
FLT_HD void xi_rows(const XiView<T>& xv, const XiBand& X, const XiItem& it, const T* lc, double xi, T* t)
{
    const int q = X.q;
    const int cl = ceil_log2_real(xi);
    const int ell = X.n_xi + 1 - cl;
    if (X.ell_hi < X.ell_lo || ell > X.ell_hi) {
#pragma unroll
        for (int s = 0; s < QM; ++s) t[s] = T(1);
        return;
    }
    const T u = (T)(ldexp(xi, 2 - cl) - 3.0);
    T tc[QM];
    tc[0] = T(1);
    tc[1] = u;
#pragma unroll
    for (int i = 2; i < QM; ++i) tc[i] = T(2) * u * tc[i - 1] - tc[i - 2];
    const int blk = ell - X.ell_lo;
    const T* a = it.nblk > 0 && blk >= it.blk_lo && blk < it.blk_lo + it.nblk
                     ? lc + (int64_t)(blk - it.blk_lo) * q * q
                     : xv.coef + X.coef_off + (int64_t)blk * q * q;
#pragma unroll
    for (int s = 0; s < QM; ++s) {
        T acc = T(0);
        if (s < q) {
            const T* row = a + s * q;
#pragma unroll
            for (int i = 0; i < QM; ++i)   // static indices keep tc in registers
                if (i < q) acc += row[i] * tc[i];
        }
        t[s] = acc;
    }
}

// Forward, frequency side: for the run of integer frequencies l of the item,
// G_s[l] = sum_k c_k t_s(xi_k) rho(sigma xi_k - l) over the exponents whose
// window reaches l, every column s of the band at once; written as the inner
// plan's coefficients of instance (band, s), index l - l_lo.  When the run's
// exponents fit (at most xi_kcap of them), c_k t_s(xi_k) is formed once per
// exponent in LDS (ct, each exponent reaches 2m frequencies); otherwise every
// frequency evaluates the rows of its exponents itself.
template <typename T, int QM> constexpr int xi_kcap() { return (32 * 1024) / (QM * (int)sizeof(cplx<T>)); }
template <class Ctx, typename T, int QM>
FLT_HD void body_xi_spread(const Ctx& ctx, const XiView<T>& xv, const XiItem* items, const cplx<T>* c,
                           cplx<T>* cin, T* lc, cplx<T>* ct)
{
    const XiItem it = items[ctx.bid()];
    const XiBand& X = xv.bands[it.band];
    xi_stage_blocks(ctx, xv, X, it, lc);
    ctx.sync();
    const int tid = ctx.tid();
    const int64_t nk = it.k_hi - it.k_lo;
    const bool staged = nk <= xi_kcap<T, QM>();
    if (staged) {
        for (int64_t kk = tid; kk < nk; kk += ctx.ntid()) {
            const int64_t k = it.k_lo + kk;
            const cplx<T> ck = c[xv.xi_perm[k]];
            T t[QM];
            xi_rows<T, QM>(xv, X, it, lc, xv.xi[k], t);
#pragma unroll
            for (int s = 0; s < QM; ++s)
                if (s < X.q) ct[kk * QM + s] = mk<T>(ck.x * t[s], ck.y * t[s]);
        }
        ctx.sync();
    }
    if (tid >= it.count) return;
    const int64_t li = it.first + tid;
    const double l = (double)(X.l_lo + li);
    const int m = xv.mw1;
    // first exponent with sigma xi - l > -m
    int64_t lo = it.k_lo, hi = it.k_hi;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (X.sig * xv.xi[mid] - l > -m) hi = mid;
        else lo = mid + 1;
    }
    T gr[QM], gi[QM];
#pragma unroll
    for (int s = 0; s < QM; ++s) gr[s] = gi[s] = T(0);
    for (int64_t k = lo; k < it.k_hi; ++k) {
        const double xk = xv.xi[k];
        const double u = X.sig * xk - l;
        if (u > m) break;
        const T w = kb_rho<T>((T)u, m, (T)X.kb_b);
        if (staged) {
            const cplx<T>* row = ct + (k - it.k_lo) * QM;
#pragma unroll
            for (int s = 0; s < QM; ++s)
                if (s < X.q) {
                    const cplx<T> v = row[s];
                    gr[s] += w * v.x;
                    gi[s] += w * v.y;
                }
        } else {
            const cplx<T> ck = c[xv.xi_perm[k]];
            const T cr = ck.x * w, ci = ck.y * w;
            T t[QM];
            xi_rows<T, QM>(xv, X, it, lc, xk, t);
#pragma unroll
            for (int s = 0; s < QM; ++s) {
                gr[s] += cr * t[s];
                gi[s] += ci * t[s];
            }
        }
    }
    cplx<T>* out = cin + X.cin_off + li;
#pragma unroll
    for (int s = 0; s < QM; ++s)
        if (s < X.q) out[(int64_t)s * X.l_count] = mk<T>(gr[s], gi[s]);
}

// Forward, node side: f_j = e^{2 pi i l_lo x'} / rho_hat(x') sum_s L_s(y_j) H_s(x'),
// x' = x_p / sigma, H_s the inner sums (instance (band, s)), FP64 sum; 0 on Z^0.
template <class Ctx, typename T>
FLT_HD void body_xi_combine(const Ctx& ctx, const XiView<T>& xv, const NodeItem* items, const cplx<T>* hin,
                            cplx<T>* f)
{
    const NodeItem it = items[ctx.bid()];
    const int i = ctx.tid();
    if (i >= it.count) return;
    const int64_t j = it.start + i;
    const XiBand& X = xv.bands[it.band];
    const int32_t dst = xv.perm[j];
    if (X.q == 0) {
        f[dst] = mk<T>(0, 0);
        return;
    }
    const int64_t local = j - X.node_start;
    const double xq = xv.xp[j] / X.sig, y = xv.ny[j];
    const double* yc = xv.ycheb + 2 * X.ycheb_off;
    const BaryY<T> by = bary_setup<T>(yc, X.q, y);
    double ar = 0, ai = 0;
    for (int s = 0; s < X.q; ++s) {
        const double L = (double)bary_at<T>(yc, by, s, y);
        const cplx<T> v = hin[X.hout_off + (int64_t)s * X.node_count + local];
        ar += L * (double)v.x;
        ai += L * (double)v.y;
    }
    double cs, sn;
    int_phase<T>((double)X.l_lo, xq, &cs, &sn);
    const double r = kb_inv_rho_hat(xq, xv.mw1, X.kb_b);
    f[dst] = mk<T>((T)((ar * cs - ai * sn) * r), (T)((ar * sn + ai * cs) * r));
}

// Transposed, node side: u_s,j = g_j L_s(y_j) e^{2 pi i l_lo x'} / rho_hat(x')
// for the inner transposed sums, stored conjugated (the inner plan's adjoint
// computes sum_j u_j conj(w_j)^i); conj_in: g conjugated first (the adjoint).
template <class Ctx, typename T>
FLT_HD void body_xi_prep(const Ctx& ctx, const XiView<T>& xv, const NodeItem* items, const cplx<T>* g, int conj_in,
                         cplx<T>* uin)
{
    const NodeItem it = items[ctx.bid()];
    const int i = ctx.tid();
    if (i >= it.count) return;
    const int64_t j = it.start + i;
    const XiBand& X = xv.bands[it.band];
    if (X.q == 0) return;
    const int64_t local = j - X.node_start;
    const double xq = xv.xp[j] / X.sig, y = xv.ny[j];
    cplx<T> gv = g[xv.perm[j]];
    if (conj_in) gv.y = -gv.y;
    double cs, sn;
    int_phase<T>((double)X.l_lo, xq, &cs, &sn);
    const double r = kb_inv_rho_hat(xq, xv.mw1, X.kb_b);
    const double ur = ((double)gv.x * cs - (double)gv.y * sn) * r;
    const double ui = ((double)gv.x * sn + (double)gv.y * cs) * r;
    const double* yc = xv.ycheb + 2 * X.ycheb_off;
    const BaryY<T> by = bary_setup<T>(yc, X.q, y);
    for (int s = 0; s < X.q; ++s) {
        const double L = (double)bary_at<T>(yc, by, s, y);
        uin[X.hout_off + (int64_t)s * X.node_count + local] = mk<T>((T)(ur * L), (T)(-ui * L));
    }
}

// Transposed, frequency side: for the item's run of sorted exponents,
// h_k += sum_s t_s(xi_k) sum_l rho(sigma xi_k - l) V_s[l] over this band, V_s
// the inner transposed sums (the inner adjoint's output, conjugated); FP64
// partials added atomically into hacc (one band per item).
template <class Ctx, typename T, int QM>
FLT_HD void body_xi_gather(const Ctx& ctx, const XiView<T>& xv, const XiItem* items, const cplx<T>* vin,
                           double* hacc, T* lc)
{
    const XiItem it = items[ctx.bid()];
    const XiBand& X = xv.bands[it.band];
    xi_stage_blocks(ctx, xv, X, it, lc);
    ctx.sync();
    const int tid = ctx.tid();
    if (tid >= it.count) return;
    const int64_t k = it.first + tid;
    const double xk = xv.xi[k];
    const int m = xv.mw1;
    T t[QM];
    xi_rows<T, QM>(xv, X, it, lc, xk, t);
    // the window's 2m taps: l = ceil(sigma xi - m) + r, u = sigma xi - l in (-m, m]
    const double sx = X.sig * xk;
    const double l0 = ceil(sx - m);
    T w[2 * MAX_MW];
#pragma unroll
    for (int r = 0; r < 2 * MAX_MW; ++r) w[r] = r < 2 * m ? kb_rho<T>((T)(sx - (l0 + r)), m, (T)X.kb_b) : T(0);
    const int64_t base = (int64_t)l0 - X.l_lo;
    double ar = 0, ai = 0;
#pragma unroll
    for (int s = 0; s < QM; ++s) {
        if (s < X.q) {
            const cplx<T>* v = vin + X.cin_off + (int64_t)s * X.l_count + base;
            T sr = 0, si = 0;
#pragma unroll
            for (int r = 0; r < 2 * MAX_MW; ++r)
                if (r < 2 * m) {
                    const cplx<T> x = v[r];
                    sr += w[r] * x.x;
                    si -= w[r] * x.y;   // V_s = conj(inner adjoint output)
                }
            ar += (double)(t[s] * sr);
            ai += (double)(t[s] * si);
        }
    }
    ctx.atomic_add(hacc + 2 * k, ar);
    ctx.atomic_add(hacc + 2 * k + 1, ai);
}

// Transposed, last step: h[caller k] = the FP64 sum in the working type
// (conjugated for the adjoint).
template <class Ctx, typename T>
FLT_HD void body_xi_finalize(const Ctx& ctx, const XiView<T>& xv, int64_t N, const double* hacc, int conj_out,
                             cplx<T>* h)
{
    const int64_t k = (int64_t)ctx.bid() * XI_THREADS + ctx.tid();
    if (k >= N) return;
    const double im = conj_out ? -hacc[2 * k + 1] : hacc[2 * k + 1];
    h[xv.xi_perm[k]] = mk<T>((T)hacc[2 * k], (T)im);
}

}  // namespace flt
