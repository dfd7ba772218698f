// Kernel bodies of the fast Fourier-Laplace transform (Kunis & Melzer,
// Algorithm 2).  Every body is a template over an execution context `Ctx`
// that supplies the workgroup geometry, the barrier and atomics, so one
// source serves the gfx950 kernels (kernels.hip) and a CPU build used by the
// tests to check indexing and bounds before anything runs on the GPU.
//
// Per band m the forward transform is, for each column s < q:
//   a2/a3  G[k, s] = c_k * t_k[s],  t_k[s] = sum_r L_r^{Omega_l}(k) K^{Y_m,Omega_l}[s, r]
//          (the frequency side of the tensor interpolant, Lemma 4.2 / Alg. 2),
//          t_k[s] = 1 on blocks l > L_m (Lemma A.2 iv), deconvolved by
//          1/(n phi_hat(k - k0)) and placed at (k - k0) mod n;
//   a4     g_s[l] = sum_k' Ghat[k', s] e^{2 pi i k' l / n}  (oversampled FFT);
//   a5     F_s(x_j) = sum_{|n x_j - l| < mw} g_s[l] phi(x_j - l/n)  (window gather);
//   a6     f_j = c_0 + e^{2 pi i k0 x_j} sum_s L_s^{Y_m}(y_j) F_s(x_j)   (FP64 sum).
// The adjoint runs the transposes in reverse order.
#pragma once
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "flt_types.h"

namespace flt {

// Calls f(std::integral_constant<int, v>) for the run-time value v in [LO, HI]
// (a uniform branch inside a kernel, or a host-side choice).
template <int LO, int HI, class F> FLT_HD bool with_log2(int v, F&& f)
{
    if constexpr (LO > HI) {
        return false;
    } else {
        if (v == LO) {
            f(std::integral_constant<int, LO>{});
            return true;
        }
        return with_log2<LO + 1, HI>(v, f);
    }
}

// Transform lengths (log2) of the FFT kernels: one-pass bands, two-pass grids
// (pass A is specialised on the whole length n) and pass B (floor(log2 n / 2)).
template <typename T> struct Log2Range {
    static constexpr int P = Sizes<T>::LOG2P;
    static constexpr int ONE_LO = 4, ONE_HI = P;
    static constexpr int TWO_LO = P + 1, TWO_HI = TW2_LOG2;
    static constexpr int B_LO = (P + 1) / 2, B_HI = TW2_LOG2 / 2;
};

// a * b for 0 <= a, b and a * b < 2^23 (a full-rate 24-bit multiply on the GPU)
FLT_HD int mul_small(int a, int b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __mul24(a, b);
#else
    return a * b;
#endif
}

FLT_HD int ceil_log2_u32(int k)  // 1 <= k < 2^31
{
    return k <= 1 ? 0 : 32 - __builtin_clz((unsigned)(k - 1));
}

// ---------------------------------------------------------------------------
// Frequency side: t_k[s], the interpolant of xi -> e^{-y_s xi} on the block
// Omega_l that holds k, evaluated from its Chebyshev coefficients (the same
// polynomial as sum_r K[s,r] L_r(k); coefficients built by the planner).
// ---------------------------------------------------------------------------
template <typename T>
FLT_HD T laplace_row(const PlanView<T>& pv, const BandDesc& B, int s, int k)
{
    const int cl = ceil_log2_u32(k);           // Omega_l = (2^(cl-1), 2^cl] holds k
    const int ell = B.n_xi + 1 - cl;
    if (ell > B.ell_hi) return T(1);           // kernel ~ 1 on l > L_m (Lemma A.2 iv)
    const int q = B.q;
    const T* a = pv.coef + B.coef_off + ((ell - B.ell_lo) * q + s) * q;
    // u = (k - centre) / half-width = k 2^(2-cl) - 3, exact in T for k < 2^24
    const T u = (T)ldexp((double)k, 2 - cl) - T(3);
    const T u2 = u + u;
    T b1 = 0, b2 = 0;
    for (int i = q - 1; i >= 1; --i) {         // Clenshaw
        T b0 = a[i] + u2 * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return a[0] + u * b1 - b2;
}

// Value of column s of band B's FFT input at natural grid index j.
template <typename T>
FLT_HD cplx<T> grid_input(const PlanView<T>& pv, const BandDesc& B, const cplx<T>* c,
                          int s, int j, int deriv)
{
    const int n = 1 << B.log2n;
    const int kp = j < (n >> 1) ? j : j - n;
    const int k = kp + (int)B.k0;
    if (k < 1 || k > B.kmax) return mk<T>(0, 0);
    T w = laplace_row(pv, B, s, k) * pv.deconv[B.deconv_off + (kp < 0 ? -kp : kp)];
    cplx<T> v = c[B.c_off + k];
    if (deriv) {                                // c'_k = 2 pi i k c_k
        w *= (T)(6.283185307179586476925286766559 * (double)k);
        v = mk(-v.y, v.x);
    }
    return scale(v, w);
}

// ---------------------------------------------------------------------------
// Radix-2/4/8 butterflies: X[a] = sum_b v[b] e^{sign 2 pi i a b / R}
// ---------------------------------------------------------------------------
template <typename T> FLT_HD void dft2(cplx<T>* v)
{
    cplx<T> a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
}
template <typename T> FLT_HD void dft4(cplx<T>* v, int sign)
{
    cplx<T> s02 = add(v[0], v[2]), d02 = sub(v[0], v[2]);
    cplx<T> s13 = add(v[1], v[3]), d13 = mul_isign(sub(v[1], v[3]), sign);
    v[0] = add(s02, s13);
    v[2] = sub(s02, s13);
    v[1] = add(d02, d13);
    v[3] = sub(d02, d13);
}
template <typename T> FLT_HD void dft8(cplx<T>* v, int sign)
{
    cplx<T> a[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> b[4] = {v[1], v[3], v[5], v[7]};
    dft4(a, sign);
    dft4(b, sign);
    const T h = T(0.70710678118654752440084436210485);
    const T sh = sign > 0 ? h : -h;
    cplx<T> w1 = mul(b[1], mk(h, sh));
    cplx<T> w2 = mul_isign(b[2], sign);
    cplx<T> w3 = mul(b[3], mk(-h, sh));
    v[0] = add(a[0], b[0]); v[4] = sub(a[0], b[0]);
    v[1] = add(a[1], w1);   v[5] = sub(a[1], w1);
    v[2] = add(a[2], w2);   v[6] = sub(a[2], w2);
    v[3] = add(a[3], w3);   v[7] = sub(a[3], w3);
}

// 16 = 4 x 4: DFT4 over n1 of x[4 n1 + n2], twiddle e^{sign 2 pi i n2 k1 / 16}, DFT4 over n2.
template <typename T> FLT_HD void dft16(cplx<T>* v, int sign)
{
    const T C1 = T(0.92387953251128675612818318939679), S1 = T(0.38268343236508977172845998403040);
    const T H = T(0.70710678118654752440084436210485);
    const T sg = sign > 0 ? T(1) : T(-1);
    cplx<T> a[4][4];
    for (int n2 = 0; n2 < 4; ++n2) {
        for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
        dft4(a[n2], sign);
    }
    // e^{sign 2 pi i m / 16} for m = n2 k1
    a[1][1] = mul(a[1][1], mk(C1, sg * S1));
    a[1][2] = mul(a[1][2], mk(H, sg * H));
    a[1][3] = mul(a[1][3], mk(S1, sg * C1));
    a[2][1] = mul(a[2][1], mk(H, sg * H));
    a[2][2] = mul_isign(a[2][2], sign);
    a[2][3] = mul(a[2][3], mk(-H, sg * H));
    a[3][1] = mul(a[3][1], mk(S1, sg * C1));
    a[3][2] = mul(a[3][2], mk(-H, sg * H));
    a[3][3] = mul(a[3][3], mk(-C1, -sg * S1));
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4(b, sign);
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
}

template <typename T, int R> FLT_HD void dft(cplx<T>* v, int sign)
{
    if (R == 2) dft2(v);
    else if (R == 4) dft4(v, sign);
    else if (R == 8) dft8(v, sign);
    else dft16(v, sign);
}

// e^{sign 2 pi i t / 2^TW_STAGE_LOG2}
template <typename T> FLT_HD cplx<T> tw_stage_at(const cplx<T>* tw, int t, int sign)
{
    cplx<T> w = tw[t];
    if (sign > 0) w.y = -w.y;
    return w;
}

// e^{sign 2 pi i e / n}, n = 2^log2n <= 2^22, from the two-level table; e is
// taken mod 2^32 (n divides 2^32, so a wrapped product j2 l1 gives e mod n).
// In two steps where several are wanted at once: the two table factors
// (tw_grid_fetch), then their product (tw_grid_join).
template <typename T> struct TwPair { cplx<T> hi, lo; };
template <typename T> FLT_HD TwPair<T> tw_grid_fetch(const PlanView<T>& pv, uint32_t e, int log2n)
{
    const uint32_t ee = (e & ((1u << log2n) - 1u)) << (TW2_LOG2 - log2n);
    return TwPair<T>{pv.tw_hi[ee >> TW2_HALF], pv.tw_lo[ee & ((1 << TW2_HALF) - 1)]};
}
template <typename T> FLT_HD cplx<T> tw_grid_join(const TwPair<T>& t, int sign)
{
    cplx<T> w = mul(t.hi, t.lo);
    if (sign > 0) w.y = -w.y;
    return w;
}
template <typename T> FLT_HD cplx<T> tw_grid_at(const PlanView<T>& pv, uint32_t e, int log2n, int sign)
{
    return tw_grid_join(tw_grid_fetch(pv, e, log2n), sign);
}

// Largest radix (log2) a thread handles in registers: the points it holds per stage.
template <typename T> struct MaxRadix;
template <> struct MaxRadix<float> { static constexpr int LOG2 = 4; };
template <> struct MaxRadix<double> { static constexpr int LOG2 = 3; };

constexpr int next_radix_log2(int rem, int maxr)
{
    int r = rem < maxr ? rem : maxr;
    if (rem - r == 1 && r > 2) r -= 1;   // leave no radix-2 stage when a larger split exists
    return r;
}

// Stage twiddles w^r, w = e^{SIGN 2 pi i k / (Ns R)}, r < R, are formed as
// w^{r1} w^{2^LA r2} (r = r1 + 2^LA r2, LA = LR / 2, LB = LR - LA): 2^LA + 2^LB - 2
// factors instead of R - 1, at most one extra rounded product each.  Two
// sources of the factors:
//
// TableTw reads them from the stage table at every stage;
template <typename T> struct TableTw {
    const cplx<T>* tw;   // e^{-2 pi i t / 2^TW_STAGE_LOG2}
    template <int LR, int LOG2NS, int SIGN>
    FLT_HD void factors(int /*i*/, int k, cplx<T>* wa, cplx<T>* wb) const
    {
        constexpr int SH = TW_STAGE_LOG2 - LOG2NS - LR;
        constexpr int LA = LR / 2, LB = LR - LA;
        for (int r1 = 1; r1 < (1 << LA); ++r1) wa[r1] = tw_stage_at(tw, (k * r1) << SH, SIGN);
        for (int r2 = 1; r2 < (1 << LB); ++r2) wb[r2] = tw_stage_at(tw, (k * r2) << (SH + LA), SIGN);
    }
    template <class Ctx> FLT_HD void load(const Ctx&, const cplx<T>* t) { tw = t; }
    FLT_HD const TableTw& next() const { return *this; }
};

// StageTw holds one thread's factors of every stage of a transform geometry
// (LOG2L, NSUB) in registers.  They depend on the thread index alone, so one
// load serves every tile of that geometry the workgroup transforms.
template <typename T, int LOG2L, int NSUB, int SIGN, int LOG2NS = 0, bool MORE = (LOG2L > LOG2NS)>
struct StageTw {
    template <class Ctx> FLT_HD void load(const Ctx&, const cplx<T>*) {}
};
template <typename T, int LOG2L, int NSUB, int SIGN, int LOG2NS>
struct StageTw<T, LOG2L, NSUB, SIGN, LOG2NS, true> {
    static constexpr int LR = next_radix_log2(LOG2L - LOG2NS, MaxRadix<T>::LOG2);
    static constexpr int LA = LR / 2, LB = LR - LA;
    static constexpr int LOG2LQ = LOG2L - LR;
    static constexpr int NBUT = (NSUB << LOG2L) >> LR;
    static constexpr int NB = (NBUT + FFT_THREADS - 1) / FFT_THREADS;
    static constexpr int NW = LOG2NS > 0 ? NB : 1;   // the first stage (Ns = 1) has no twiddles
    cplx<T> wa[NW][1 << LA], wb[NW][1 << LB];
    StageTw<T, LOG2L, NSUB, SIGN, LOG2NS + LR> nx;

    template <class Ctx> FLT_HD void load(const Ctx& ctx, const cplx<T>* tw)
    {
        if constexpr (LOG2NS > 0) {
            const TableTw<T> tab{tw};
            for (int i = 0; i < NB; ++i) {
                const int u = ctx.tid() + i * FFT_THREADS;
                const int k = u & ((1 << LOG2NS) - 1);   // u mod (L / R) mod Ns
                if ((NBUT % FFT_THREADS) == 0 || u < NBUT) tab.template factors<LR, LOG2NS, SIGN>(i, k, wa[i], wb[i]);
            }
        }
        nx.load(ctx, tw);
    }
    template <int LR_, int LOG2NS_, int SIGN_>
    FLT_HD void factors(int i, int /*k*/, cplx<T>* a, cplx<T>* b) const
    {
        static_assert(LR_ == LR && LOG2NS_ == LOG2NS && SIGN_ == SIGN, "twiddles of another geometry");
        for (int r1 = 1; r1 < (1 << LA); ++r1) a[r1] = wa[i][r1];
        for (int r2 = 1; r2 < (1 << LB); ++r2) b[r2] = wb[i][r2];
    }
    FLT_HD const StageTw<T, LOG2L, NSUB, SIGN, LOG2NS + LR>& next() const { return nx; }
};

// The twiddle source of an FFT: registers (REG) or the table.
template <bool REG, typename T, int LOG2L, int NSUB, int SIGN> struct TwSel { using type = StageTw<T, LOG2L, NSUB, SIGN>; };
template <typename T, int LOG2L, int NSUB, int SIGN> struct TwSel<false, T, LOG2L, NSUB, SIGN> { using type = TableTw<T>; };

// Stage twiddles of transforms of one length L = 2^LOG2L from a half table in
// LDS, th[t] = e^{-2 pi i t / L} for t < L/2, and e^{-2 pi i t / L} = -th[t - L/2]
// above: the persistent pass B's factors without a global gather per factor
// (its registers hold the prefetched tile instead).
template <int LOG2L> constexpr int lds_tw_half() { return 1 << (LOG2L - 1); }
template <typename T, int LOG2L> struct LdsTw {
    const cplx<T>* th;
    template <int SIGN> FLT_HD cplx<T> at(int e) const   // e in [0, L)
    {
        constexpr int H = lds_tw_half<LOG2L>();
        cplx<T> w = th[e & (H - 1)];
        if (e & H) w = mk(-w.x, -w.y);
        if (SIGN > 0) w.y = -w.y;
        return w;
    }
    template <int LR, int LOG2NS, int SIGN>
    FLT_HD void factors(int /*i*/, int k, cplx<T>* wa, cplx<T>* wb) const
    {
        constexpr int SH = LOG2L - LOG2NS - LR;   // k r < Ns R <= L: indices below L
        constexpr int LA = LR / 2, LB = LR - LA;
        for (int r1 = 1; r1 < (1 << LA); ++r1) wa[r1] = at<SIGN>((k * r1) << SH);
        for (int r2 = 1; r2 < (1 << LB); ++r2) wb[r2] = at<SIGN>((k * r2) << (SH + LA));
    }
    // every thread writes its share of the table; a barrier must follow before use
    template <class Ctx> FLT_HD void fill(const Ctx& ctx, const cplx<T>* tw_global, cplx<T>* lds_table)
    {
        th = lds_table;
        for (int t = ctx.tid(); t < lds_tw_half<LOG2L>(); t += ctx.ntid())
            lds_table[t] = tw_global[t << (TW_STAGE_LOG2 - LOG2L)];
    }
    FLT_HD const LdsTw& next() const { return *this; }
};

// The geometry of one Stockham stage: NB butterflies of radix R per thread.
template <int LR, int LOG2L, int NSUB> struct StageGeo {
    static constexpr int R = 1 << LR;
    static constexpr int NBUT = (NSUB << LOG2L) >> LR;
    static constexpr int NB = (NBUT + FFT_THREADS - 1) / FFT_THREADS;
};

// The read and butterfly half of a stage: v[i] receives butterfly i's R
// outputs, whose tile elements are dsti[i] + r 2^LOG2NS (dsti[i] < 0: the
// thread has no butterfly i).
template <class Ctx, typename T, int LR, int LOG2L, int NSUB, int LOG2NS, int SIGN, class TW>
FLT_HD void fft_stage_compute(const Ctx& ctx, const cplx<T>* src, const TW& tw,
                              cplx<T> (&v)[StageGeo<LR, LOG2L, NSUB>::NB][1 << LR],
                              int (&dsti)[StageGeo<LR, LOG2L, NSUB>::NB])
{
    constexpr int R = 1 << LR;
    constexpr int NBUT = StageGeo<LR, LOG2L, NSUB>::NBUT;
    constexpr int LOG2LQ = LOG2L - LR;
    constexpr int NB = StageGeo<LR, LOG2L, NSUB>::NB;
    for (int i = 0; i < NB; ++i) {
        const int u = ctx.tid() + i * FFT_THREADS;
        dsti[i] = -1;
        if ((NBUT % FFT_THREADS) == 0 || u < NBUT) {
            const int sub = u >> LOG2LQ;
            const int j = u & ((1 << LOG2LQ) - 1);
            const int srci = (sub << LOG2L) + j;
            if constexpr (LOG2LQ >= 4) {   // strides of multiples of 16: the pad is a constant offset
                const int sp = lds_at(srci);
                for (int r = 0; r < R; ++r) v[i][r] = src[sp + (r << LOG2LQ) + (r << (LOG2LQ - 4))];
            } else {
                for (int r = 0; r < R; ++r) v[i][r] = src[lds_at(srci + (r << LOG2LQ))];
            }
            const int k = j & ((1 << LOG2NS) - 1);
            if constexpr (LOG2NS > 0) {
                constexpr int LA = LR / 2, LB = LR - LA;
                cplx<T> wa[1 << LA], wb[1 << LB];
                tw.template factors<LR, LOG2NS, SIGN>(i, k, wa, wb);
                for (int r = 1; r < R; ++r) {
                    const int r1 = r & ((1 << LA) - 1), r2 = r >> LA;
                    const cplx<T> w = r2 == 0 ? wa[r1] : r1 == 0 ? wb[r2] : mul(wa[r1], wb[r2]);
                    v[i][r] = mul(v[i][r], w);
                }
            }
            dft<T, R>(v[i], SIGN);
            dsti[i] = (sub << LOG2L) + ((j >> LOG2NS) << (LOG2NS + LR)) + k;
        }
    }
}

// One Stockham autosort radix-2^LR stage over NSUB contiguous transforms of
// length 2^LOG2L, all geometry known at compile time, reading `src` and
// writing `dst` (LDS).  In place (src == dst, INPLACE): reads, barrier,
// writes, barrier; out of place: reads, writes, barrier.  Twiddles
// e^{SIGN 2 pi i k r / (Ns R)} from the provider tw (TableTw or StageTw).
template <class Ctx, typename T, int LR, int LOG2L, int NSUB, int LOG2NS, int SIGN, bool INPLACE, class TW>
FLT_HD void fft_stage_io(const Ctx& ctx, const cplx<T>* src, cplx<T>* dst, const TW& tw)
{
    constexpr int R = 1 << LR;
    constexpr int NB = StageGeo<LR, LOG2L, NSUB>::NB;
    cplx<T> v[NB][R];
    int dsti[NB];
    fft_stage_compute<Ctx, T, LR, LOG2L, NSUB, LOG2NS, SIGN>(ctx, src, tw, v, dsti);
    if constexpr (INPLACE) ctx.sync();
    for (int i = 0; i < NB; ++i) {
        if (dsti[i] < 0) continue;
        if constexpr (LOG2NS >= 4) {
            const int dp = lds_at(dsti[i]);
            for (int r = 0; r < R; ++r) dst[dp + (r << LOG2NS) + (r << (LOG2NS - 4))] = v[i][r];
        } else if constexpr (LOG2NS + LR <= 4) {
            // dst = base + k with base a multiple of NS R <= 16 and k + r NS < NS R: no carry into bit 4
            const int dp = lds_at(dsti[i]);
            for (int r = 0; r < R; ++r) dst[dp + (r << LOG2NS)] = v[i][r];
        } else {
            for (int r = 0; r < R; ++r) dst[lds_at(dsti[i] + (r << LOG2NS))] = v[i][r];
        }
    }
    ctx.sync();
}

template <class Ctx, typename T, int LR, int LOG2L, int NSUB, int LOG2NS, int SIGN, class TW>
FLT_HD void fft_stage_ct(const Ctx& ctx, cplx<T>* buf, const TW& tw)
{
    fft_stage_io<Ctx, T, LR, LOG2L, NSUB, LOG2NS, SIGN, true>(ctx, buf, buf, tw);
}

// In-place DFTs X[l] = sum_j x[j] e^{SIGN 2 pi i j l / L} of NSUB transforms of
// length L = 2^LOG2L stored contiguously in LDS (Stockham, natural order in and
// out); tw supplies the stage twiddles (TableTw, or the StageTw of this geometry).
template <class Ctx, typename T, int LOG2L, int NSUB, int SIGN, int LOG2NS = 0, class TW>
FLT_HD void lds_fft_ct(const Ctx& ctx, cplx<T>* buf, const TW& tw)
{
    constexpr int REM = LOG2L - LOG2NS;
    if constexpr (REM > 0) {
        constexpr int LR = next_radix_log2(REM, MaxRadix<T>::LOG2);
        fft_stage_ct<Ctx, T, LR, LOG2L, NSUB, LOG2NS, SIGN>(ctx, buf, tw);
        lds_fft_ct<Ctx, T, LOG2L, NSUB, SIGN, LOG2NS + LR>(ctx, buf, tw.next());
    }
}

// The same DFTs from stage LOG2NS on with two LDS tiles in turn (one barrier
// per stage): the input in a, b free; returns the tile that holds the result.
template <class Ctx, typename T, int LOG2L, int NSUB, int SIGN, int LOG2NS = 0, class TW>
FLT_HD cplx<T>* lds_fft_pp(const Ctx& ctx, cplx<T>* a, cplx<T>* b, const TW& tw)
{
    constexpr int REM = LOG2L - LOG2NS;
    if constexpr (REM > 0) {
        constexpr int LR = next_radix_log2(REM, MaxRadix<T>::LOG2);
        fft_stage_io<Ctx, T, LR, LOG2L, NSUB, LOG2NS, SIGN, false>(ctx, a, b, tw);
        return lds_fft_pp<Ctx, T, LOG2L, NSUB, SIGN, LOG2NS + LR>(ctx, b, a, tw.next());
    } else {
        return a;
    }
}

// Radix (log2) of the last stage of the DFTs run from stage LOG2NS on.
constexpr int last_stage_lr(int log2l, int log2ns, int maxr)
{
    int rem = log2l - log2ns;
    for (;;) {
        const int r = next_radix_log2(rem, maxr);
        if (r == rem) return r;
        rem -= r;
    }
}

// The same DFTs from stage LOG2NS on with two LDS tiles in turn, the last
// stage kept in registers: fin(v, dsti) receives its outputs (the butterflies
// of fft_stage_compute at the last stage's geometry).  Returns the tile the
// last stage read.
template <class Ctx, typename T, int LOG2L, int NSUB, int SIGN, int LOG2NS, class TW, class FIN>
FLT_HD cplx<T>* lds_fft_pp_last_regs(const Ctx& ctx, cplx<T>* a, cplx<T>* b, const TW& tw, FIN&& fin)
{
    constexpr int REM = LOG2L - LOG2NS;
    constexpr int LR = next_radix_log2(REM, MaxRadix<T>::LOG2);
    if constexpr (LR == REM) {
        constexpr int NB = StageGeo<LR, LOG2L, NSUB>::NB;
        cplx<T> v[NB][1 << LR];
        int dsti[NB];
        fft_stage_compute<Ctx, T, LR, LOG2L, NSUB, LOG2NS, SIGN>(ctx, a, tw, v, dsti);
        fin(v, dsti);
        return a;
    } else {
        fft_stage_io<Ctx, T, LR, LOG2L, NSUB, LOG2NS, SIGN, false>(ctx, a, b, tw);
        return lds_fft_pp_last_regs<Ctx, T, LOG2L, NSUB, SIGN, LOG2NS + LR>(ctx, b, a, tw.next(), fin);
    }
}

// Points of the 64 KB LDS tile: P = 2^LOG2P complex values, ITEMS per thread.
template <typename T> constexpr int tile_points() { return 1 << Sizes<T>::LOG2P; }
template <typename T> constexpr int tile_items() { return tile_points<T>() / FFT_THREADS; }

// Chebyshev coefficients staged in LDS: each block's q coefficients padded
// with zeros to a whole number of 16-byte vectors (CV values), read as vectors.
template <typename T> struct alignas(16) CoefVec {
    static constexpr int N = 16 / (int)sizeof(T);
    T a[N];
};
FLT_HD int coef_stride(int q, int cv) { return (q + cv - 1) / cv * cv; }

// Column s's Chebyshev coefficients of every interpolated block of band B,
// staged into LDS as lc[(l - ell_lo) QP + i], QP = q padded to whole vectors.
template <class Ctx, typename T>
FLT_HD void stage_coef(const Ctx& ctx, const PlanView<T>& pv, const BandDesc& B, int s, T* lc)
{
    const int q = B.q, qp = coef_stride(q, CoefVec<T>::N);
    const int nblk = B.ell_hi - B.ell_lo + 1;
    for (int idx = ctx.tid(); idx < nblk * qp; idx += ctx.ntid()) {
        const int e = idx / qp, i = idx - e * qp;
        lc[idx] = i < q ? pv.coef[B.coef_off + (e * q + s) * q + i] : T(0);
    }
}

// t_k[s] from the staged coefficients of column s (see laplace_row): the
// same Clenshaw recurrence, the zero padding on top leaving it unchanged.
template <typename T>
FLT_HD T laplace_row_lds(const T* lc, const BandDesc& B, int k)
{
    constexpr int CV = CoefVec<T>::N;
    const int cl = ceil_log2_u32(k);
    const int ell = B.n_xi + 1 - cl;
    if (ell > B.ell_hi) return T(1);
    const int qp = coef_stride(B.q, CV);
    const CoefVec<T>* a = (const CoefVec<T>*)(lc + mul_small(ell - B.ell_lo, qp));
    const T u = ldexp((T)k, 2 - cl) - T(3);
    const T u2 = u + u;
    T b1 = 0, b2 = 0;
    for (int c = qp / CV - 1; c >= 1; --c) {
        const CoefVec<T> w = a[c];
        for (int j = CV - 1; j >= 0; --j) {
            const T b0 = w.a[j] + u2 * b1 - b2;
            b2 = b1;
            b1 = b0;
        }
    }
    const CoefVec<T> w = a[0];
    for (int j = CV - 1; j >= 1; --j) {
        const T b0 = w.a[j] + u2 * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return w.a[0] + u * b1 - b2;
}

// c_k / (n phi_hat(k - k0)), times 2 pi i k for the derivative transform.
template <typename T>
FLT_HD cplx<T> point_base(const PlanView<T>& pv, const BandDesc& B, const cplx<T>* c, int kp, int k, int deriv)
{
    T w = pv.deconv[B.deconv_off + (kp < 0 ? -kp : kp)];
    cplx<T> v = c[B.c_off + k];
    if (deriv) {
        w *= (T)(6.283185307179586476925286766559 * (double)k);
        v = mk(-v.y, v.x);
    }
    return scale(v, w);
}

// frac(k x) in [-1/2, 1/2] with the error-free product k x = p + e (FMA), FP64.
FLT_HD double frac_kx(double k, double x)
{
    const double p = k * x;
    const double e = fma(k, x, -p);
    return (p - rint(p)) + e;
}

// ---------------------------------------------------------------------------
// a2-a4, one-pass bands: generate `ns` columns, FFT them in LDS, store.
// ---------------------------------------------------------------------------
// cols = 2 (forward and derivative in one pass): the band has 2q columns,
// column q + s being column s of the derivative transform; the band's grid
// region is then twice as long (offsets doubled).
// LDS beside the tile for the staged coefficients: what keeps the pair under
// 80 KB (two workgroups per compute unit).
template <typename T> constexpr int onepass_coef() { return (80 * 1024 - (int)sizeof(cplx<T>) * tile_alloc<T>()) / (int)sizeof(T); }

// When the Chebyshev coefficients of all the workgroup's columns (every block
// of the band, see stage_coef) fit lc together, they are staged there first;
// otherwise the generation reads them from global memory (more passes of
// staging, each behind a barrier, cost more than they save).
template <class Ctx, typename T, int LOG2N>
FLT_HD void body_onepass_fwd(const Ctx& ctx, const PlanView<T>& pv, const FftItem* items,
                             const cplx<T>* c, cplx<T>* grids, int deriv, int cols, cplx<T>* lds, T* lc)
{
    // columns per workgroup: a full tile, but never more than a band has (q <= MAX_Q)
    constexpr int NSUB = (tile_points<T>() >> LOG2N) < MAX_Q ? (tile_points<T>() >> LOG2N) : MAX_Q;
    constexpr int P = NSUB << LOG2N;
    constexpr int n = 1 << LOG2N;
    const FftItem it = items[ctx.bid()];
    const BandDesc& B = pv.bands[it.band];
    StageTw<T, LOG2N, NSUB, +1> stw;
    stw.load(ctx, pv.tw_stage);
    auto column = [&](int sl, bool& dcol) {   // band column of tile column sl
        const int s = it.s0 + sl;
        dcol = s >= B.q;   // a derivative column (cols = 2)
        return dcol ? s - B.q : s;
    };
    const int nblk = B.ell_hi - B.ell_lo + 1;
    const int per_col = nblk > 0 ? nblk * coef_stride(B.q, CoefVec<T>::N) : 0;
    const int cpc = per_col == 0 ? it.ns : onepass_coef<T>() / per_col >= it.ns ? it.ns : 0;
    // the padding columns of the tile: zeros
    for (int p = (it.ns << LOG2N) + ctx.tid(); p < P; p += FFT_THREADS) lds[lds_at(p)] = mk<T>(0, 0);
    if (cpc == 0) {
        for (int p = ctx.tid(); p < (it.ns << LOG2N); p += FFT_THREADS) {
            bool dcol;
            const int s = column(p >> LOG2N, dcol);
            lds[lds_at(p)] = grid_input(pv, B, c, s, p & (n - 1), deriv || dcol);
        }
    } else {
        if (per_col > 0) {
            for (int sl = 0; sl < it.ns; ++sl) {
                bool dcol;
                stage_coef(ctx, pv, B, column(sl, dcol), lc + sl * per_col);
            }
            ctx.sync();
        }
        for (int p = ctx.tid(); p < (it.ns << LOG2N); p += FFT_THREADS) {
            const int sl = p >> LOG2N;
            bool dcol;
            column(sl, dcol);
            const int j = p & (n - 1);
            const int kp = j < (n >> 1) ? j : j - n;
            const int k = kp + (int)B.k0;
            cplx<T> v = mk<T>(0, 0);
            if (k >= 1 && k <= B.kmax) {
                v = point_base(pv, B, c, kp, k, deriv || dcol);
                if (per_col > 0) v = scale(v, laplace_row_lds(lc + sl * per_col, B, k));
            }
            lds[lds_at(p)] = v;
        }
    }
    ctx.sync();
    lds_fft_ct<Ctx, T, LOG2N, NSUB, +1>(ctx, lds, stw);
    cplx<T>* out = grids + B.grid_off * cols + ((int64_t)it.s0 << LOG2N);
    const int Pv = it.ns << LOG2N;
    for (int p = ctx.tid(); p < Pv; p += FFT_THREADS) out[p] = lds[lds_at(p)];
}

// ---------------------------------------------------------------------------
// a2-a4, two-pass bands, pass A: for b = 2^log2b consecutive j2, the length-n1
// DFTs over j1 of x[j2 + n2 j1] (generated from c), times e^{2 pi i j2 l1 / n},
// stored as Y[l1 / B][j2][l1 mod B].
// ---------------------------------------------------------------------------
// The split n = n1 n2 of a two-pass grid of length 2^LOG2N and the tile
// shapes of both passes (as the planner sets them), known at compile time.
template <typename T, int LOG2N> struct TwoPassGeo {
    static constexpr int log2n = LOG2N;
    static constexpr int log2n1 = (LOG2N + 1) / 2, log2n2 = LOG2N - log2n1;
    static constexpr int log2b = Sizes<T>::LOG2P - log2n1;   // pass A: sub-transforms per tile
    static constexpr int log2B = Sizes<T>::LOG2P - log2n2;   // pass B: sub-transforms per tile
};

// Pass A of the FP32 form and its thread geometry at compile time.  Each
// thread's c_k / (n phi_hat(k')) values stay in registers across the q columns
// of its band.  The first FFT stage (radix
// R1 = 2^LR1, no twiddles) is done in registers right after the column is
// generated: thread u holds sub-transform jj = u >> LOG2LQ and the points
// j1 = jl + r 2^LOG2LQ, r < R1, jl = u mod 2^LOG2LQ.  A band's support
// (k - k0 in [1 - n/4, n/4]) fills half the grid: x[j2 + n2 j1] can be
// non-zero only for j1 <= n1/4 or j1 >= 3 n1/4, i.e. r <= R1/4 or r >= 3 R1/4
// (LIVE), and r = R1/4 only at j2 = 0, jl = 0.
//
// Output twiddles e^{2 pi i j2 l1 / n} at the tile elements p = tid + i 512:
// when the bits of i fall in l1's high part only (SEP, the larger grids), l1 =
// l1_t + i DL and the factor is tw_t w(j2)^i, tw_t per thread, the powers
// w(j2)^i = e^{2 pi i j2 DL i / n} for the workgroup's b values of j2 in an LDS
// table of b * ITEMS entries; otherwise two reads of the global table per point.
template <typename T, int LOG2N> struct PassAGeo {
    using G = TwoPassGeo<T, LOG2N>;
    static constexpr int ITEMS = tile_items<T>();
    static constexpr int LR1 = next_radix_log2(G::log2n1, MaxRadix<T>::LOG2);
    static constexpr int R1 = 1 << LR1;
    static constexpr int LOG2LQ = G::log2n1 - LR1;
    static constexpr int LOG2T = 9;   // log2(FFT_THREADS)
    static constexpr bool SEP = G::log2B + G::log2b <= LOG2T;
    static constexpr int DL = SEP ? 1 << (LOG2T - G::log2b) : 0;
    static constexpr int OMEGA = SEP ? (1 << G::log2b) * ITEMS : 0;   // LDS table entries
    FLT_HD static constexpr bool live(int r) { return r <= R1 / 4 || r >= 3 * R1 / 4; }
    static_assert(ITEMS == R1, "one first-stage butterfly per thread");
    static_assert((1 << LOG2T) == FFT_THREADS, "thread count");
};
// LDS entries the output-twiddle table of pass A needs at most (FP32).
constexpr int PASSA_OMEGA_MAX = 256;

// k of grid index j of band B (the band's support centred at k0), or 0 when
// the point lies outside the support 1 <= k <= kmax.
FLT_HD int passA_k(int j, int n, int k0, int kmax)
{
    const int k = (j < (n >> 1) ? j : j - n) + k0;
    return k >= 1 && k <= kmax ? k : 0;
}

// The FP32 pass A.  LDS: two FFT tiles (lds, lds + tile_alloc) used in turn, so that an FFT
// stage needs one barrier and a column's output can be read from one tile
// while the next column is generated into the other; two coefficient buffers
// (lc, lc + COEF), the next column's staged during the current generation.
// Three barriers per column.
template <class Ctx, typename T, int LOG2N>
FLT_HD void body_passA_fwd(const Ctx& ctx, const PlanView<T>& pv, const FftItem* items,
                           const cplx<T>* c, cplx<T>* scratch, int deriv, int cols,
                           cplx<T>* lds, T* lc, cplx<T>* omega)
{
    static_assert(sizeof(T) == 4, "the FP32 form's pass A (FP64: body_passA_fwd_slot)");
    using G = TwoPassGeo<T, LOG2N>;
    using A = PassAGeo<T, LOG2N>;
    constexpr int ITEMS = A::ITEMS, R1 = A::R1, LR1 = A::LR1, LOG2LQ = A::LOG2LQ;
    constexpr int log2n1 = G::log2n1, log2n2 = G::log2n2, log2b = G::log2b, log2B = G::log2B;
    constexpr int n = 1 << LOG2N;
    const FftItem it = items[ctx.bid()];
    const BandDesc B = pv.bands[it.band];   // a copy: the stores below cannot alias it
    const int k0 = (int)B.k0, kmax = (int)B.kmax;
    const int j2_0 = it.blk << log2b;
    const int tid = ctx.tid();
    StageTw<T, log2n1, (1 << log2b), +1> stw;   // stage twiddles in registers
    stw.load(ctx, pv.tw_stage);

    // c_k / (n phi_hat(k')) of the workgroup's points, read from c in address
    // order (jj fastest) and transposed through the LDS tile ...
    for (int i = 0; i < ITEMS; ++i) {
        const int p = tid + i * FFT_THREADS;
        const int jj = p & ((1 << log2b) - 1);
        const int j1 = p >> log2b;
        const int j = j2_0 + jj + (j1 << log2n2);
        const int k = passA_k(j, n, k0, kmax);
        lds[lds_at((jj << log2n1) + j1)] = k ? point_base(pv, B, c, j < (n >> 1) ? j : j - n, k, deriv)
                                             : mk<T>(0, 0);
    }
    // ... the output-twiddle powers and the first column's coefficients
    const int o_l1lo = tid & ((1 << log2B) - 1);
    const int o_jj = (tid >> log2B) & ((1 << log2b) - 1);
    const int o_l1hi = tid >> (log2B + log2b);
    cplx<T> tw_t = mk<T>(1, 0);
    if constexpr (A::OMEGA > 0) {
        static_assert(A::OMEGA <= PASSA_OMEGA_MAX && A::OMEGA <= FFT_THREADS, "output twiddle table size");
        if (tid < A::OMEGA) {
            const int jj = tid / ITEMS, i = tid % ITEMS;
            omega[tid] = tw_grid_at(pv, (uint32_t)(j2_0 + jj) * (uint32_t)(A::DL * i), LOG2N, +1);
        }
        tw_t = tw_grid_at(pv, (uint32_t)(j2_0 + o_jj) * (uint32_t)((o_l1hi << log2B) + o_l1lo), LOG2N, +1);
    }
    stage_coef(ctx, pv, B, 0, lc);
    ctx.sync();
    cplx<T>* const tile[2] = {lds, lds + tile_alloc<T>()};
    // ... into registers, in the first stage's layout: only the live points
    const int jj_u = tid >> LOG2LQ;
    const int jl = tid & ((1 << LOG2LQ) - 1);
    const bool j2zero = j2_0 + jj_u == 0;          // the one grid row where r = R1/4 can be live
    cplx<T> base[R1];
    int kr[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
        base[r] = mk<T>(0, 0);
        kr[r] = 0;
        if (!A::live(r)) continue;
        const int j1 = jl + (r << LOG2LQ);
        base[r] = lds[lds_at((jj_u << log2n1) + j1)];
        kr[r] = passA_k(j2_0 + jj_u + (j1 << log2n2), n, k0, kmax);
    }
    ctx.sync();

    cplx<T>* const Ybase = scratch + B.scratch_off * cols;
    const int ncol = cols * B.q;
    cplx<T>* gen = tile[1];   // the tile the next column is generated into
    for (int s = 0; s < ncol; ++s) {
        // cols = 2: columns q .. 2q - 1 are the derivative's, the same
        // interpolant rows times 2 pi i k
        const bool dcol = s >= B.q;
        const T* lcs = lc + (s & 1) * Sizes<T>::COEF;
        // the next column's coefficients into the other buffer (last read by
        // the column before this one, before this column's first barrier)
        if (s + 1 < ncol) stage_coef(ctx, pv, B, s + 1 >= B.q ? s + 1 - B.q : s + 1, lc + ((s + 1) & 1) * Sizes<T>::COEF);
        // generate the live points of the column (the rest is zero), apply the
        // first radix-R1 stage in registers, store its output
        cplx<T> v[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            v[r] = mk<T>(0, 0);
            if (!A::live(r)) continue;
            if (r == R1 / 4 && !j2zero) continue;
            const int k = kr[r];
            T w = k ? laplace_row_lds(lcs, B, k) : T(0);
            cplx<T> b = base[r];
            if (dcol) {   // c'_k = 2 pi i k c_k
                w *= (T)(6.283185307179586476925286766559 * (double)k);
                b = mk(-b.y, b.x);
            }
            v[r] = scale(b, w);
        }
        dft<T, R1>(v, +1);
        {
            // Stockham output of a first stage: element (jj, jl R1 + r)
            const int dp = lds_at((jj_u << log2n1) + (jl << LR1));
#pragma unroll
            for (int r = 0; r < R1; ++r) gen[dp + r] = v[r];
        }
        ctx.sync();
        cplx<T>* const res =
            lds_fft_pp<Ctx, T, log2n1, (1 << log2b), +1, LR1>(ctx, gen, gen == tile[0] ? tile[1] : tile[0], stw.next());
        gen = res == tile[0] ? tile[1] : tile[0];
        // output: Y[l1 / B][j2][l1 mod B] = X_jj[l1] e^{2 pi i j2 l1 / n}, read
        // from res while the next column is generated into the other tile
        cplx<T>* Y = Ybase + ((int64_t)s << LOG2N);
        if constexpr (A::OMEGA > 0) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int l1 = (o_l1hi << log2B) + o_l1lo + i * A::DL;
                const int l1hi = l1 >> log2B;
                const cplx<T> wv = mul(tw_t, omega[o_jj * ITEMS + i]);
                Y[(l1hi << (log2n2 + log2B)) + ((j2_0 + o_jj) << log2B) + o_l1lo] =
                    mul(res[lds_at((o_jj << log2n1) + l1)], wv);
            }
        } else {
            // in groups of GO points: the group's table reads first (in flight
            // together), then the products and stores
            constexpr int GO = sizeof(T) == 4 ? 8 : 4;
#pragma unroll 1
            for (int i0 = 0; i0 < ITEMS; i0 += GO) {
                TwPair<T> w[GO];
                for (int u = 0; u < GO; ++u) {
                    const int p = tid + (i0 + u) * FFT_THREADS;
                    const int l1lo = p & ((1 << log2B) - 1);
                    const int jj = (p >> log2B) & ((1 << log2b) - 1);
                    const int l1 = ((p >> (log2B + log2b)) << log2B) + l1lo;
                    w[u] = tw_grid_fetch(pv, (uint32_t)(j2_0 + jj) * (uint32_t)l1, LOG2N);
                }
                for (int u = 0; u < GO; ++u) {
                    const int p = tid + (i0 + u) * FFT_THREADS;
                    const int l1lo = p & ((1 << log2B) - 1);
                    const int jj = (p >> log2B) & ((1 << log2b) - 1);
                    const int l1hi = p >> (log2B + log2b);
                    const int l1 = (l1hi << log2B) + l1lo;
                    Y[(l1hi << (log2n2 + log2B)) + ((j2_0 + jj) << log2B) + l1lo] =
                        mul(res[lds_at((jj << log2n1) + l1)], tw_grid_join(w[u], +1));
                }
            }
        }
    }
}

// Pass A of the FP64 form: the same transform as body_passA_fwd, each
// point's c_k / (n phi_hat(k')) formed once per workgroup and kept in the
// workgroup's own slot of the workspace (band's base_off), re-read for the
// other columns; every thread re-reads only what it wrote.  (FP64 registers
// would not hold a thread's bases beside its FFT values without spilling.)
template <class Ctx, typename T, int LOG2N>
FLT_HD void body_passA_fwd_slot(const Ctx& ctx, const PlanView<T>& pv, const FftItem* items,
                           const cplx<T>* c, cplx<T>* scratch, cplx<T>* basebuf, int deriv, int cols,
                           cplx<T>* lds, T* lc)
{
    using G = TwoPassGeo<T, LOG2N>;
    constexpr int ITEMS = tile_items<T>();
    constexpr int log2n1 = G::log2n1, log2n2 = G::log2n2, log2b = G::log2b, log2B = G::log2B;
    constexpr int LOG2N1 = log2n1;
    constexpr int P = tile_points<T>();
    constexpr int n = 1 << LOG2N;
    const FftItem it = items[ctx.bid()];
    const BandDesc B = pv.bands[it.band];   // a copy: the stores below cannot alias it
    const int k0 = (int)B.k0, kmax = (int)B.kmax;
    const int j2_0 = it.blk << log2b;
    // c_k / (n phi_hat(k')) of this workgroup's points: formed once, reading c
    // in address order (jj fastest) and transposing through LDS, then kept in
    // the workgroup's own slot for the other columns; every thread re-reads
    // only what it wrote.  Tile element p = (jj << log2n1) + j1.
    cplx<T>* slot = basebuf + B.base_off + (int64_t)it.blk * P;
    // FP32: twiddles in registers; FP64: from the table (its registers would
    // cost the second workgroup per CU)
    typename TwSel<sizeof(T) == 4, T, LOG2N1, (1 << log2b), +1>::type stw;
    stw.load(ctx, pv.tw_stage);
    // cols = 2: columns q .. 2q - 1 are the derivative's, the same interpolant
    // rows times 2 pi i k (base slot shared)
    for (int s = 0; s < cols * B.q; ++s) {
        const bool dcol = s >= B.q;
        stage_coef(ctx, pv, B, dcol ? s - B.q : s, lc);
        if (s == 0) {
#pragma unroll 1   // one point at a time: keeps the kernel at four waves per SIMD
            for (int i = 0; i < ITEMS; ++i) {
                const int p = ctx.tid() + i * FFT_THREADS;
                const int jj = p & ((1 << log2b) - 1);
                const int j1 = p >> log2b;
                const int j = j2_0 + jj + (j1 << log2n2);
                const int kp = j < (n >> 1) ? j : j - n;
                const int k = kp + k0;
                lds[lds_at((jj << log2n1) + j1)] =
                    k >= 1 && k <= kmax ? point_base(pv, B, c, kp, k, deriv) : mk<T>(0, 0);
            }
        }
        ctx.sync();
        // points in groups of GU: the group's bases are fetched first (for
        // s > 0 the slot reads are in flight together), then its Chebyshev rows
        // evaluated; k = 0 marks a point outside the support (half the grid),
        // whose input is zero
        constexpr int GU = sizeof(T) == 4 ? 8 : 2;
        auto point_k = [&](int p) {
            const int j1 = p & ((1 << log2n1) - 1);
            const int jj = p >> log2n1;
            const int j = j2_0 + jj + (j1 << log2n2);
            const int k = (j < (n >> 1) ? j : j - n) + k0;
            return k >= 1 && k <= kmax ? k : 0;
        };
        auto finish = [&](int i0, const cplx<T>* base, const int* kk) {
            for (int u = 0; u < GU; ++u) {
                const int p = ctx.tid() + (i0 + u) * FFT_THREADS;
                T w = kk[u] > 0 ? laplace_row_lds(lc, B, kk[u]) : T(0);
                cplx<T> b = base[u];
                if (dcol) {   // c'_k = 2 pi i k c_k
                    w *= (T)(6.283185307179586476925286766559 * (double)kk[u]);
                    b = mk(-b.y, b.x);
                }
                lds[lds_at(p)] = kk[u] > 0 ? scale(b, w) : mk<T>(0, 0);
            }
        };
        if (s == 0) {
#pragma unroll 1
            for (int i0 = 0; i0 < ITEMS; i0 += GU) {
                cplx<T> base[GU];
                int kk[GU];
                for (int u = 0; u < GU; ++u) {
                    const int p = ctx.tid() + (i0 + u) * FFT_THREADS;
                    kk[u] = point_k(p);
                    base[u] = lds[lds_at(p)];
                    if (kk[u] > 0) slot[p] = base[u];
                }
                finish(i0, base, kk);
            }
        } else {
#pragma unroll 1
            for (int i0 = 0; i0 < ITEMS; i0 += GU) {
                cplx<T> base[GU];
                int kk[GU];
                for (int u = 0; u < GU; ++u) {
                    const int p = ctx.tid() + (i0 + u) * FFT_THREADS;
                    kk[u] = point_k(p);
                    base[u] = kk[u] > 0 ? slot[p] : mk<T>(0, 0);
                }
                finish(i0, base, kk);
            }
        }
        ctx.sync();
        lds_fft_ct<Ctx, T, LOG2N1, (1 << log2b), +1>(ctx, lds, stw);
        cplx<T>* Y = scratch + B.scratch_off * cols + ((int64_t)s << LOG2N);
        // in groups of GO points: the group's table reads first (in flight
        // together), then the products and stores
        constexpr int GO = sizeof(T) == 4 ? 8 : 4;
#pragma unroll 1
        for (int i0 = 0; i0 < ITEMS; i0 += GO) {
            TwPair<T> w[GO];
            for (int u = 0; u < GO; ++u) {
                const int p = ctx.tid() + (i0 + u) * FFT_THREADS;
                const int l1lo = p & ((1 << log2B) - 1);
                const int jj = (p >> log2B) & ((1 << log2b) - 1);
                const int l1 = ((p >> (log2B + log2b)) << log2B) + l1lo;
                w[u] = tw_grid_fetch(pv, (uint32_t)(j2_0 + jj) * (uint32_t)l1, LOG2N);
            }
            for (int u = 0; u < GO; ++u) {
                const int p = ctx.tid() + (i0 + u) * FFT_THREADS;
                const int l1lo = p & ((1 << log2B) - 1);
                const int jj = (p >> log2B) & ((1 << log2b) - 1);
                const int l1hi = p >> (log2B + log2b);
                const int l1 = (l1hi << log2B) + l1lo;
                const int j2 = j2_0 + jj;
                Y[(l1hi << (log2n2 + log2B)) + (j2 << log2B) + l1lo] =
                    mul(lds[lds_at((jj << log2n1) + l1)], tw_grid_join(w[u], +1));
            }
        }
        ctx.sync();
    }
}

// The thread index, hidden from the optimiser once per loop iteration: in the
// persistent loops every per-thread address depends only on it, and hoisting
// all of them out of the loop (for every transform length) would exhaust the
// registers.  An empty asm statement on the value; no instruction is emitted.
FLT_HD int opaque(int v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+v"(v));
#else
    asm volatile("" : "+r"(v));
#endif
    return v;
}

template <class Ctx> struct IterCtx {
    const Ctx& c;
    int t;
    FLT_HD int tid() const { return t; }
    FLT_HD int ntid() const { return c.ntid(); }
    FLT_HD int bid() const { return c.bid(); }
    FLT_HD void sync() const { c.sync(); }
};

// pass B: for B = 2^log2B consecutive l1, the length-n2 DFTs over j2 of
// Y[j2][l1]; X[l1 + n1 l2] stored blocked as [l1 / B][l2][l1 mod B], only at
// the cells of the band's mask (the only ones a window reads).  Adjoint
// direction (SIGN = -1): grid -> scratch, only the masked cells are loaded,
// the others are zero.
//
// A tile's elements are held by the threads as rows of B consecutive HBM
// elements cut into runs of V = min(B, 8): element r < tile_items of a
// thread is row j2 = ch mod n2, column lo = (ch / n2) V + r mod V, with run
// ch = tid + (r / V) FFT_THREADS; lanes take consecutive rows, so the
// transposed LDS accesses are contiguous.
template <typename T, int LOG2N2> struct PassBGeo {
    static constexpr int log2n2 = LOG2N2, log2B = Sizes<T>::LOG2P - LOG2N2;
    static constexpr int log2V = log2B < 3 ? log2B : 3;
    static constexpr int V = 1 << log2V;
    FLT_HD static int ch(int tid, int r) { return tid + (r >> log2V) * FFT_THREADS; }
    FLT_HD static int row(int ch) { return ch & ((1 << log2n2) - 1); }
    FLT_HD static int col(int ch, int r) { return ((ch >> log2n2) << log2V) + (r & (V - 1)); }
};

// A pass-B tile held in registers, tile_items<T>() values per thread: complex
// pairs for FP32, separate real and imaginary parts for FP64 (the form the
// compiler keeps in registers rather than in scratch memory).
template <typename T> struct TileRegs;
template <> struct TileRegs<float> {
    cplx<float> v[tile_items<float>()];
    FLT_HD void set(int r, cplx<float> x) { v[r] = x; }
    FLT_HD cplx<float> get(int r) const { return v[r]; }
};
template <> struct TileRegs<double> {
    double re[tile_items<double>()], im[tile_items<double>()];
    FLT_HD void set(int r, cplx<double> x) { re[r] = x.x; im[r] = x.y; }
    FLT_HD cplx<double> get(int r) const { return mk(re[r], im[r]); }
};

// Load item `it`'s tile into the registers v; in the adjoint direction (ADJ:
// grid -> scratch) the cells outside the band's read mask (never written) as
// zeros.
template <class Ctx, typename T, int LOG2N2, bool ADJ>
FLT_HD void passB_fetch(const Ctx& ctx, const PlanView<T>& pv, const FftItem& it, const cplx<T>* src_base,
                        int cols, TileRegs<T>& v)
{
    using G = PassBGeo<T, LOG2N2>;
    const BandDesc& B = pv.bands[it.band];
    const int64_t blk_off = ((int64_t)it.s0 << B.log2n) + ((int64_t)it.blk << Sizes<T>::LOG2P);
    const cplx<T>* src = src_base + (ADJ ? B.grid_off : B.scratch_off) * cols + blk_off;
    const uint32_t* mask = pv.mask + B.mask_off + ((int64_t)it.blk << (Sizes<T>::LOG2P - 5));
    for (int m = 0; m < tile_items<T>() / G::V; ++m) {
        const int ch = ctx.tid() + m * FFT_THREADS;
        const int p0 = (G::row(ch) << G::log2B) + G::col(ch, 0);   // multiple of V: one mask word
        if (ADJ) {
            // FP32: runs holding a cell some window wrote are read whole, in
            // 16-byte pairs (V even, p0 a multiple of V), and the cells no
            // window wrote are zeroed
            const uint32_t b = mask[p0 >> 5] >> (p0 & 31);
            if constexpr (sizeof(T) == 4 && G::V >= 2) {
                if (b & ((1u << G::V) - 1u)) {
                    for (int u = 0; u < G::V; u += 2) {
                        const cplx2<T> pr = load_pair(src + p0 + u);
                        v.set(m * G::V + u, ((b >> u) & 1u) ? pr.a : mk<T>(0, 0));
                        v.set(m * G::V + u + 1, ((b >> (u + 1)) & 1u) ? pr.b : mk<T>(0, 0));
                    }
                } else {
                    for (int u = 0; u < G::V; ++u) v.set(m * G::V + u, mk<T>(0, 0));
                }
            } else {
                for (int u = 0; u < G::V; ++u) v.set(m * G::V + u, ((b >> u) & 1u) ? src[p0 + u] : mk<T>(0, 0));
            }
        } else {
            for (int u = 0; u < G::V; ++u) v.set(m * G::V + u, src[p0 + u]);
        }
    }
}

// Whether the pass-B variant prefetches the next tile during the current
// FFT: the FP32 forward, the one whose registers hold the extra tile within
// four waves per SIMD.  The others are launched one workgroup per item.
template <typename T, int SIGN> constexpr bool passB_prefetch() { return sizeof(T) == 4 && SIGN > 0; }

// Pass-B items of one transform length, as long as the workgroup's next item
// has that length: each tile is in the registers (vr, vi) before its FFT; with
// prefetch the next item's tile is fetched right after this one went to LDS,
// so its loads are in flight while this tile is transformed.  Returns the
// index of the workgroup's first item not processed.
template <class Ctx, typename T, int LOG2N2, int SIGN>
FLT_HD int passB_run(const Ctx& ctx0, const PlanView<T>& pv, const FftItem* items, int i, int nitems, int nblocks,
                     const cplx<T>* src_base, cplx<T>* dst_base, int cols, cplx<T>* lds, cplx<T>* twl)
{
    constexpr bool ADJ = SIGN < 0;
    constexpr bool PREFETCH = passB_prefetch<T, SIGN>();
    using G = PassBGeo<T, LOG2N2>;
    constexpr int CHUNKS = tile_points<T>() / G::V;
    TileRegs<T> v;
    passB_fetch<Ctx, T, LOG2N2, ADJ>(ctx0, pv, items[i], src_base, cols, v);
    // with prefetch the registers hold the next tile instead of the twiddles,
    // which come from a half table in LDS (written here, read after the
    // barrier that follows the first tile's store to LDS; the previous run's
    // readers finished at its last barrier)
    using TwP = typename std::conditional<PREFETCH, LdsTw<T, LOG2N2>,
                                          typename TwSel<true, T, LOG2N2, (1 << G::log2B), SIGN>::type>::type;
    TwP stw;
    if constexpr (PREFETCH) stw.fill(ctx0, pv.tw_stage, twl);
    else stw.load(ctx0, pv.tw_stage);
    for (;;) {
        const IterCtx<Ctx> ctx{ctx0, opaque(ctx0.tid())};
        const FftItem it = items[i];
        const BandDesc& B = pv.bands[it.band];
        for (int r = 0; r < tile_items<T>(); ++r) {
            const int ch = G::ch(ctx.tid(), r);
            lds[lds_at((G::col(ch, r) << LOG2N2) + G::row(ch))] = v.get(r);
        }
        ctx.sync();
        const int nx = i + nblocks;
        const bool more = nx < nitems && pv.bands[items[nx].band].log2n2 == LOG2N2;
        if (PREFETCH && more)
            passB_fetch<IterCtx<Ctx>, T, LOG2N2, ADJ>(ctx, pv, items[nx], src_base, cols, v);
        lds_fft_ct<IterCtx<Ctx>, T, LOG2N2, (1 << G::log2B), SIGN>(ctx, lds, stw);
        const int64_t blk_off = ((int64_t)it.s0 << B.log2n) + ((int64_t)it.blk << Sizes<T>::LOG2P);
        cplx<T>* dst = dst_base + (ADJ ? B.scratch_off : B.grid_off) * cols + blk_off;
        const uint32_t* mask = pv.mask + B.mask_off + ((int64_t)it.blk << (Sizes<T>::LOG2P - 5));
        for (int t = ctx.tid(); t < CHUNKS; t += FFT_THREADS) {
            const int l2 = t & ((1 << LOG2N2) - 1);
            const int lo0 = (t >> LOG2N2) * G::V;
            const int p0 = (l2 << G::log2B) + lo0;
            const uint32_t keep = ADJ ? ~0u : mask[p0 >> 5] >> (p0 & 31);
            constexpr uint32_t full = G::V >= 32 ? ~0u : (1u << G::V) - 1u;
            if (sizeof(T) == 4 && G::V >= 2 && (keep & full) == full) {   // FP32, a whole run: pair stores
                for (int u = 0; u < G::V; u += 2) {
                    cplx2<T> pr;
                    pr.a = lds[lds_at(((lo0 + u) << LOG2N2) + l2)];
                    pr.b = lds[lds_at(((lo0 + u + 1) << LOG2N2) + l2)];
                    store_pair(dst + p0 + u, pr);
                }
            } else {
                for (int u = 0; u < G::V; ++u)
                    if ((keep >> u) & 1u) dst[p0 + u] = lds[lds_at(((lo0 + u) << LOG2N2) + l2)];
            }
        }
        ctx.sync();
        i = nx;
        if (!PREFETCH || !more) return i;
    }
}

// Persistent pass B: workgroup g takes items g, g + nblocks, g + 2 nblocks, ...
// (forward: scratch -> grids, SIGN = +1; adjoint: grids -> scratch, SIGN = -1).
template <class Ctx, typename T, int SIGN>
FLT_HD void body_passB(const Ctx& ctx, const PlanView<T>& pv, const FftItem* items, int nitems, int nblocks,
                       const cplx<T>* src_base, cplx<T>* dst_base, int cols, cplx<T>* lds, cplx<T>* twl)
{
    using RG = Log2Range<T>;
    int i = ctx.bid();
    if constexpr (!passB_prefetch<T, SIGN>()) {   // one item per workgroup (nblocks = nitems)
        if (i < nitems)
            with_log2<RG::B_LO, RG::B_HI>(pv.bands[items[i].band].log2n2, [&](auto LG) {
                passB_run<Ctx, T, decltype(LG)::value, SIGN>(ctx, pv, items, i, nitems, nitems, src_base, dst_base,
                                                             cols, lds, twl);
            });
        return;
    }
    while (i < nitems) {
        with_log2<RG::B_LO, RG::B_HI>(pv.bands[items[i].band].log2n2, [&](auto LG) {
            i = passB_run<Ctx, T, decltype(LG)::value, SIGN>(ctx, pv, items, i, nitems, nblocks, src_base, dst_base,
                                                             cols, lds, twl);
        });
    }
}

// ---------------------------------------------------------------------------
// Window and node weights
// ---------------------------------------------------------------------------
// Hardware reciprocal, square root and 2^x in FP32 (about 1 ulp); the CPU
// build uses the correctly rounded library forms.
FLT_HD float rcp_f32(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
FLT_HD float sqrt_f32(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}
FLT_HD float exp2_f32(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(x);
#else
    return exp2f(x);
#endif
}
FLT_HD float rsq_f32(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsqf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}
// sin(2 pi r) and cos(2 pi r) for a phase r given in revolutions (|r| a little
// above 1/2 at most): the hardware's revolution-based sine and cosine, which on
// gfx950 stay within 1.3e-7 absolute over [-1/2, 1/2] (measured against FP64;
// sincosf of the FP32 product 2 pi r, 2.1e-7).  The CPU build rounds the FP64
// values.
FLT_HD void sincos_rev_f32(float r, float* s, float* c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
#else
    *s = (float)sin(6.283185307179586476925286766559 * (double)r);
    *c = (float)cos(6.283185307179586476925286766559 * (double)r);
#endif
}

// Kaiser-Bessel window at grid offsets u_t = delta + mw - 1 - t, t < 2 mw:
// phi = sinh(b v) / (pi v), v = sqrt(mw^2 - u^2).  FP32: sinh(b v) =
// (e - 1/e) / 2 with e = 2^(b log2(e) v); the cancellation for small b v only
// touches the edge taps, whose weights are about 1e-9 of the central ones.
// The inner taps (0 < t < 2 mw - 1) have |u| <= mw - 1, so v >= sqrt(2 mw - 1)
// and, with the integer grids' b = 3 pi / 2 and mw >= 3, 1/e^2 < 1e-9: there
// the window is e / (2 pi v), from one reciprocal square root and one 2^x.
template <typename T, int MW>
FLT_HD void kb_weights(T delta, T b, T* phi)
{
    const T inv_pi = T(0.31830988618379067153776752674503);
    if constexpr (sizeof(T) == 4) {
        const float bl2e = b * 1.4426950408889634f;
        for (int t = 0; t < 2 * MW; ++t) {
            const float u = delta + float(MW - 1 - t);
            const float v2 = float(MW * MW) - u * u;
            if (MW >= 3 && t > 0 && t < 2 * MW - 1) {
                const float r = rsq_f32(v2);
                phi[t] = exp2_f32(bl2e * (v2 * r)) * (0.5f * inv_pi) * r;
            } else {
                const float v = v2 > 0.0f ? sqrt_f32(v2) : 0.0f;
                const float e = exp2_f32(bl2e * v);
                phi[t] = v > 0.0f ? (e - rcp_f32(e)) * (0.5f * inv_pi) * rcp_f32(v) : b * inv_pi;
            }
        }
    } else {
        for (int t = 0; t < 2 * MW; ++t) {
            const T u = delta + T(MW - 1 - t);
            const T v2 = T(MW * MW) - u * u;
            const T v = v2 > T(0) ? (T)sqrt(v2) : T(0);
            phi[t] = v > T(0) ? (T)sinh(b * v) / v * inv_pi : b * inv_pi;
        }
    }
}

// Barycentric weights on the band's q Chebyshev nodes (Sect. 2):
// L_s(y) = (lambda_s / (y - y_s)) / sum_r lambda_r / (y - y_r); a node hit gives
// the Kronecker delta.  bary_setup returns 1/sum (or 0 with hit set).  FP64
// for the FP64 form; FP32 for the FP32 form, from the differences y - y_s
// formed in FP64 (the second barycentric form is stable at Chebyshev nodes,
// also for y next to a node).
template <typename W> struct BaryY {
    W inv;
    int hit;
};
template <typename W> FLT_HD BaryY<W> bary_setup(const double* yc, int q, double y)
{
    BaryY<W> r;
    r.hit = -1;
    W sum = 0;
    for (int s = 0; s < q; ++s) {
        const double d = y - yc[2 * s];
        if (d == 0.0) r.hit = s;
        else if constexpr (sizeof(W) == 4) sum += (float)yc[2 * s + 1] * rcp_f32((float)d);
        else sum += yc[2 * s + 1] / d;
    }
    if constexpr (sizeof(W) == 4) r.inv = r.hit >= 0 ? 0.0f : rcp_f32(sum);
    else r.inv = r.hit >= 0 ? 0.0 : 1.0 / sum;
    return r;
}
template <typename W> FLT_HD W bary_at(const double* yc, const BaryY<W>& b, int s, double y)
{
    if (b.hit >= 0) return s == b.hit ? W(1) : W(0);
    if constexpr (sizeof(W) == 4) return (float)yc[2 * s + 1] * rcp_f32((float)(y - yc[2 * s])) * b.inv;
    else return yc[2 * s + 1] / (y - yc[2 * s]) * b.inv;
}

// e^{sign 2 pi i k0 x} for a band centre k0 (0 or a power of two, so k0 x and
// its fraction are exact in FP64); the sine and cosine of the reduced phase
// in FP64 for the FP64 form, FP32 for the FP32 form.
template <typename T> FLT_HD void modulation(double k0, double x, double* cs, double* sn)
{
    double ph = k0 * x;
    ph -= rint(ph);   // in [-1/2, 1/2]
    if constexpr (sizeof(T) == 4) {
        float s, c;
        sincos_rev_f32((float)ph, &s, &c);
        *cs = c;
        *sn = s;
    } else {
        sincos(6.283185307179586476925286766559 * ph, sn, cs);
    }
}

// ---------------------------------------------------------------------------
// a5 + a6: per node, gather the window from the q grids, weight by L_s(y),
// sum in FP64, modulate by e^{2 pi i k0 x} and add c0.
// ---------------------------------------------------------------------------
// f2 != null (cols = 2): columns q .. 2q - 1 of each band hold the derivative
// transform's grids, whose sums go to f2 (no c_0 term: c'_0 = 0).
//
// A workgroup's nodes are consecutive in the band's sorted order, so their
// windows cover one run of the grid: the cells from l0(first) - mw + 1 to
// l0(last) + mw.  The planner sorts the items by that run's length: when it is
// short (dense bands: many nodes per cell) the workgroup loads it once per
// column, coalesced, into LDS (as many columns at a time as GATHER_STAGE
// values hold) and every node reads its taps there (STAGED); otherwise each
// node loads its own taps from the grid.  The two are separate kernels, each
// compiled for its own path.
template <class Ctx, typename T, int MW, bool STAGED>
FLT_HD void body_gather(const Ctx& ctx, const PlanView<T>& pv, const NodeItem* items, const cplx<T>* c,
                        const cplx<T>* grids, cplx<T>* f, int with_c0, cplx<T>* f2, cplx<T>* stage)
{
    const NodeItem it = items[ctx.bid()];
    const int i = ctx.tid();
    const bool active = i < it.count;
    const int64_t jj = it.start + (active ? i : 0);
    const BandDesc& B = pv.bands[it.band];
    const double c0r = with_c0 ? (double)c[B.c_off].x : 0.0;
    const double c0i = with_c0 ? (double)c[B.c_off].y : 0.0;
    if (!STAGED && B.q == 0) {   // the constant band (the whole item)
        if (active) {
            const int32_t dst = pv.perm[jj];
            f[dst] = mk<T>((T)c0r, (T)c0i);
            if (f2) f2[dst] = mk<T>(0, 0);
        }
        return;
    }
    const double x = pv.nx[jj], y = pv.ny[jj];
    const int log2n = B.log2n;
    const int nmask = (1 << log2n) - 1;
    const double nxv = ldexp(x, log2n);
    const double fl = floor(nxv);
    const int l0 = (int)fl;
    T phi[2 * MW];
    kb_weights<T, MW>((T)(nxv - fl), pv.kb_b, phi);
    const double* yc = pv.ycheb + 2 * B.ycheb_off;
    // Barycentric weighting in the second form (Sect. 2), summed along with
    // the columns: sum_s L_s(y) F_s = sum_s w_s F_s / sum_s w_s with
    // w_s = lambda_s / (y - y_s); a node on a Chebyshev node y_s takes F_s.
    // The weights are FP32 in the FP32 form (from y - y_s formed in FP64), the
    // sums FP64.
    T wsum = 0;
    int hit = -1;
    double ar = 0, ai = 0, dr = 0, di = 0, hr = 0, hi = 0, hdr = 0, hdi = 0;
    auto accumulate = [&](int s, T fr, T fi) {
        const bool dcol = s >= B.q;   // a derivative column (f2): weight of column s - q
        const int sb = dcol ? s - B.q : s;
        const double d = y - yc[2 * sb];
        T w;
        if constexpr (sizeof(T) == 4) w = (float)yc[2 * sb + 1] * rcp_f32((float)d);
        else w = yc[2 * sb + 1] / d;
        if (d == 0.0) {
            w = 0;
            hit = sb;
            if (dcol) {
                hdr = fr;
                hdi = fi;
            } else {
                hr = fr;
                hi = fi;
            }
        }
        if (dcol) {
            dr += (double)w * (double)fr;
            di += (double)w * (double)fi;
        } else {
            wsum += w;
            ar += (double)w * (double)fr;
            ai += (double)w * (double)fi;
        }
    };
    // grid address of cell l (one-pass bands: natural order; two-pass: pass B's
    // output layout Y[l1 / B][l2][l1 mod B], l = l1 + n1 l2)
    const int lb = B.log2n2 > 0 ? B.log2B : 30;
    const int l1m = (1 << B.log2n1) - 1, bm = (1 << lb) - 1;
    auto addr_of = [&](int l) {
        const int l1 = l & l1m, l2 = l >> B.log2n1;
        return B.log2n2 > 0 ? ((l1 >> lb) << (B.log2n2 + lb)) + (l2 << lb) + (l1 & bm) : l;
    };
    const cplx<T>* g = grids + B.grid_off * (f2 ? 2 : 1);
    const int ncol = f2 ? 2 * B.q : B.q;
    if constexpr (STAGED) {
        // the workgroup's run of cells (uniform: first and last node of the
        // item; the planner placed the item here because it fits the stage)
        const int lf = (int)floor(ldexp(pv.nx[it.start], log2n));
        const int ll = (int)floor(ldexp(pv.nx[it.start + it.count - 1], log2n));
        const int span = ll - lf + 2 * MW;
        if (span > GATHER_STAGE) {   // not a staged item: NaN, never LDS out of bounds
            if (active) {
                const T nan = T(__builtin_nan(""));
                f[pv.perm[jj]] = mk<T>(nan, nan);
                if (f2) f2[pv.perm[jj]] = mk<T>(nan, nan);
            }
            return;
        }
        const int base = lf - MW + 1;
        const int off = l0 - lf;   // in [0, span - 2 mw] (sorted nodes)
        const int per = GATHER_STAGE / span;
        // thread i loads stage elements e = i, i + GATHER_THREADS, ...: column
        // cc = e / span, cell r = e mod span, stepped without divisions
        const int cc0 = i / span, r0 = i - cc0 * span;
        const int step_c = GATHER_THREADS / span, step_r = GATHER_THREADS - step_c * span;
        for (int s0 = 0; s0 < ncol; s0 += per) {
            const int nc = ncol - s0 < per ? ncol - s0 : per;
            if (s0 > 0) ctx.sync();   // the previous columns' reads are done
            int cc = cc0, r = r0;
            for (int e = i; e < nc * span; e += GATHER_THREADS) {
                stage[e] = g[((int64_t)(s0 + cc) << log2n) + addr_of((base + r) & nmask)];
                cc += step_c;
                r += step_r;
                if (r >= span) {
                    r -= span;
                    ++cc;
                }
            }
            ctx.sync();
            if (active) {
                for (int cc = 0; cc < nc; ++cc) {
                    const cplx<T>* st = stage + cc * span + off;
                    T fr = 0, fi = 0;
                    for (int t = 0; t < 2 * MW; ++t) {
                        const cplx<T> v = st[t];
                        fr += v.x * phi[t];
                        fi += v.y * phi[t];
                    }
                    accumulate(s0 + cc, fr, fi);
                }
            }
        }
    } else if (active) {
        if constexpr (sizeof(T) == 4) {
            // FP32: the window's cells c0 .. c0 + 2 mw - 1 (c0 = l0 - mw + 1)
            // read as mw + 1 aligned pairs from the even cell at or below c0
            // (both layouts keep an even cell and its successor adjacent, at an
            // even offset); the weights shift by the parity of c0, not the values.
            // The pairs' two cells outside the window (c0 - 1 and c0 + 2 mw for
            // odd c0; the whole last pair for even c0, which is not read) may be
            // cells pass B never wrote: they are replaced by 0, not multiplied
            // by a zero weight.
            const int c0 = (l0 - MW + 1) & nmask;
            const int par = c0 & 1, e0 = c0 - par;
            T phi2[2 * MW + 2];
            for (int j = 0; j < 2 * MW + 2; ++j) {
                const T lo = j < 2 * MW ? phi[j] : T(0);
                const T hi2 = j >= 1 && j - 1 < 2 * MW ? phi[j - 1] : T(0);
                phi2[j] = par ? hi2 : lo;
            }
            int paddr[MW + 1];
            for (int k = 0; k <= MW; ++k) paddr[k] = addr_of((e0 + 2 * k) & nmask);
            // two columns' loads in flight
#pragma unroll 2
            for (int s = 0; s < ncol; ++s) {
                const cplx<T>* gs = g + ((int64_t)s << log2n);
                T fr = 0, fi = 0;
                for (int k = 0; k <= MW; ++k) {
                    cplx2<T> v;
                    if (k < MW || par) v = load_pair(gs + paddr[k]);
                    else v.a = mk<T>(0, 0);
                    if (k == 0 && par) v.a = mk<T>(0, 0);
                    if (k == MW) v.b = mk<T>(0, 0);
                    fr += v.a.x * phi2[2 * k] + v.b.x * phi2[2 * k + 1];
                    fi += v.a.y * phi2[2 * k] + v.b.y * phi2[2 * k + 1];
                }
                accumulate(s, fr, fi);
            }
        } else {
            // offsets within a column (a grid has at most 2^22 points)
            int addr[2 * MW];
            for (int t = 0; t < 2 * MW; ++t) addr[t] = addr_of((l0 - MW + 1 + t) & nmask);
            for (int s = 0; s < ncol; ++s) {
                const cplx<T>* gs = g + ((int64_t)s << log2n);
                T fr = 0, fi = 0;
                for (int t = 0; t < 2 * MW; ++t) {
                    const cplx<T> v = gs[addr[t]];
                    fr += v.x * phi[t];
                    fi += v.y * phi[t];
                }
                accumulate(s, fr, fi);
            }
        }
    }
    if (!active) return;
    if (hit >= 0) {
        ar = hr;
        ai = hi;
        dr = hdr;
        di = hdi;
    } else {
        double inv;
        if constexpr (sizeof(T) == 4) inv = (double)rcp_f32(wsum);
        else inv = 1.0 / wsum;
        ar *= inv;
        ai *= inv;
        dr *= inv;
        di *= inv;
    }
    const int32_t dst = pv.perm[jj];
    double sn, cs;
    modulation<T>((double)B.k0, x, &cs, &sn);   // e^{2 pi i k0 x}
    f[dst] = mk<T>((T)(c0r + ar * cs - ai * sn), (T)(c0i + ar * sn + ai * cs));
    if (f2) f2[dst] = mk<T>((T)(dr * cs - di * sn), (T)(dr * sn + di * cs));
}

// ---------------------------------------------------------------------------
// Adjoint a7, node side: per node of an NFFT band, u_j^s = g_j e^{-2 pi i k0 x_j}
// L_s(y_j) (FP64, rounded to T), the window weights of its 2 mw taps and its cell.
// ---------------------------------------------------------------------------
template <class Ctx, typename T, int MW>
FLT_HD void body_adj_prep(const Ctx& ctx, const PlanView<T>& pv, const NodeItem* items, const cplx<T>* gin,
                          int qs, cplx<T>* U, T* Phi, int32_t* L0)
{
    const NodeItem it = items[ctx.bid()];
    const int i = ctx.tid();
    if (i >= it.count) return;
    const int64_t j = it.start + i;
    const BandDesc& B = pv.bands[it.band];
    const double x = pv.nx[j], y = pv.ny[j];
    const double nxv = ldexp(x, B.log2n);
    const double fl = floor(nxv);
    L0[j] = (int32_t)fl;
    T phi[2 * MW];
    kb_weights<T, MW>((T)(nxv - fl), pv.kb_b, phi);
    for (int t = 0; t < 2 * MW; t += 2) {   // tap pairs (8-byte aligned in FP32, 16 in FP64)
        RealPair<T> pr;
        pr.a = phi[t];
        pr.b = phi[t + 1];
        *reinterpret_cast<RealPair<T>*>(Phi + j * (2 * MW) + t) = pr;
    }
    const cplx<T> gv = gin[pv.perm[j]];
    double sn, cs;
    modulation<T>((double)B.k0, x, &cs, &sn);
    const double ur = (double)gv.x * cs + (double)gv.y * sn;   // g e^{-2 pi i k0 x}
    const double ui = (double)gv.y * cs - (double)gv.x * sn;
    const double* yc = pv.ycheb + 2 * B.ycheb_off;
    const BaryY<T> by = bary_setup<T>(yc, B.q, y);
    // column pairs (the row stride qs is even; a padding column gets 0)
    for (int s = 0; s < B.q; s += 2) {
        const double L0s = (double)bary_at<T>(yc, by, s, y);
        const double L1s = s + 1 < B.q ? (double)bary_at<T>(yc, by, s + 1, y) : 0.0;
        cplx2<T> v;
        v.a = mk<T>((T)(ur * L0s), (T)(ui * L0s));
        v.b = mk<T>((T)(ur * L1s), (T)(ui * L1s));
        store_pair(U + j * qs + s, v);
    }
}

// Adjoint a7, grid side (no atomics): cell l of each column of band B
// receives sum_j u_j^s phi(n x_j - l) over the nodes whose window covers l.
// Nodes are sorted by cell l0 = floor(n x), and l is covered iff l0 lies in
// [l - mw, l + mw) (mod n), so the contributors form at most two runs of the
// sorted order, found in the band's cell-start table.  Each cell is summed by
// a group of 2^log2tpc threads (sized by the band's node density) that split
// its runs: every contributor's weight is read once per ADJ_QC columns, which
// are summed in registers and reduced through LDS, ADJ_RC columns at a time.  Cells of two-pass bands that no window
// reads are skipped (pass B loads only masked cells); one-pass bands get
// every cell, zeros included.
template <typename T> constexpr int ADJ_QC() { return sizeof(T) == 4 ? 12 : 8; }
constexpr int ADJ_RC = 4;

template <class Ctx, typename T, int MW>
FLT_HD void body_adj_cells(const Ctx& ctx, const PlanView<T>& pv, const CellItem* items, int qs,
                           const cplx<T>* U, const T* Phi, const int32_t* L0, const int32_t* cstart,
                           const int32_t* clist, cplx<T>* grids, T* red)
{
    const CellItem it = items[ctx.bid()];
    const BandDesc& B = pv.bands[it.band];
    const int n = 1 << B.log2n;
    const int lt = it.log2tpc, tpc = 1 << lt;
    const int tid = ctx.tid();
    const int r = tid & (tpc - 1);
    const int l = it.listed ? clist[it.cell0 + (tid >> lt)] : it.cell0 + (tid >> lt);
    bool write = l >= 0 && l < n;
    int64_t addr = 0;
    if (write) {
        addr = grid_addr(B, l);
        if (B.log2n2 > 0 && !((pv.mask[B.mask_off + (addr >> 5)] >> (addr & 31)) & 1u)) write = false;
    }
    int32_t r0s = 0, r0e = 0, r1s = 0, r1e = 0;
    if (write) {
        const int32_t* c0 = cstart + B.cs_off;   // c0[c]: first sorted node of the band with cell >= c
        const int a = l - MW, b = l + MW;
        if (a < 0) { r0s = c0[a + n]; r0e = c0[n]; r1s = c0[0]; r1e = c0[b]; }
        else if (b > n) { r0s = c0[a]; r0e = c0[n]; r1s = c0[0]; r1e = c0[b - n]; }
        else { r0s = c0[a]; r0e = c0[b]; }
    }
    cplx<T> * const g = grids + B.grid_off;
    for (int s0 = 0; s0 < B.q; s0 += ADJ_QC<T>()) {
        constexpr int QC = ADJ_QC<T>(), RC = ADJ_RC;
        T ar[QC], ai[QC];
        for (int c = 0; c < QC; ++c) ar[c] = ai[c] = 0;
        for (int run = 0; run < 2; ++run) {
            const int32_t js = run ? r1s : r0s, je = run ? r1e : r0e;
            for (int32_t j = js + r; j < je; j += tpc) {
                int t = l - L0[j] + (MW - 1);   // tap index of l in node j's window
                if (t < 0) t += n;
                if (t >= n) t -= n;
                const T w = Phi[(int64_t)j * (2 * MW) + t];
                const cplx<T>* u = U + (int64_t)j * qs + s0;
                // column pairs, one 16-byte load each in FP32 (QC and qs even;
                // a padding column's sum is never stored)
                for (int c = 0; c < QC; c += 2)
                    if (s0 + c < B.q) {
                        const cplx2<T> uv = load_pair(u + c);
                        ar[c] += uv.a.x * w;
                        ai[c] += uv.a.y * w;
                        ar[c + 1] += uv.b.x * w;
                        ai[c + 1] += uv.b.y * w;
                    }
            }
        }
        if (tpc > 1) {                           // uniform over the workgroup
            for (int c0 = 0; c0 < QC; c0 += RC) {
                for (int c = 0; c < RC; ++c) {
                    red[2 * (tid * RC + c)] = ar[c0 + c];
                    red[2 * (tid * RC + c) + 1] = ai[c0 + c];
                }
                ctx.sync();
                for (int h = tpc >> 1; h > 0; h >>= 1) {
                    if (r < h)
                        for (int c = 0; c < RC; ++c) {
                            red[2 * (tid * RC + c)] += red[2 * ((tid + h) * RC + c)];
                            red[2 * (tid * RC + c) + 1] += red[2 * ((tid + h) * RC + c) + 1];
                        }
                    ctx.sync();
                }
                for (int c = 0; c < RC; ++c) {
                    ar[c0 + c] = red[2 * (tid * RC + c)];
                    ai[c0 + c] = red[2 * (tid * RC + c) + 1];
                }
                ctx.sync();
            }
        }
        if (write && r == 0)
            for (int c = 0; c < QC; ++c)
                if (s0 + c < B.q) g[((int64_t)(s0 + c) << B.log2n) + addr] = mk(ar[c], ai[c]);
    }
}

// sum_j g_j over a run of one instance's nodes (the k = 0 coefficient of the
// adjoint), FP64, into that instance's acc[0..1].
template <class Ctx, typename T>
FLT_HD void body_sum_g(const Ctx& ctx, const PlanView<T>& pv, const SumItem* items, const cplx<T>* g, double* acc,
                       double* red)
{
    const int tid = ctx.tid(), nt = ctx.ntid();
    const SumItem it = items[ctx.bid()];
    const InstDesc I = pv.inst[it.inst];
    const int64_t end = I.f_off + I.M;
    double sr = 0, si = 0;
    for (int t = 0; t < SUMG_PER_THREAD; ++t) {
        const int64_t i = it.start + (int64_t)t * nt + tid;
        if (i < end) {
            sr += (double)g[i].x;
            si += (double)g[i].y;
        }
    }
    red[2 * tid] = sr;
    red[2 * tid + 1] = si;
    ctx.sync();
    for (int h = nt >> 1; h > 0; h >>= 1) {
        if (tid < h) {
            red[2 * tid] += red[2 * (tid + h)];
            red[2 * tid + 1] += red[2 * (tid + h) + 1];
        }
        ctx.sync();
    }
    if (tid == 0) {
        ctx.atomic_add(acc + 2 * I.c_off, red[0]);
        ctx.atomic_add(acc + 2 * I.c_off + 1, red[1]);
    }
}

// ---------------------------------------------------------------------------
// Bands the plan evaluates by the direct sum (few nodes, large grids): the
// exact f_j = sum_{k<N} c_k w_j^k.  Every thread takes DIRECT_TPT consecutive
// terms k0 .. k0 + DIRECT_TPT - 1: forward, w^{k0} sum_t c_{k0+t} w^t with the
// inner sum by Horner's scheme in T and the anchor w^{k0} formed directly;
// adjoint, the powers by the recurrence p <- p w from the anchor.  Partial
// sums are combined in FP64.  A forward workgroup holds DIRECT_NG nodes (their
// w in LDS, then registers) and up to direct_cpw chunks of terms, reduced
// once; a thread runs the Horner recurrences of its group's nodes side by
// side (independent chains: all 8 in FP32, fewer in FP64), the derivative's
// 2 pi i k factors, applied as c is loaded, only in the DERIV instance.  For
// short sums (GROUPED) the workgroup is several such groups of 2^log2tpg
// threads, each with its own DIRECT_NG nodes and one 32-term piece per thread.
// ---------------------------------------------------------------------------

// w^k0 = e^{-k0 y} cis(sign 2 pi k0 x) with the phase reduced exactly in FP64
// (frac_kx, |phase| <= pi); FP32 plans evaluate the sine and cosine of the
// reduced phase and 2^(-k0 y log2 e) (exponent formed in FP64) in FP32, FP64
// plans everything in FP64.
template <typename T>
FLT_HD cplx<T> direct_anchor(double k0, double x, double y, double sign)
{
    const double r = frac_kx(k0, x);
    if constexpr (sizeof(T) == 4) {
        float sn, cs;
        sincos_rev_f32((float)(sign * r), &sn, &cs);
        const float mag = exp2_f32((float)(-k0 * y * 1.4426950408889634074));
        return mk(mag * cs, mag * sn);
    } else {
        double sn, cs;
        sincos(sign * 6.283185307179586476925286766559 * r, &sn, &cs);
        const double mag = exp(-k0 * y);
        return mk(mag * cs, mag * sn);
    }
}

// w = e^{-y} cis(sign 2 pi x) of sorted node j, in FP64, rounded to T.
template <typename T> FLT_HD cplx<T> direct_w(const PlanView<T>& pv, int32_t j, double sign)
{
    double sn, cs;
    sincos(sign * 6.283185307179586476925286766559 * pv.nx[j], &sn, &cs);
    const double m1 = exp(-pv.ny[j]);
    return mk<T>((T)(m1 * cs), (T)(m1 * sn));
}

template <class Ctx, typename T, bool DERIV, bool GROUPED>
FLT_HD void body_direct_fwd(const Ctx& ctx, const PlanView<T>& pv, const DirectItem* items, const int32_t* dlist,
                            const cplx<T>* call, double* dacc, double* red, cplx<T>* nw)
{
    const DirectItem it = items[ctx.bid()];
    const int64_t N = pv.inst[it.inst].N;
    const cplx<T>* c = call + pv.inst[it.inst].c_off;
    const int tid = ctx.tid(), nt = ctx.ntid();
    // thread groups of 2^lt threads, each with DIRECT_NG nodes of the run: one
    // group spanning the workgroup for long sums; several (GROUPED) for short
    // ones, whose terms would leave most threads idle
    const int lt = GROUPED ? it.log2tpg : 8, tpg = 1 << lt;
    const int ng = GROUPED ? ((nt >> lt) < DIRECT_GMAX ? (nt >> lt) : DIRECT_GMAX) : 1;   // groups
    const int grp = GROUPED ? tid >> lt : 0, r = GROUPED ? tid & (tpg - 1) : tid;
    const int gfirst = grp * DIRECT_NG;         // the group's first node in the run
    for (int e = tid; e < DIRECT_NG * ng; e += nt)
        nw[e] = e < it.count ? direct_w(pv, dlist[it.first + e], +1.0) : mk<T>(0, 0);
    for (int q = 0; q < 2 * DIRECT_NG; ++q) red[q * nt + tid] = 0.0;   // this thread's partial sums
    ctx.sync();
    const int gcount = it.count - gfirst;       // the group's nodes (<= 0: none)
    // Horner chains side by side (registers): all 8 nodes in FP32, 4 at a time
    // for the FP64 forward, one at a time for the FP64 derivative
    constexpr int NC = sizeof(T) == 4 ? DIRECT_NG : DERIV ? 1 : DIRECT_NG / 2;
    for (int cc = 0; cc < it.nch && gcount > 0; ++cc) {
        const int64_t k0 = (GROUPED ? (((int64_t)it.chunk + cc) << lt) + r : ((int64_t)it.chunk + cc) * nt + r) *
                           DIRECT_TPT;
        if (k0 >= N) break;
        cplx<T> cv[DIRECT_TPT];
        if (k0 + DIRECT_TPT <= N) {   // unconditional loads (no per-term branch), then the tail
            for (int t = 0; t < DIRECT_TPT; ++t) cv[t] = c[k0 + t];
        } else {
            for (int t = 0; t < DIRECT_TPT; ++t) cv[t] = k0 + t < N ? c[k0 + t] : mk<T>(0, 0);
        }
        const T sc0 = (T)(6.283185307179586476925286766559 * (double)k0);   // 2 pi k = 2 pi k0 + 2 pi t
        for (int t = 0; t < DIRECT_TPT; ++t) {   // c_t, or 2 pi i k c_t for the derivative
            cplx<T> v = cv[t];
            if constexpr (DERIV) {   // (FP32: a literal per t; FP64: one product per t, no table of constants)
                const T sc = sizeof(T) == 4 ? sc0 + (T)(6.283185307179586476925286766559 * t)
                                            : (T)(6.283185307179586476925286766559 * (double)(k0 + t));
                v = mk(-v.y * sc, v.x * sc);
            }
            cv[t] = v;
        }
        auto coef = [&](int t) -> cplx<T> { return cv[t]; };
        for (int g0 = 0; g0 < DIRECT_NG; g0 += NC) {
            if (g0 >= gcount) break;
            // Horner, h <- h w + c_t for t descending, NC nodes of the group at once
            cplx<T> w[NC];
            T hr[NC], hi[NC];
            const cplx<T> cl = coef(DIRECT_TPT - 1);
            for (int g = 0; g < NC; ++g) {
                w[g] = nw[gfirst + g0 + g];
                hr[g] = cl.x;
                hi[g] = cl.y;
            }
            for (int t = DIRECT_TPT - 2; t >= 0; --t) {
                const cplx<T> ct = coef(t);
                for (int g = 0; g < NC; ++g) {
                    const T nr = hr[g] * w[g].x - hi[g] * w[g].y + ct.x;
                    hi[g] = hr[g] * w[g].y + hi[g] * w[g].x + ct.y;
                    hr[g] = nr;
                }
            }
            for (int g = 0; g < NC; ++g) {
                if (g0 + g >= gcount) break;
                const int32_t j = dlist[it.first + gfirst + g0 + g];
                const cplx<T> a = mul(direct_anchor<T>((double)k0, pv.nx[j], pv.ny[j], +1.0), mk(hr[g], hi[g]));
                red[(2 * (g0 + g)) * nt + tid] += (double)a.x;
                red[(2 * (g0 + g) + 1) * nt + tid] += (double)a.y;
            }
        }
    }
    ctx.sync();
    for (int h = (GROUPED ? tpg : nt) >> 1; h > 0; h >>= 1) {   // within each group
        if (r < h)
            for (int q = 0; q < 2 * DIRECT_NG; ++q) red[q * nt + tid] += red[q * nt + tid + h];
        ctx.sync();
    }
    // the groups' sums (row q of group g2 in column g2 2^lt) to their nodes
    for (int e = tid; e < 2 * DIRECT_NG * ng; e += nt) {
        const int g2 = e / (2 * DIRECT_NG), q = e - g2 * (2 * DIRECT_NG);
        const int node = g2 * DIRECT_NG + (q >> 1);
        if (node < it.count) {
            const int32_t j = dlist[it.first + node];
            ctx.atomic_add(dacc + 2 * (int64_t)j + (q & 1), red[q * nt + (GROUPED ? g2 << lt : 0)]);
        }
    }
}

template <class Ctx, typename T>
FLT_HD void body_direct_io(const Ctx& ctx, const PlanView<T>& pv, const int32_t* dlist, int64_t nd, double* dacc,
                           cplx<T>* f, int op)
{
    const int64_t i = (int64_t)ctx.bid() * ctx.ntid() + ctx.tid();
    if (i >= nd) return;
    const int32_t j = dlist[i];
    if (op == 0) {
        dacc[2 * (int64_t)j] = 0.0;
        dacc[2 * (int64_t)j + 1] = 0.0;
    } else {
        f[pv.perm[j]] = mk<T>((T)dacc[2 * (int64_t)j], (T)dacc[2 * (int64_t)j + 1]);
    }
}

// Direct adjoint: acc_k += sum_j g_j conj(w_j)^k over a group of up to
// DIRECT_ANG direct nodes (their conj(w) and g in LDS), direct_atpt
// consecutive k >= 1 per thread (k = 0 is summed over all nodes apart).
// ADJ_TS: the sums leave in slices of that many consecutive k per thread,
// transposed through LDS (red, GATHER_THREADS * ADJ_TS values) so that
// consecutive lanes add into consecutive coefficients.
constexpr int ADJ_TS = 8;
template <class Ctx, typename T>
FLT_HD void body_direct_adj(const Ctx& ctx, const PlanView<T>& pv, const DirectItem* items, const int32_t* dlist,
                            const cplx<T>* gin, double* accall, cplx<T>* nw, cplx<T>* ng, cplx<T>* red)
{
    constexpr int ATPT = direct_atpt((int)sizeof(T));
    const DirectItem it = items[ctx.bid()];
    const int64_t N = pv.inst[it.inst].N;
    double* acc = accall + 2 * pv.inst[it.inst].c_off;
    for (int gi = ctx.tid(); gi < it.count; gi += ctx.ntid()) {
        const int32_t j = dlist[it.first + gi];
        nw[gi] = direct_w(pv, j, -1.0);
        ng[gi] = gin[pv.perm[j]];
    }
    ctx.sync();
    const int64_t kc = (int64_t)it.chunk * ctx.ntid() * ATPT;   // first k of the workgroup
    const int64_t k0 = kc + (int64_t)ctx.tid() * ATPT;
    T ar[ATPT], ai[ATPT];
    for (int t = 0; t < ATPT; ++t) ar[t] = ai[t] = 0;
    for (int gi = 0; gi < (k0 < N ? it.count : 0); ++gi) {
        const int32_t j = dlist[it.first + gi];
        const cplx<T> gv = ng[gi], w = nw[gi];
        cplx<T> p = direct_anchor<T>((double)k0, pv.nx[j], pv.ny[j], -1.0);
        for (int t = 0; t < ATPT; ++t) {
            ar[t] += gv.x * p.x - gv.y * p.y;
            ai[t] += gv.x * p.y + gv.y * p.x;
            p = mul(p, w);
        }
    }
    static_assert(ATPT % ADJ_TS == 0, "whole slices");
    const int tid = ctx.tid(), nt = ctx.ntid();
    for (int t0 = 0; t0 < ATPT; t0 += ADJ_TS) {
        ctx.sync();
        for (int u = 0; u < ADJ_TS; ++u) red[tid * ADJ_TS + u] = mk(ar[t0 + u], ai[t0 + u]);
        ctx.sync();
        for (int u = 0; u < ADJ_TS; ++u) {
            const int e = u * nt + tid;                       // thread e / ADJ_TS, its term t0 + e % ADJ_TS
            const int64_t k = kc + (int64_t)(e / ADJ_TS) * ATPT + t0 + e % ADJ_TS;
            if (k >= 1 && k < N) {
                const cplx<T> v = red[e];
                ctx.atomic_add(acc + 2 * k, (double)v.x);
                ctx.atomic_add(acc + 2 * k + 1, (double)v.y);
            }
        }
    }
}

// Adjoint of one-pass bands: the item's ns columns as sub-transforms of one
// LDS tile (as in the forward), one inverse-sign FFT over all of them, then
// per frequency the transposed contraction sum_s t_k[s] Ghat_s[k - k0] over
// the item's columns, deconvolved and added into acc_k (FP64, atomics; a band
// with more columns than a tile holds has several items).
template <class Ctx, typename T, int LOG2N>
FLT_HD void body_onepass_adj(const Ctx& ctx, const PlanView<T>& pv, const FftItem* items,
                             const cplx<T>* grids, double* acc, cplx<T>* lds)
{
    constexpr int NSUB = (tile_points<T>() >> LOG2N) < MAX_Q ? (tile_points<T>() >> LOG2N) : MAX_Q;
    constexpr int P = NSUB << LOG2N;
    constexpr int n = 1 << LOG2N;
    const FftItem it = items[ctx.bid()];
    const BandDesc B = pv.bands[it.band];   // a copy: the stores below cannot alias it
    StageTw<T, LOG2N, NSUB, -1> stw;
    stw.load(ctx, pv.tw_stage);
    const cplx<T>* src = grids + B.grid_off + ((int64_t)it.s0 << LOG2N);
    const int Pv = it.ns << LOG2N;
    for (int p = ctx.tid(); p < P; p += FFT_THREADS) lds[lds_at(p)] = p < Pv ? src[p] : mk<T>(0, 0);
    ctx.sync();
    lds_fft_ct<Ctx, T, LOG2N, NSUB, -1>(ctx, lds, stw);
    for (int p = ctx.tid(); p < n; p += FFT_THREADS) {
        const int kp = p < (n >> 1) ? p : p - n;
        const int k = kp + (int)B.k0;
        if (k < 1 || k > B.kmax) continue;
        T ar = 0, ai = 0;
        for (int sl = 0; sl < it.ns; ++sl) {
            const T w = laplace_row(pv, B, it.s0 + sl, k);   // the deconvolution is applied once, below
            const cplx<T> v = lds[lds_at((sl << LOG2N) + p)];
            ar += v.x * w;
            ai += v.y * w;
        }
        const double d = (double)pv.deconv[B.deconv_off + (kp < 0 ? -kp : kp)];
        ctx.atomic_add(acc + 2 * (B.c_off + k), d * (double)ar);
        ctx.atomic_add(acc + 2 * (B.c_off + k) + 1, d * (double)ai);
    }
}

// Adjoint pass A: for b consecutive j2, all columns s: Y[j2][l1] e^{-2 pi i j2 l1 / n},
// inverse-sign DFT over l1 -> j1, transposed contraction over s, deconvolved
// once and added into acc.  The FP64 form's (one LDS tile; the FP32 form's is
// body_passA_adj below).
template <class Ctx, typename T, int LOG2N>
FLT_HD void body_passA_adj_1tile(const Ctx& ctx, const PlanView<T>& pv, const FftItem* items,
                           const cplx<T>* scratch, double* acc, cplx<T>* lds, T* lc)
{
    using G = TwoPassGeo<T, LOG2N>;
    constexpr int ITEMS = tile_items<T>();
    constexpr int log2n1 = G::log2n1, log2n2 = G::log2n2, log2b = G::log2b, log2B = G::log2B;
    constexpr int LOG2N1 = log2n1;
    constexpr int P = tile_points<T>();
    constexpr int n = 1 << LOG2N;
    const FftItem it = items[ctx.bid()];
    const BandDesc& B = pv.bands[it.band];
    const int j2_0 = it.blk << log2b;
    // FP64: twiddles in registers (one workgroup per CU either way); FP32: from
    // the table, as the accumulators already fill the four-wave register budget
    typename TwSel<sizeof(T) == 8, T, LOG2N1, (1 << log2b), -1>::type stw;
    stw.load(ctx, pv.tw_stage);
    T accr[ITEMS], acci[ITEMS];   // sum over the q columns of one frequency
    for (int i = 0; i < ITEMS; ++i) accr[i] = acci[i] = 0;
    for (int s = 0; s < B.q; ++s) {
        const cplx<T>* Y = scratch + B.scratch_off + ((int64_t)s << LOG2N);
        // in groups of GI points: the group's reads (values and table
        // factors) in flight together, then the products go to LDS
        constexpr int GI = sizeof(T) == 4 ? 8 : 4;
#pragma unroll 1
        for (int i0 = 0; i0 < ITEMS; i0 += GI) {
            cplx<T> v[GI];
            TwPair<T> w[GI];
            for (int u = 0; u < GI; ++u) {
                const int p = ctx.tid() + (i0 + u) * FFT_THREADS;
                const int l1lo = p & ((1 << log2B) - 1);
                const int jj = (p >> log2B) & ((1 << log2b) - 1);
                const int l1hi = p >> (log2B + log2b);
                const int l1 = (l1hi << log2B) + l1lo;
                const int j2 = j2_0 + jj;
                v[u] = Y[(l1hi << (log2n2 + log2B)) + (j2 << log2B) + l1lo];
                w[u] = tw_grid_fetch(pv, (uint32_t)j2 * (uint32_t)l1, LOG2N);
            }
            for (int u = 0; u < GI; ++u) {
                const int p = ctx.tid() + (i0 + u) * FFT_THREADS;
                const int l1lo = p & ((1 << log2B) - 1);
                const int jj = (p >> log2B) & ((1 << log2b) - 1);
                const int l1 = ((p >> (log2B + log2b)) << log2B) + l1lo;
                lds[lds_at((jj << log2n1) + l1)] = mul(v[u], tw_grid_join(w[u], -1));
            }
        }
        stage_coef(ctx, pv, B, s, lc);
        ctx.sync();
        lds_fft_ct<Ctx, T, LOG2N1, (1 << log2b), -1>(ctx, lds, stw);
        for (int i = 0; i < ITEMS; ++i) {
            const int p = ctx.tid() + i * FFT_THREADS;
            if (p >= P) break;
            const int j1 = p & ((1 << log2n1) - 1);   // tile element p = (jj << log2n1) + j1
            const int jj = p >> log2n1;
            const int j = j2_0 + jj + (j1 << log2n2);
            const int kp = j < (n >> 1) ? j : j - n;
            const int k = kp + (int)B.k0;
            if (k < 1 || k > B.kmax) continue;
            const T w = laplace_row_lds(lc, B, k);   // the deconvolution is applied once, below
            const cplx<T> v = lds[lds_at(p)];
            accr[i] += v.x * w;
            acci[i] += v.y * w;
        }
        ctx.sync();
    }
    // the per-point sums leave through the LDS tile, re-read with the b
    // sub-transforms (consecutive k) fastest: a wave's atomics then fall on
    // runs of consecutive coefficients instead of one cache line per lane
    for (int i = 0; i < ITEMS; ++i) {
        const int p = ctx.tid() + i * FFT_THREADS;
        lds[lds_at(p)] = mk(accr[i], acci[i]);
    }
    ctx.sync();
    for (int i = 0; i < ITEMS; ++i) {
        const int r = ctx.tid() + i * FFT_THREADS;
        const int jj = r & ((1 << log2b) - 1);
        const int j1 = r >> log2b;
        const int j = j2_0 + jj + (j1 << log2n2);
        const int kp = j < (n >> 1) ? j : j - n;
        const int k = kp + (int)B.k0;
        if (k < 1 || k > B.kmax) continue;
        const cplx<T> a = lds[lds_at((jj << log2n1) + j1)];
        const double d = (double)pv.deconv[B.deconv_off + (kp < 0 ? -kp : kp)];
        ctx.atomic_add(acc + 2 * (B.c_off + k), d * (double)a.x);
        ctx.atomic_add(acc + 2 * (B.c_off + k) + 1, d * (double)a.y);
    }
}

// Adjoint pass A of the FP32 form: the transform of body_passA_adj_1tile with
// the LDS of a workgroup per CU (two tiles in turn, two coefficient buffers)
// and the last DFT stage kept in registers: the transposed contraction
// sum_s t_k[s] Ghat_s(k) runs on the thread's last-stage outputs that lie in
// the band's support (half of them, known at compile time as in pass A), its
// sums held in registers across the columns.  Input twiddles as pass A's
// output twiddles (the LDS power table for the larger grids).  Three barriers
// per column.
template <class Ctx, typename T, int LOG2N>
FLT_HD void body_passA_adj(const Ctx& ctx, const PlanView<T>& pv, const FftItem* items,
                           const cplx<T>* scratch, double* acc, cplx<T>* lds, T* lc, cplx<T>* omega)
{
    static_assert(sizeof(T) == 4, "the FP32 form's adjoint pass A (FP64: body_passA_adj_1tile)");
    using G = TwoPassGeo<T, LOG2N>;
    using A = PassAGeo<T, LOG2N>;
    constexpr int ITEMS = A::ITEMS;
    constexpr int log2n1 = G::log2n1, log2n2 = G::log2n2, log2b = G::log2b, log2B = G::log2B;
    constexpr int n = 1 << LOG2N;
    constexpr int NSUB = 1 << log2b;
    constexpr int LRL = last_stage_lr(log2n1, 0, MaxRadix<T>::LOG2);   // the last stage
    constexpr int RL = 1 << LRL;
    constexpr int LOG2NSL = log2n1 - LRL;
    constexpr int NBL = StageGeo<LRL, log2n1, NSUB>::NB;
    constexpr int COEF = Sizes<T>::COEF;
    // output r of a last-stage butterfly is sub-transform element jl + r 2^LOG2NSL:
    // in the support only for r <= RL/4 or r >= 3 RL/4 (r = RL/4 only at jl = 0)
    auto live = [](int r) { return r <= RL / 4 || r >= 3 * RL / 4; };
    const FftItem it = items[ctx.bid()];
    const BandDesc B = pv.bands[it.band];
    const int k0 = (int)B.k0, kmax = (int)B.kmax;
    const int j2_0 = it.blk << log2b;
    const int tid = ctx.tid();
    cplx<T>* const tile[2] = {lds, lds + tile_alloc<T>()};
    StageTw<T, log2n1, NSUB, -1> stw;
    stw.load(ctx, pv.tw_stage);
    const int o_l1lo = tid & ((1 << log2B) - 1);
    const int o_jj = (tid >> log2B) & ((1 << log2b) - 1);
    const int o_l1hi = tid >> (log2B + log2b);
    cplx<T> tw_t = mk<T>(1, 0);
    if constexpr (A::OMEGA > 0) {
        static_assert(A::OMEGA <= PASSA_OMEGA_MAX && A::OMEGA <= FFT_THREADS, "input twiddle table size");
        if (tid < A::OMEGA) {
            const int jj = tid / ITEMS, i = tid % ITEMS;
            omega[tid] = tw_grid_at(pv, (uint32_t)(j2_0 + jj) * (uint32_t)(A::DL * i), LOG2N, -1);
        }
        tw_t = tw_grid_at(pv, (uint32_t)(j2_0 + o_jj) * (uint32_t)((o_l1hi << log2B) + o_l1lo), LOG2N, -1);
    }
    stage_coef(ctx, pv, B, 0, lc);
    // the thread's last-stage points: k (0 outside the support), sums
    int kr[NBL][RL];
    cplx<T> sum[NBL][RL];
    {
        constexpr int LOG2LQ = log2n1 - LRL;   // = LOG2NSL
        for (int i = 0; i < NBL; ++i)
            for (int r = 0; r < RL; ++r) {
                sum[i][r] = mk<T>(0, 0);
                kr[i][r] = 0;
                const int u = tid + i * FFT_THREADS;
                if (!live(r) || u >= StageGeo<LRL, log2n1, NSUB>::NBUT) continue;
                const int jj = u >> LOG2LQ, jl = u & ((1 << LOG2LQ) - 1);
                const int j1 = jl + (r << LOG2NSL);
                kr[i][r] = passA_k(j2_0 + jj + (j1 << log2n2), n, k0, kmax);
            }
    }
    ctx.sync();

    cplx<T>* ld = tile[0];   // the tile the next column is loaded into
    for (int s = 0; s < B.q; ++s) {
        const cplx<T>* Y = scratch + B.scratch_off + ((int64_t)s << LOG2N);
        if constexpr (A::OMEGA > 0) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int l1 = (o_l1hi << log2B) + o_l1lo + i * A::DL;
                const cplx<T> v = Y[((l1 >> log2B) << (log2n2 + log2B)) + ((j2_0 + o_jj) << log2B) + o_l1lo];
                ld[lds_at((o_jj << log2n1) + l1)] = mul(v, mul(tw_t, omega[o_jj * ITEMS + i]));
            }
        } else {
            constexpr int GI = 8;
#pragma unroll 1
            for (int i0 = 0; i0 < ITEMS; i0 += GI) {
                cplx<T> v[GI];
                TwPair<T> w[GI];
                for (int u = 0; u < GI; ++u) {
                    const int p = tid + (i0 + u) * FFT_THREADS;
                    const int l1lo = p & ((1 << log2B) - 1);
                    const int jj = (p >> log2B) & ((1 << log2b) - 1);
                    const int l1hi = p >> (log2B + log2b);
                    const int l1 = (l1hi << log2B) + l1lo;
                    v[u] = Y[(l1hi << (log2n2 + log2B)) + ((j2_0 + jj) << log2B) + l1lo];
                    w[u] = tw_grid_fetch(pv, (uint32_t)(j2_0 + jj) * (uint32_t)l1, LOG2N);
                }
                for (int u = 0; u < GI; ++u) {
                    const int p = tid + (i0 + u) * FFT_THREADS;
                    const int l1lo = p & ((1 << log2B) - 1);
                    const int jj = (p >> log2B) & ((1 << log2b) - 1);
                    const int l1 = ((p >> (log2B + log2b)) << log2B) + l1lo;
                    ld[lds_at((jj << log2n1) + l1)] = mul(v[u], tw_grid_join(w[u], -1));
                }
            }
        }
        ctx.sync();
        // the next column's coefficients (the other buffer was last read by
        // the previous column's contraction, before the barrier above)
        if (s + 1 < B.q) stage_coef(ctx, pv, B, s + 1, lc + ((s + 1) & 1) * COEF);
        const T* lcs = lc + (s & 1) * COEF;
        cplx<T>* const other = ld == tile[0] ? tile[1] : tile[0];
        cplx<T>* const last = lds_fft_pp_last_regs<Ctx, T, log2n1, NSUB, -1, 0>(
            ctx, ld, other, stw, [&](cplx<T> (&v)[NBL][RL], int (&dsti)[NBL]) {
                for (int i = 0; i < NBL; ++i)
                    for (int r = 0; r < RL; ++r) {
                        if (!live(r) || dsti[i] < 0) continue;
                        const int k = kr[i][r];
                        const T w = k ? laplace_row_lds(lcs, B, k) : T(0);   // deconvolved once, below
                        sum[i][r].x += v[i][r].x * w;
                        sum[i][r].y += v[i][r].y * w;
                    }
            });
        ld = last == tile[0] ? tile[1] : tile[0];
    }
    // the sums leave through LDS (the tile the last stage did not read), re-read
    // with the b sub-transforms (consecutive k) fastest, so that a wave's
    // atomics fall on runs of consecutive coefficients
    for (int i = 0; i < NBL; ++i)
        for (int r = 0; r < RL; ++r) {
            const int u = tid + i * FFT_THREADS;
            if (!live(r) || u >= StageGeo<LRL, log2n1, NSUB>::NBUT) continue;
            const int jj = u >> LOG2NSL, jl = u & ((1 << LOG2NSL) - 1);
            ld[lds_at((jj << log2n1) + jl + (r << LOG2NSL))] = sum[i][r];
        }
    ctx.sync();
    for (int i = 0; i < ITEMS; ++i) {
        const int r = tid + i * FFT_THREADS;
        const int jj = r & ((1 << log2b) - 1);
        const int j1 = r >> log2b;
        const int j = j2_0 + jj + (j1 << log2n2);
        const int k = passA_k(j, n, k0, kmax);
        if (!k) continue;
        const int kp = j < (n >> 1) ? j : j - n;
        const cplx<T> a = ld[lds_at((jj << log2n1) + j1)];
        const double d = (double)pv.deconv[B.deconv_off + (kp < 0 ? -kp : kp)];
        ctx.atomic_add(acc + 2 * (B.c_off + k), d * (double)a.x);
        ctx.atomic_add(acc + 2 * (B.c_off + k) + 1, d * (double)a.y);
    }
}

}  // namespace flt
