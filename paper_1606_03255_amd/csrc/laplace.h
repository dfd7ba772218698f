// The discrete Laplace transform f_j = sum_k fhat_k exp(-y_j xi_k) (Sect. 3,
// Algorithm 1): planner types and the bodies of its kernels, shared by the
// gfx950 build and the CPU build.
#pragma once
#include <stdint.h>

#include <vector>

#include "flt_types.h"

namespace flt {

constexpr int LAP_THREADS = 256;   // threads of every Laplace workgroup
constexpr int LAP_CHUNK = 2048;    // moments: frequencies per workgroup (one block)
constexpr int LAP_PER = LAP_CHUNK / LAP_THREADS;
constexpr int LAP_NODE_PER = 4;     // nodes per thread of the node kernel
constexpr int LAP_NODE_LDS = 8192;  // node kernel: most doubles of band data staged in LDS
constexpr int LAP_MAX_Q = 32;      // largest rank (eps >= 4^-31)

// Work item of the moments kernel: `count` sorted frequencies of block `blk`
// from `start`.
struct LapItem {
    int32_t blk;
    int32_t count;
    int64_t start;
};

// The interpolation of Algorithm 1 in Chebyshev coefficients.  On an
// interval with centre c and half-width w, t = (x - c) / w, the Lagrange
// basis at the q Chebyshev nodes tau_r = cos((2r+1) pi / (2q)) is
// L_r(t) = sum_{p<q} a_p T_p(tau_r) T_p(t), a_0 = 1/q, a_p = 2/q (discrete
// orthogonality of T_0..T_{q-1} on those nodes).  Hence the block moments
// v_r = sum_p a_p T_p(tau_r) mu_p with mu_p = sum_k fhat_k T_p(t_k), and the
// band's interpolant sum_s L_s(t) h_s = sum_p beta_p T_p(t) with
// beta = C K C^T mu summed over the blocks, C[p][r] = a_p T_p(tau_r): the same
// polynomial as the Lagrange form, evaluated without divisions (three-term
// recurrence on the frequencies, Clenshaw's on the nodes).
//
// The plan as the kernels read it (device or host pointers).  Levels are
// 1..L (the paper's M): blocks Omega_l and bands Y_m, l, m < L interpolated,
// Omega_L and Y_L the intervals at 0.
// Kernels (Sect. 3; Thm 3.3 and its example): 0 exp(-y xi) by Algorithm 1;
// 1 K_{1/2}(y xi) = sqrt(pi / (2 y xi)) exp(-y xi), asymptotically smooth: every
// block l < L interpolated, the near fields Omega_L and Y_L summed directly.
constexpr int LAP_KERNEL_EXP = 0;
constexpr int LAP_KERNEL_K12 = 1;

FLT_HD double lap_kernel_k12(double x) { return sqrt(1.5707963267948966192 / x) * exp(-x); }

struct LapView {
    int32_t q, L;
    int32_t kernel;          // LAP_KERNEL_*
    int32_t pad;
    int64_t near0, nnear;    // general kernels: the sorted frequencies of Omega_L (near field)
    int64_t N;
    const double* xs;        // frequencies sorted by block
    const int32_t* kperm;    // caller index of each sorted frequency
    const double* bcw;       // 2 (l - 1): centre, 1 / half-width of Omega_l's closure
    const double* ycw;       // 2 (m - 1): centre, 1 / half-width of Y_m's closure; (0, 0) for m = L
    const int32_t* lm;       // per band m (index m - 1): first interpolated block l_m
    const int32_t* Lm;       // per band m: last interpolated block L_m = L - m
    const int64_t* koff;     // per band m: first entry of its tables
    const double* K;         // (C K^{Y_m,Omega_l} C^T)[p'][p], K[s][r] = exp(-y_s xi_r), l = l_m..L_m, band after band
    const double* y;         // nodes, caller order
    const int32_t* band;     // band of each node, 1..L
    const int32_t* bitem;    // L + 1: the items of block l are bitem[l - 1] .. bitem[l] - 1
    int32_t nitems;
    double* part;            // per item partial moments: part[item * 2q + v], v = 2p (re), 2p + 1 (im)
    double* acc;             // mu (L q complex), S (L + 2 complex), beta (L q complex)
};

// Accumulator layout (complex FP64 = 2 doubles each).
FLT_HD int64_t lap_mu(int L, int q, int l, int p) { return 2 * ((int64_t)(l - 1) * q + p); }
FLT_HD int64_t lap_S(int L, int q, int l) { return 2 * ((int64_t)L * q + l); }
FLT_HD int64_t lap_beta(int L, int q, int m, int p) { return 2 * ((int64_t)L * q + L + 2 + (int64_t)(m - 1) * q + p); }
FLT_HD int64_t lap_acc_doubles(int L, int q) { return 2 * (2 * (int64_t)L * q + L + 2); }

// Host plan (planner output, uploaded as is).
struct LapHost {
    int64_t N = 0, M = 0;
    int dtype = 0;
    int kernel = LAP_KERNEL_EXP;
    int64_t near0 = 0, nnear = 0;   // general kernels: Omega_L's sorted frequencies
    double eps = 0, y1 = 0, xi1 = 0;
    int q = 0, L = 1;
    std::vector<double> xs, bcw, ycw, K, y;
    std::vector<int32_t> kperm, lm, Lm, band, bitem;
    std::vector<int64_t> koff;
    std::vector<LapItem> items;
};

// Builds the plan (Def. 3.2 partition, tables); FLT_OK or an FLT_E* code.
int build_laplace_plan(LapHost& hp, int64_t N, const double* xi, int64_t M, const double* y, double eps,
                       int dtype, int kernel = LAP_KERNEL_EXP);

// ---------------------------------------------------------------------------
// Kernels (bodies).  Ctx supplies tid(), ntid(), bid() and sync().
// ---------------------------------------------------------------------------
// Register buckets of the moments kernel: the q accumulators of a thread
// live in registers, so their count is a compile-time bound QB >= q.
FLT_HD constexpr int lap_qbucket(int q) { return q <= 8 ? 8 : q <= 12 ? 12 : q <= 16 ? 16 : q <= 24 ? 24 : 32; }

// Moments of one chunk (item) of block l: the partial sums of
// mu_p = sum_k fhat_k T_p(t_k), p < q (for l = L only mu_0 is used: T_0 = 1,
// and mu_0 = S_l = sum_k fhat_k on every block).  Each thread takes LAP_PER
// frequencies (all loads issued before the first is used) and keeps q complex
// sums in registers, T_p by the three-term recurrence; the 2q sums are added
// over the workgroup through LDS in rounds of 8 values (red: 8 LAP_THREADS
// doubles, red2: LAP_THREADS doubles) and stored as the item's partials (no
// atomics: many items share a block).
template <class Ctx, typename T, int QB>
FLT_HD void lap_body_moments(const Ctx& ctx, const LapView& V, const LapItem* items, const cplx<T>* fhat,
                             double* red, double* red2)
{
    const LapItem it = items[ctx.bid()];
    const int tid = ctx.tid();
    const int q = V.q, l = it.blk;
    const bool interp = l < V.L;
    const double c = interp ? V.bcw[2 * (l - 1)] : 0.0, iw = interp ? V.bcw[2 * (l - 1) + 1] : 0.0;
    int32_t kp[LAP_PER];
    double xv[LAP_PER];
    cplx<T> fv[LAP_PER];
#pragma unroll
    for (int j = 0; j < LAP_PER; ++j) {   // clamped, unconditional loads (count >= 1)
        const int i = tid + j * LAP_THREADS < it.count ? tid + j * LAP_THREADS : it.count - 1;
        kp[j] = V.kperm[it.start + i];
        xv[j] = V.xs[it.start + i];
    }
#pragma unroll
    for (int j = 0; j < LAP_PER; ++j) fv[j] = fhat[kp[j]];
    double ar[QB], ai[QB];
#pragma unroll
    for (int p = 0; p < QB; ++p) ar[p] = ai[p] = 0.0;
#pragma unroll
    for (int j = 0; j < LAP_PER; ++j) {
        const bool in = tid + j * LAP_THREADS < it.count;
        const double fr = in ? (double)fv[j].x : 0.0, fi = in ? (double)fv[j].y : 0.0;
        const double t = (xv[j] - c) * iw, t2 = 2.0 * t;
        double tm = 1.0, tc = t;   // T_{p-1}, T_p
        ar[0] += fr;
        ai[0] += fi;
        if (1 < q) {
            ar[1] += fr * t;
            ai[1] += fi * t;
        }
#pragma unroll
        for (int p = 2; p < QB; ++p)
            if (p < q) {
                const double tn = t2 * tc - tm;
                tm = tc;
                tc = tn;
                ar[p] += fr * tn;
                ai[p] += fi * tn;
            }
    }
    double* dst = V.part + (int64_t)ctx.bid() * 2 * q;
#pragma unroll
    for (int v0 = 0; v0 < 2 * QB; v0 += 8) {
        if (v0 >= 2 * q) break;   // (uniform)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int v = v0 + e;   // value v: mu_{v/2}, re (even) or im (odd)
            red[e * LAP_THREADS + tid] = (v & 1) ? ai[v / 2] : ar[v / 2];
        }
        ctx.sync();
        {   // value e = tid / 32: the sum of 8 of its 256 entries, a fixed order
            const int e = tid >> 5, s = tid & 31;
            double a = 0.0;
            for (int k = 0; k < 8; ++k) a += red[e * LAP_THREADS + k * 32 + s];
            red2[tid] = a;
        }
        ctx.sync();
        if (tid < 8 && v0 + tid < 2 * q) {
            double a = 0.0;
            for (int s = 0; s < 32; ++s) a += red2[tid * 32 + s];
            dst[v0 + tid] = a;
        }
        ctx.sync();
    }
}

// Sums the item partials of each block, workgroup l: thread (v, w), v < 2q,
// w < W = 256 / 2q, sums value v of every W-th item of the block (the items'
// values are contiguous); the W sums of each v are added through LDS (red,
// LAP_THREADS doubles) into mu^{Omega_l} (re/im interleaved); S_l = mu_0.  A
// fixed summation order: every call gives the same bits.
template <class Ctx>
FLT_HD void lap_body_reduce(const Ctx& ctx, const LapView& V, double* red)
{
    const int q = V.q, nv = 2 * q, W = LAP_THREADS / nv;
    const int l = ctx.bid() + 1, tid = ctx.tid(), v = tid % nv, w = tid / nv;
    double a = 0.0;
    if (w < W) {
        const int i1 = V.bitem[l];
#pragma unroll 16
        for (int i = V.bitem[l - 1] + w; i < i1; i += W) a += V.part[(int64_t)i * nv + v];
    }
    red[tid] = a;
    ctx.sync();
    if (tid < nv) {
        double t = 0.0;
        for (int u = 0; u < W; ++u) t += red[u * nv + tid];
        V.acc[lap_mu(V.L, q, l, tid / 2) + (tid & 1)] = t;
        if (tid < 2) V.acc[lap_S(V.L, q, l) + tid] = t;
    }
}

// The band side, workgroup m = 1..L.  For m < L:
// beta^{Y_m} = sum_{l = l_m}^{L_m} (C K^{Y_m,Omega_l} C^T) mu^{Omega_l}, the
// (p', l) products spread over the threads (U = 256 / q per p', each a share
// of the blocks, the q values of a row loaded at once), plus, in beta_0
// (T_0 = 1), the far part g_{L_m + 1} = sum_{l > L_m} S_l.  For m = L (the
// band at 0, t = 0): beta = (g_1, 0, ..., 0), g_1 the sum of all S_l.  Both
// sums are reduced through LDS (red, 4 LAP_THREADS doubles) in a fixed order.
template <class Ctx, int QB>
FLT_HD void lap_body_bands(const Ctx& ctx, const LapView& V, double* red)
{
    const int q = V.q, L = V.L, m = ctx.bid() + 1, tid = ctx.tid();
    const int U = LAP_THREADS / q;
    const int s = tid / U, u = tid % U;
    double hr = 0.0, hi = 0.0;
    if (m < L && s < q) {
        const int l0 = V.lm[m - 1], l1 = V.Lm[m - 1];
        const double* Km = V.K + V.koff[m - 1];
        for (int l = l0 + u; l <= l1; l += U) {
            const double* row = Km + ((int64_t)(l - l0) * q + s) * q;
            const double* mu = V.acc + lap_mu(L, q, l, 0);
            double kr[QB], vr[QB], vi[QB];
#pragma unroll
            for (int r = 0; r < QB; ++r) {   // clamped, unconditional loads
                const int rc = r < q ? r : q - 1;
                kr[r] = row[rc];
                vr[r] = mu[2 * rc];
                vi[r] = mu[2 * rc + 1];
            }
#pragma unroll
            for (int r = 0; r < QB; ++r)
                if (r < q) {
                    hr += kr[r] * vr[r];
                    hi += kr[r] * vi[r];
                }
        }
    }
    // g_{g0} = sum_{l = g0}^{L} S_l (Algorithm 1's blocks where the kernel is 1;
    // general kernels have none: their near field is summed at the nodes)
    const int g0 = V.kernel != LAP_KERNEL_EXP ? L + 1 : m < L ? V.Lm[m - 1] + 1 : 1;
    double gr = 0.0, gi = 0.0;
    for (int l = g0 + tid; l <= L; l += LAP_THREADS) {
        gr += V.acc[lap_S(L, q, l)];
        gi += V.acc[lap_S(L, q, l) + 1];
    }
    red[2 * tid] = hr;
    red[2 * tid + 1] = hi;
    red[2 * LAP_THREADS + 2 * tid] = gr;
    red[2 * LAP_THREADS + 2 * tid + 1] = gi;
    ctx.sync();
    if (m < L && s < q && u == 0) {
        double tr = 0.0, ti = 0.0;
        for (int v = 0; v < U; ++v) {
            tr += red[2 * (tid + v)];
            ti += red[2 * (tid + v) + 1];
        }
        if (s == 0 && g0 <= L) {
            const int n = L - g0 + 1 < LAP_THREADS ? L - g0 + 1 : LAP_THREADS;
            for (int v = 0; v < n; ++v) {
                tr += red[2 * LAP_THREADS + 2 * v];
                ti += red[2 * LAP_THREADS + 2 * v + 1];
            }
        }
        V.acc[lap_beta(L, q, m, s)] = tr;
        V.acc[lap_beta(L, q, m, s) + 1] = ti;
    }
    if (m == L && tid < q) {
        double tr = 0.0, ti = 0.0;
        if (tid == 0 && V.kernel == LAP_KERNEL_EXP) {
            const int n = L < LAP_THREADS ? L : LAP_THREADS;
            for (int v = 0; v < n; ++v) {
                tr += red[2 * LAP_THREADS + 2 * v];
                ti += red[2 * LAP_THREADS + 2 * v + 1];
            }
        }
        V.acc[lap_beta(L, q, m, tid)] = tr;
        V.acc[lap_beta(L, q, m, tid) + 1] = ti;
    }
}

// Doubles of band data the node kernel stages in LDS (every beta^{Y_m}, then
// the (centre, 1 / half-width) pairs), 0 when they do not fit LAP_NODE_LDS.
FLT_HD int64_t lap_node_stage(int L, int q)
{
    const int64_t n = 2 * (int64_t)L * q + 2 * (int64_t)L;
    return n <= LAP_NODE_LDS ? n : 0;
}

// The node side: f_j = sum_p beta^{Y_m}_p T_p(t_j) by Clenshaw's recurrence,
// m the band of y_j (for m = L: t = 0 and beta = (g_1, 0, ...), f_j = g_1).
// LAP_NODE_PER nodes per thread, their loads issued at once; the band data
// read from LDS (sb, lap_node_stage doubles, staged by the workgroup) when
// sb is set, else from global memory.
// General kernels add the near fields directly: for a node of band m < L the
// frequencies of Omega_L, for a node of Y_L all of them (FP64 sums).
template <typename T>
FLT_HD void lap_near(const LapView& V, const cplx<T>* fhat, double y, int64_t k0, int64_t k1, double* sr, double* si)
{
    double ar = 0.0, ai = 0.0;
    for (int64_t i = k0; i < k1; ++i) {
        const double w = lap_kernel_k12(y * V.xs[i]);
        const cplx<T> v = fhat[V.kperm[i]];
        ar += w * (double)v.x;
        ai += w * (double)v.y;
    }
    *sr += ar;
    *si += ai;
}

template <class Ctx, typename T, int QB>
FLT_HD void lap_body_nodes(const Ctx& ctx, const LapView& V, int64_t M, cplx<T>* f, double* sb,
                           const cplx<T>* fhat)
{
    const int q = V.q, L = V.L, tid = ctx.tid();
    int m[LAP_NODE_PER];
    double yv[LAP_NODE_PER];
    const int64_t j0 = (int64_t)ctx.bid() * LAP_NODE_PER * ctx.ntid() + tid;
#pragma unroll
    for (int k = 0; k < LAP_NODE_PER; ++k) {   // clamped, unconditional loads, issued before the staging
        const int64_t j = j0 + (int64_t)k * ctx.ntid() < M ? j0 + (int64_t)k * ctx.ntid() : M - 1;
        m[k] = V.band[j];
        yv[k] = V.y[j];
    }
    const double* beta = V.acc + lap_beta(L, q, 1, 0);   // band m at 2 (m - 1) q
    const double* cw = V.ycw;
    if (sb) {   // (uniform)
        const int64_t nb = 2 * (int64_t)L * q;
        for (int64_t i = tid; i < nb; i += ctx.ntid()) sb[i] = beta[i];
        for (int i = tid; i < 2 * L; i += ctx.ntid()) sb[nb + i] = cw[i];
        ctx.sync();
        beta = sb;
        cw = sb + nb;
    }
#pragma unroll
    for (int k = 0; k < LAP_NODE_PER; ++k) {
        const double* b = beta + 2 * (int64_t)(m[k] - 1) * q;
        double br[QB], bi[QB];
#pragma unroll
        for (int p = 0; p < QB; ++p) {
            const int pc = p < q ? p : q - 1;
            br[p] = b[2 * pc];
            bi[p] = b[2 * pc + 1];
        }
        const double t = (yv[k] - cw[2 * (m[k] - 1)]) * cw[2 * (m[k] - 1) + 1], t2 = 2.0 * t;
        double b1r = 0.0, b1i = 0.0, b2r = 0.0, b2i = 0.0;   // b_{n+1}, b_{n+2}
#pragma unroll
        for (int n = QB - 1; n >= 1; --n)
            if (n < q) {
                const double nr = br[n] + t2 * b1r - b2r, ni = bi[n] + t2 * b1i - b2i;
                b2r = b1r;
                b2i = b1i;
                b1r = nr;
                b1i = ni;
            }
        const int64_t j = j0 + (int64_t)k * ctx.ntid();
        double fr = br[0] + t * b1r - b2r, fi = bi[0] + t * b1i - b2i;
        if (V.kernel != LAP_KERNEL_EXP && j < M) {
            if (m[k] < L) lap_near(V, fhat, yv[k], V.near0, V.near0 + V.nnear, &fr, &fi);
            else lap_near(V, fhat, yv[k], 0, V.N, &fr, &fi);
        }
        if (j < M) f[j] = mk<T>((T)fr, (T)fi);
    }
}

}  // namespace flt
