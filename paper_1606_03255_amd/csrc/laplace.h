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
constexpr int LAP_MAX_Q = 32;      // largest rank (eps >= 4^-31)

// Work item of the moments kernel: `count` sorted frequencies of block `blk`
// from `start`.
struct LapItem {
    int32_t blk;
    int32_t count;
    int64_t start;
};

// The plan as the kernels read it (device or host pointers).  Levels are
// 1..L (the paper's M): blocks Omega_l and bands Y_m, l, m < L interpolated,
// Omega_L and Y_L the intervals at 0.
struct LapView {
    int32_t q, L;
    const double* xs;        // frequencies sorted by block
    const int32_t* kperm;    // caller index of each sorted frequency
    const double* bnodes;    // (l - 1) q + r: Chebyshev nodes of Omega_l's closure
    const double* ynodes;    // (m - 1) q + s: Chebyshev nodes of Y_m's closure
    const double* bw;        // q barycentric weights (-1)^r sin((2r+1) pi / (2q))
    const int32_t* lm;       // per band m (index m - 1): first interpolated block l_m
    const int32_t* Lm;       // per band m: last interpolated block L_m = L - m
    const int64_t* koff;     // per band m: first entry of its K tables
    const double* K;         // K^{Y_m,Omega_l}[s][r] = exp(-y_s xi_r), l = l_m..L_m, band after band
    const double* y;         // nodes, caller order
    const int32_t* band;     // band of each node, 1..L
    double* acc;             // v (L q complex), S (L + 2 complex), h (L q complex), g (L + 2 complex)
};

// Accumulator layout (complex FP64 = 2 doubles each).
FLT_HD int64_t lap_v(int L, int q, int l, int r) { return 2 * ((int64_t)(l - 1) * q + r); }
FLT_HD int64_t lap_S(int L, int q, int l) { return 2 * ((int64_t)L * q + l); }
FLT_HD int64_t lap_h(int L, int q, int m, int s) { return 2 * ((int64_t)L * q + L + 2 + (int64_t)(m - 1) * q + s); }
FLT_HD int64_t lap_g(int L, int q, int m) { return 2 * (2 * (int64_t)L * q + L + 2 + m); }
FLT_HD int64_t lap_acc_doubles(int L, int q) { return 2 * (2 * (int64_t)L * q + 2 * (int64_t)L + 4); }

// Host plan (planner output, uploaded as is).
struct LapHost {
    int64_t N = 0, M = 0;
    int dtype = 0;
    double eps = 0, y1 = 0, xi1 = 0;
    int q = 0, L = 1;
    std::vector<double> xs, bnodes, ynodes, bw, K, y;
    std::vector<int32_t> kperm, lm, Lm, band;
    std::vector<int64_t> koff;
    std::vector<LapItem> items;
};

// Builds the plan (Def. 3.2 partition, tables); FLT_OK or an FLT_E* code.
int build_laplace_plan(LapHost& hp, int64_t N, const double* xi, int64_t M, const double* y, double eps,
                       int dtype);

// ---------------------------------------------------------------------------
// Kernels (bodies).  Ctx supplies tid(), ntid(), bid(), sync(), atomic_add.
// ---------------------------------------------------------------------------
template <class Ctx>
FLT_HD void lap_body_zero(const Ctx& ctx, double* acc, int64_t n)   // a fill kernel: capturable
{
    const int64_t i = (int64_t)ctx.bid() * ctx.ntid() + ctx.tid();
    if (i < n) acc[i] = 0.0;
}

// Moments of one chunk of block l: v_r += sum_k fhat_k L_r^{Omega_l}(xi_k)
// (r < q, l < L) and S_l += sum_k fhat_k.  Phase 1: per frequency the inverse
// of the barycentric denominator (or the node it hits) into LDS; phase 2:
// thread (r, u) sums every (256 / 32)-th frequency for basis function r;
// the partial sums of each r are reduced through LDS and added atomically.
template <class Ctx, typename T>
FLT_HD void lap_body_moments(const Ctx& ctx, const LapView& V, const LapItem* items, const cplx<T>* fhat,
                             double* sden, int32_t* shit, double* sf, double* red)
{
    const LapItem it = items[ctx.bid()];
    const int tid = ctx.tid();
    const int q = V.q, l = it.blk;
    const bool interp = l < V.L;
    const double* xn = V.bnodes + (int64_t)(l - 1) * q;
    for (int i = tid; i < it.count; i += LAP_THREADS) {
        const int64_t k = it.start + i;
        const cplx<T> f = fhat[V.kperm[k]];
        sf[2 * i] = (double)f.x;
        sf[2 * i + 1] = (double)f.y;
        if (interp) {
            const double x = V.xs[k];
            double den = 0.0;
            int hit = -1;
            for (int r = 0; r < q; ++r) {
                const double d = x - xn[r];
                if (d == 0.0) hit = r;
                else den += V.bw[r] / d;
            }
            shit[i] = hit;
            sden[i] = hit >= 0 ? 0.0 : 1.0 / den;
        }
    }
    ctx.sync();
    // S_l: 256 threads, strided partial sums, reduced below together with r = q
    constexpr int U = LAP_THREADS / LAP_MAX_Q;   // threads per basis function
    const int r = tid / U, u = tid % U;
    double ar = 0.0, ai = 0.0;
    if (r < q && interp) {
        const double xr = xn[r], lr = V.bw[r];
        for (int i = u; i < it.count; i += U) {
            double w;
            if (shit[i] >= 0) w = shit[i] == r ? 1.0 : 0.0;
            else w = lr / (V.xs[it.start + i] - xr) * sden[i];
            ar += sf[2 * i] * w;
            ai += sf[2 * i + 1] * w;
        }
    }
    double sr = 0.0, si = 0.0;   // block sum: every thread a strided part
    for (int i = tid; i < it.count; i += LAP_THREADS) {
        sr += sf[2 * i];
        si += sf[2 * i + 1];
    }
    red[4 * tid] = ar;
    red[4 * tid + 1] = ai;
    red[4 * tid + 2] = sr;
    red[4 * tid + 3] = si;
    ctx.sync();
    if (u == 0 && r < q && interp) {
        double tr = 0.0, ti = 0.0;
        for (int v = 0; v < U; ++v) {
            tr += red[4 * (tid + v)];
            ti += red[4 * (tid + v) + 1];
        }
        ctx.atomic_add(V.acc + lap_v(V.L, q, l, r), tr);
        ctx.atomic_add(V.acc + lap_v(V.L, q, l, r) + 1, ti);
    }
    if (tid == LAP_THREADS - 1) {
        double tr = 0.0, ti = 0.0;
        for (int v = 0; v < LAP_THREADS; ++v) {
            tr += red[4 * v + 2];
            ti += red[4 * v + 3];
        }
        ctx.atomic_add(V.acc + lap_S(V.L, q, l), tr);
        ctx.atomic_add(V.acc + lap_S(V.L, q, l) + 1, ti);
    }
}

// The band side (one workgroup): g_m = sum_{l >= m} S_l (cumulative, from
// l = L down), then h^{Y_m}_s = sum_{l = l_m}^{L_m} sum_r K^{Y_m,Omega_l}[s][r] v^{Omega_l}_r.
template <class Ctx>
FLT_HD void lap_body_bands(const Ctx& ctx, const LapView& V)
{
    const int q = V.q, L = V.L;
    if (ctx.tid() == 0) {
        double gr = 0.0, gi = 0.0;
        V.acc[lap_g(L, q, L + 1)] = 0.0;
        V.acc[lap_g(L, q, L + 1) + 1] = 0.0;
        for (int m = L; m >= 1; --m) {
            gr += V.acc[lap_S(L, q, m)];
            gi += V.acc[lap_S(L, q, m) + 1];
            V.acc[lap_g(L, q, m)] = gr;
            V.acc[lap_g(L, q, m) + 1] = gi;
        }
    }
    for (int e = ctx.tid(); e < (L - 1) * q; e += ctx.ntid()) {
        const int m = e / q + 1, s = e % q;
        const double* Km = V.K + V.koff[m - 1];
        double hr = 0.0, hi = 0.0;
        for (int l = V.lm[m - 1]; l <= V.Lm[m - 1]; ++l) {
            const double* row = Km + ((int64_t)(l - V.lm[m - 1]) * q + s) * q;
            for (int r = 0; r < q; ++r) {
                hr += row[r] * V.acc[lap_v(L, q, l, r)];
                hi += row[r] * V.acc[lap_v(L, q, l, r) + 1];
            }
        }
        V.acc[lap_h(L, q, m, s)] = hr;
        V.acc[lap_h(L, q, m, s) + 1] = hi;
    }
}

// The node side: f_j = g_1 on Y_L, else sum_s L_s^{Y_m}(y_j) h^{Y_m}_s + g_{L_m + 1}.
template <class Ctx, typename T>
FLT_HD void lap_body_nodes(const Ctx& ctx, const LapView& V, int64_t M, cplx<T>* f)
{
    const int64_t j = (int64_t)ctx.bid() * ctx.ntid() + ctx.tid();
    if (j >= M) return;
    const int q = V.q, L = V.L;
    const int m = V.band[j];
    double fr, fi;
    if (m >= L) {
        fr = V.acc[lap_g(L, q, 1)];
        fi = V.acc[lap_g(L, q, 1) + 1];
    } else {
        const double yv = V.y[j];
        const double* yn = V.ynodes + (int64_t)(m - 1) * q;
        double den = 0.0;
        int hit = -1;
        for (int s = 0; s < q; ++s) {
            const double d = yv - yn[s];
            if (d == 0.0) hit = s;
            else den += V.bw[s] / d;
        }
        fr = V.acc[lap_g(L, q, V.Lm[m - 1] + 1)];
        fi = V.acc[lap_g(L, q, V.Lm[m - 1] + 1) + 1];
        double ar = 0.0, ai = 0.0;
        for (int s = 0; s < q; ++s) {
            const double w = hit >= 0 ? (s == hit ? 1.0 : 0.0) : V.bw[s] / (yv - yn[s]) / den;
            ar += w * V.acc[lap_h(L, q, m, s)];
            ai += w * V.acc[lap_h(L, q, m, s) + 1];
        }
        fr += ar;
        fi += ai;
    }
    f[j] = mk<T>((T)fr, (T)fi);
}

}  // namespace flt
