/*
 * ORACLE — test infrastructure only.  Nothing in the product path may link,
 * load or call this file; only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg do.
 *
 * Plain FP64 evaluation of the exponential sums that the fast
 * Fourier-Laplace transform approximates (Kunis & Melzer, "Fast evaluation
 * of real and complex exponential sums"):
 *
 *   forward     f_j  = sum_{k=0}^{N-1} c_k w_j^k                  (eq. 4.1, xi_k = k)
 *   adjoint     h_k  = sum_{j=0}^{M-1} g_j conj(w_j)^k            (Sect. 4, closing remarks: C^*)
 *   derivative  f'_j = sum_{k=0}^{N-1} (2 pi i k) c_k w_j^k       (d/dz of f(z) = sum c_k e^{2 pi i k z})
 *
 * with the polar form of eq. 4.2:  w_j = exp(2 pi i z_j) = e^{-y_j} e^{2 pi i x_j},
 * x_j = Re z_j mod 1, y_j = 2 pi Im z_j >= 0.
 *
 * Method (no blocking beyond what keeps the definition exact in FP64):
 *   powers w^k are taken from an exactly re-anchored value every BLK terms,
 *   w^{k0} = e^{-k0 y} * cis(2 pi frac(k0 x)), where frac(k0 x) is formed from
 *   an error-free product (FMA) so the phase carries no k0-amplified error;
 *   inside a block the plain recurrence p <- p w runs for at most BLK steps.
 *   Block sums are combined with Neumaier's compensated summation.
 *   Terms whose magnitude e^{-k0 y} underflows to zero are zero in FP64 and
 *   are skipped.
 *
 * A second, independent algorithm (complex compensated Horner, Graillat &
 * Menissier-Morain) is provided as a cross-check for moderate N.
 *
 * Real exponents (eq. 4.1 with xi_k in [1, N]; Sect. 4, closing remarks: the
 * transposed evaluation g(xi)):
 *
 *   forward_xi     f_j  = sum_k c_k w_j^{xi_k}
 *   transposed_xi  h_k  = sum_j g_j w_j^{xi_k}
 *
 * with the principal power w^p = exp(p Log w), Log w = -y + 2 pi i x_p, where
 * x_p is Re z reduced to (-1/2, 1/2] (arg w in (-pi, pi]); the paper leaves
 * the nonpositive real axis out, the half-open interval fixes its side.  Each
 * term is formed on its own: e^{-xi y} times cis(2 pi frac(xi x_p)), frac
 * from the error-free product as above; sums are Neumaier-compensated.
 *
 * Complex arrays are interleaved (re, im) doubles.  OpenMP parallelises over
 * nodes (forward, derivative, Horner) or over blocks of k (adjoint).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BLK 32
static const double TWO_PI = 6.283185307179586476925286766559;

/* frac(k*x) in [-1/2, 1/2] (plus one rounding), using p = fl(kx), e = kx - p exactly. */
static double frac_kx(double k, double x)
{
    double p = k * x;
    double e = fma(k, x, -p);
    double r = p - nearbyint(p); /* exact: round(p) is a multiple of ulp(p) */
    return r + e;
}

typedef struct { double x, y; int inf; } node_t;

static node_t polar(const double* z)
{
    node_t n;
    double re = z[0], im = z[1];
    n.x = re - floor(re);
    if (n.x >= 1.0) n.x = 0.0; /* only reachable when re is a tiny negative number */
    n.inf = isinf(im) && im > 0;
    n.y = n.inf ? 0.0 : TWO_PI * im;
    return n;
}

static void neumaier(double* s, double* comp, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *comp += (*s - t) + v;
    else                     *comp += (v - t) + *s;
    *s = t;
}

/* sum_k a_k w^k for one node (a interleaved, length N) */
static void eval_one(int64_t N, const double* a, node_t nd, double* out)
{
    if (nd.inf) { out[0] = a[0]; out[1] = a[1]; return; }
    const double mag1 = exp(-nd.y);
    const double wr = mag1 * cos(TWO_PI * nd.x), wi = mag1 * sin(TWO_PI * nd.x);
    double sr = 0, cr = 0, si = 0, ci = 0;
    for (int64_t k0 = 0; k0 < N; k0 += BLK) {
        double mag = exp(-(double)k0 * nd.y);
        if (mag == 0.0) break;
        double ph = TWO_PI * frac_kx((double)k0, nd.x);
        double pr = mag * cos(ph), pi = mag * sin(ph);
        double br = 0, bi = 0;
        int64_t kend = k0 + BLK < N ? k0 + BLK : N;
        for (int64_t k = k0; k < kend; ++k) {
            double ar = a[2 * k], ai = a[2 * k + 1];
            br += ar * pr - ai * pi;
            bi += ar * pi + ai * pr;
            double tr = pr * wr - pi * wi;
            pi = pr * wi + pi * wr;
            pr = tr;
        }
        neumaier(&sr, &cr, br);
        neumaier(&si, &ci, bi);
    }
    out[0] = sr + cr;
    out[1] = si + ci;
}

/* O1 forward: f[j] = sum_{k<N} c_k w_j^k. */
void oracle_forward(int64_t N, int64_t M, const double* c, const double* z, double* f)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < M; ++j) eval_one(N, c, polar(z + 2 * j), f + 2 * j);
}

/* O1 derivative: fp[j] = sum_{k<N} 2 pi i k c_k w_j^k. */
void oracle_derivative(int64_t N, int64_t M, const double* c, const double* z, double* fp)
{
    double* cd = (double*)malloc(sizeof(double) * 2 * (size_t)(N > 0 ? N : 1));
    for (int64_t k = 0; k < N; ++k) {
        double s = TWO_PI * (double)k; /* i*s*(a + ib) = -s b + i s a */
        cd[2 * k]     = -s * c[2 * k + 1];
        cd[2 * k + 1] =  s * c[2 * k];
    }
    oracle_forward(N, M, cd, z, fp);
    free(cd);
}

/* h[k], k0 <= k < kend (kend - k0 <= BLK), of the O1 adjoint: one anchor
 * conj(w_j)^k0 per node, the recurrence inside the block, Neumaier sums over j. */
static void adjoint_block(int64_t k0, int64_t kend, int64_t M, const double* g, const double* z, double* hout)
{
    double sr[BLK], cr[BLK], si[BLK], ci[BLK];
    for (int i = 0; i < BLK; ++i) sr[i] = cr[i] = si[i] = ci[i] = 0;
    for (int64_t j = 0; j < M; ++j) {
        node_t nd = polar(z + 2 * j);
        double gr = g[2 * j], gi = g[2 * j + 1];
        if (nd.inf) { /* conj(w)^k = [k == 0] */
            if (k0 == 0) { neumaier(&sr[0], &cr[0], gr); neumaier(&si[0], &ci[0], gi); }
            continue;
        }
        double mag = exp(-(double)k0 * nd.y);
        if (mag == 0.0) continue;
        double mag1 = exp(-nd.y);
        double wr = mag1 * cos(TWO_PI * nd.x), wi = -mag1 * sin(TWO_PI * nd.x);
        double ph = -TWO_PI * frac_kx((double)k0, nd.x);
        double pr = mag * cos(ph), pi = mag * sin(ph);
        for (int64_t k = k0; k < kend; ++k) {
            int i = (int)(k - k0);
            neumaier(&sr[i], &cr[i], gr * pr - gi * pi);
            neumaier(&si[i], &ci[i], gr * pi + gi * pr);
            double tr = pr * wr - pi * wi;
            pi = pr * wi + pi * wr;
            pr = tr;
        }
    }
    for (int64_t k = k0; k < kend; ++k) {
        int i = (int)(k - k0);
        hout[2 * i] = sr[i] + cr[i];
        hout[2 * i + 1] = si[i] + ci[i];
    }
}

/* O1 adjoint: h[k] = sum_{j<M} g_j conj(w_j)^k, k < N. */
void oracle_adjoint(int64_t N, int64_t M, const double* g, const double* z, double* h)
{
    int64_t nblk = (N + BLK - 1) / BLK;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nblk; ++b) {
        int64_t k0 = b * BLK;
        int64_t kend = k0 + BLK < N ? k0 + BLK : N;
        adjoint_block(k0, kend, M, g, z, h + 2 * k0);
    }
}

/* The O1 adjoint on chosen blocks of BLK consecutive coefficients only (for
 * sizes where all N of them would take too long): block i covers
 * k = BLK*blocks[i] .. BLK*blocks[i] + BLK - 1; h receives BLK values per
 * block (h[BLK*i + t] for k = BLK*blocks[i] + t), entries with k >= N zero. */
void oracle_adjoint_blocks(int64_t N, int64_t M, const double* g, const double* z, int64_t nb,
                           const int64_t* blocks, double* h)
{
    memset(h, 0, sizeof(double) * 2 * BLK * (size_t)(nb > 0 ? nb : 0));
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nb; ++i) {
        int64_t k0 = blocks[i] * BLK;
        if (k0 < 0 || k0 >= N) continue;
        int64_t kend = k0 + BLK < N ? k0 + BLK : N;
        adjoint_block(k0, kend, M, g, z, h + 2 * BLK * i);
    }
}

int oracle_block_size(void) { return BLK; }

/* ---- cross-check: complex compensated Horner on the rounded w_j ---- */
static void two_sum(double a, double b, double* s, double* e)
{
    *s = a + b;
    double z = *s - a;
    *e = (a - (*s - z)) + (b - z);
}
static void two_prod(double a, double b, double* p, double* e)
{
    *p = a * b;
    *e = fma(a, b, -*p);
}

/* Evaluates sum_k c_k w^k with w = fl(e^{-y} cis(2 pi x)) exactly-rounded-ish
 * (error ~ u|f| + O(N^2 u^2) sum|c_k||w|^k for the rounded w).  The rounding
 * of w itself is amplified by k, so this agrees with oracle_forward only to
 * ~k*u relative: use for N up to ~1e3. */
void oracle_horner_comp(int64_t N, int64_t M, const double* c, const double* z, double* f)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < M; ++j) {
        node_t nd = polar(z + 2 * j);
        if (nd.inf || N == 0) {
            f[2 * j] = N ? c[0] : 0; f[2 * j + 1] = N ? c[1] : 0; continue;
        }
        double mag1 = exp(-nd.y);
        double wr = mag1 * cos(TWO_PI * nd.x), wi = mag1 * sin(TWO_PI * nd.x);
        double sr = c[2 * (N - 1)], si = c[2 * (N - 1) + 1];
        double er = 0, ei = 0;
        for (int64_t k = N - 2; k >= 0; --k) {
            double p1, e1, p2, e2, p3, e3, p4, e4, h1, g1, h2, g2, g3, g4;
            two_prod(sr, wr, &p1, &e1);
            two_prod(si, wi, &p2, &e2);
            two_prod(sr, wi, &p3, &e3);
            two_prod(si, wr, &p4, &e4);
            two_sum(p1, -p2, &h1, &g1);
            two_sum(p3, p4, &h2, &g2);
            two_sum(h1, c[2 * k], &sr, &g3);
            two_sum(h2, c[2 * k + 1], &si, &g4);
            double lr = (e1 - e2) + (g1 + g3);
            double li = (e3 + e4) + (g2 + g4);
            double tr = er * wr - ei * wi + lr;
            ei = er * wi + ei * wr + li;
            er = tr;
        }
        f[2 * j] = sr + er;
        f[2 * j + 1] = si + ei;
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Real exponents.  x_p: Re z reduced to (-1/2, 1/2].
 * ------------------------------------------------------------------------ */
static double principal_x(double re)
{
    double x = re - floor(re);
    if (x >= 1.0) x = 0.0;
    return x > 0.5 ? x - 1.0 : x;
}

/* w^xi = e^{-xi y} cis(2 pi xi x_p) (0 for Im z = +inf) */
static void principal_pow(double xi, double xp, double y, int inf, double* re, double* im)
{
    if (inf) { *re = 0.0; *im = 0.0; return; }
    double mag = exp(-xi * y);
    double ph = TWO_PI * frac_kx(xi, xp);
    *re = mag * cos(ph);
    *im = mag * sin(ph);
}

void oracle_forward_xi(int64_t N, const double* xi, const double* c, int64_t M, const double* z, double* f)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < M; ++j) {
        const double im = z[2 * j + 1];
        const int inf = isinf(im) && im > 0;
        const double y = inf ? 0.0 : TWO_PI * im, xp = principal_x(z[2 * j]);
        double sr = 0, cr = 0, si = 0, ci = 0;
        for (int64_t k = 0; k < N; ++k) {
            double pr, pi;
            principal_pow(xi[k], xp, y, inf, &pr, &pi);
            if (pr == 0.0 && pi == 0.0) continue;
            const double ar = c[2 * k], ai = c[2 * k + 1];
            neumaier(&sr, &cr, ar * pr - ai * pi);
            neumaier(&si, &ci, ar * pi + ai * pr);
        }
        f[2 * j] = sr + cr;
        f[2 * j + 1] = si + ci;
    }
}

void oracle_transposed_xi(int64_t M, const double* z, const double* g, int64_t N, const double* xi, double* h)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < N; ++k) {
        double sr = 0, cr = 0, si = 0, ci = 0;
        for (int64_t j = 0; j < M; ++j) {
            const double im = z[2 * j + 1];
            const int inf = isinf(im) && im > 0;
            const double y = inf ? 0.0 : TWO_PI * im, xp = principal_x(z[2 * j]);
            double pr, pi;
            principal_pow(xi[k], xp, y, inf, &pr, &pi);
            if (pr == 0.0 && pi == 0.0) continue;
            const double ar = g[2 * j], ai = g[2 * j + 1];
            neumaier(&sr, &cr, ar * pr - ai * pi);
            neumaier(&si, &ci, ar * pi + ai * pr);
        }
        h[2 * k] = sr + cr;
        h[2 * k + 1] = si + ci;
    }
}
