// Real exponents (eq. 4.1 with xi_k in [1, N]; the transposed evaluation
// g(xi) of Sect. 4): host planner.
//
// The Laplace side is the integer plan's: its node partition (Def. 3.2),
// Chebyshev tables and barycentric y-weights serve unchanged, the interpolant
// t_{m,s}(xi) of a block being a polynomial in continuous xi.  The Fourier
// side of band m, column s, sum_k c_k t_{m,s}(xi_k) e^{2 pi i xi_k x}, is an
// NNFFT: a Kaiser-Bessel window rho in frequency spreads the real xi_k onto
// the integers l (spacing 1/sigma in xi),
//
//   e^{2 pi i xi x} ~ (1 / rho_hat(x / sigma)) sum_l rho(sigma xi - l) e^{2 pi i l x / sigma},
//
// (Poisson summation; aliases at x / sigma + r, r != 0, the same geometry as
// the NFFT's), leaving an integer-frequency sum at the nodes x / sigma that
// one batched integer plan evaluates for every (band, column) at once.
#pragma once
#include <stdint.h>

#include <vector>

#include "plan_host.h"

namespace flt {

// One NFFT band of the real-exponent plan (q = 0: the Z^0 band, f = 0 there).
struct XiBand {
    int32_t q;           // columns (the band's rank; 1 for Y_D)
    int32_t ell_lo, ell_hi;   // interpolated blocks (ell_hi < ell_lo: none, t = 1)
    int32_t n_xi;        // xi_1 = 2^n_xi
    int32_t coef_off;    // Chebyshev table of block ell_lo (q * q per block)
    int32_t ycheb_off;   // q (node, weight) pairs of the y interpolation
    int32_t pad0, pad1;
    double sig;          // frequency grid density sigma (l = sigma xi)
    double kb_b;         // window shape b = pi (2 - 1 / sigma)
    int64_t l_lo;        // integer frequencies l = l_lo .. l_lo + l_count - 1
    int64_t l_count;
    int64_t k_end;       // sorted exponents xi_k, k < k_end, lie in the band's support
    int64_t node_start;  // sorted nodes of the band
    int64_t node_count;
    int64_t cin_off;     // inner coefficients of column s: cin_off + s l_count
    int64_t hout_off;    // inner node values of column s: hout_off + s node_count
};

// Work item of the frequency-side kernels: a run of a band's integer
// frequencies (spread) or of its sorted exponents (transposed gather), with
// the range of exponents they touch and the interpolated blocks among them.
struct XiItem {
    int32_t band;
    int32_t count;       // frequencies / exponents in the run (<= 256)
    int64_t first;       // first l - l_lo (spread) or first k (gather)
    int64_t k_lo, k_hi;  // exponents the run's windows reach (spread)
    int32_t blk_lo;      // blocks ell_lo + blk_lo .. + nblk - 1 staged in LDS (nblk <= XI_NBLK)
    int32_t nblk;        // -1: more than XI_NBLK blocks, read from global memory
};

constexpr int XI_THREADS = 256;
constexpr int XI_NBLK = 8;          // interpolated blocks staged per item at most

struct XiHost {
    int64_t N = 0, M = 0;
    int dtype = 0;
    double eps = 0, eps_w = 0, eps_in = 0;
    int mw1 = 0;                     // frequency window half-width
    double sig_min = 0, amp = 0;     // smallest sigma used; inner-error amplification
    HostPlan outer;                  // the integer plan's partition (tables, sorted nodes)
    std::vector<double> xi;          // exponents, ascending
    std::vector<int32_t> xi_perm;    // caller index of sorted exponent k
    std::vector<double> xp;          // sorted nodes: Re z reduced to (-1/2, 1/2]
    std::vector<XiBand> bands;       // one per outer band, same index
    std::vector<XiItem> spread, gather;
    std::vector<NodeItem> nodes;     // node items of every band (Z^0 included)
    // the inner batched integer plan: instance (b, s) for every NFFT band b
    // and column s, l_count coefficients, the band's nodes at x / sigma
    std::vector<int64_t> in_N, in_M;
    std::vector<double> in_z;        // packed (Re, Im) of every instance's nodes
    int64_t cin_elems = 0, hout_elems = 0;
};

// What the real-exponent kernels read from the plan.
template <typename T> struct XiView {
    const XiBand* bands;
    const T* coef;           // the integer plan's Chebyshev table
    const double* ycheb;     // its y nodes and barycentric weights
    const double* xi;        // exponents, ascending
    const int32_t* xi_perm;  // caller index of sorted exponent k
    const double* xp;        // sorted nodes: Re z in (-1/2, 1/2]
    const double* ny;        // sorted nodes: y = 2 pi Im z
    const int32_t* perm;     // caller index of sorted node j
    int32_t mw1;             // frequency window half-width
};

// Returns FLT_OK or a negative FLT_E* code.  xi: N finite exponents >= 1
// (any order); z: M nodes (Re, Im interleaved, Im >= 0).
int build_xi_plan(XiHost& hp, int64_t N, const double* xi, int64_t M, const double* z, double eps, int dtype);

// The error bound of the truncated Kaiser-Bessel window with half-width m and
// oversampling sigma (the NFFT's, which by symmetry also bounds the
// frequency-side spread).
double kb_bound(int m, double sigma);

}  // namespace flt
