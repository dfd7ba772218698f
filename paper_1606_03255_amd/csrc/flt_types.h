// Types shared by the host planner and the kernels.
#pragma once
#include <stdint.h>

#if defined(__HIP__)
#include <hip/hip_runtime.h>
#else  // host-only translation units (planner, CPU build of the kernel bodies)
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#ifndef __forceinline__
#define __forceinline__ inline
#endif
#endif

#define FLT_HD __host__ __device__ __forceinline__

namespace flt {

template <typename T> struct alignas(2 * sizeof(T)) cplx { T x, y; };

template <typename T> FLT_HD cplx<T> mk(T a, T b) { cplx<T> r; r.x = a; r.y = b; return r; }
// Two adjacent complex values at a 16-byte boundary: one 16-byte load or store
// in FP32 (the gather's paired window reads, the adjoint's column pairs).
template <typename T> struct alignas(16) cplx2 { cplx<T> a, b; };
template <typename T> FLT_HD cplx2<T> load_pair(const cplx<T>* p) { return *reinterpret_cast<const cplx2<T>*>(p); }
template <typename T> FLT_HD void store_pair(cplx<T>* p, const cplx2<T>& v) { *reinterpret_cast<cplx2<T>*>(p) = v; }
// Two adjacent reals at their joint alignment.
template <typename T> struct alignas(2 * sizeof(T)) RealPair { T a, b; };
template <typename T> FLT_HD cplx<T> add(cplx<T> a, cplx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> FLT_HD cplx<T> sub(cplx<T> a, cplx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> FLT_HD cplx<T> mul(cplx<T> a, cplx<T> b)
{
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> FLT_HD cplx<T> scale(cplx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by i*sign (sign = +1 or -1)
template <typename T> FLT_HD cplx<T> mul_isign(cplx<T> a, int sign)
{
    return sign > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

// Sizes fixed at compile time.
constexpr int FFT_THREADS = 512;          // threads of every FFT workgroup
constexpr int TW_STAGE_LOG2 = 13;         // stage twiddle table: e^{-2 pi i t / 2^13}
constexpr int TW2_LOG2 = 22;              // two-level table resolution 2^22 (largest grid)
constexpr int TW2_HALF = 11;              // lo/hi tables of 2^11 entries each
constexpr int GATHER_THREADS = 256;       // nodes per gather/spread workgroup
constexpr int GATHER_STAGE = 2048;        // grid values a gather workgroup stages in LDS at a time
constexpr int MAX_Q = 32;                 // largest Chebyshev rank supported
constexpr int MAX_MW = 10;                // largest window half-width supported
constexpr int DIRECT_TPT = 32;            // direct sum: terms per thread and chunk (one anchor each)
constexpr int DIRECT_NG = 8;              // direct sum: nodes per thread group
constexpr int DIRECT_GMAX = 32;           // direct sum: most thread groups per workgroup (short sums)
// direct sum: most chunks of 256 * DIRECT_TPT terms per workgroup, by working type
constexpr int direct_cpw(int dtype_bytes) { return dtype_bytes == 4 ? 4 : 1; }
constexpr int DIRECT_ANG = 256;           // direct adjoint: nodes per workgroup
// direct adjoint: consecutive coefficients per thread (one anchor each); 16 for
// both working types (more workgroups: the sums have few nodes to spread over)
constexpr int direct_atpt(int /*dtype_bytes*/) { return 16; }
constexpr int SUMG_PER_THREAD = 16;       // sum of g: elements per thread
constexpr int CELL_TARGET = 16;           // adjoint spread: contributions per thread a cell's group aims at

template <typename T> struct Sizes;
// LOG2P: FFT tile of 2^LOG2P complex values (64 KB); COEF: LDS slots for one
// column's Chebyshev coefficients of every block of a band.  Tile plus
// coefficients stay under 80 KB, so two 512-thread workgroups share a CU.
template <> struct Sizes<float>  { static constexpr int LOG2P = 13; static constexpr int COEF = 2048; };
template <> struct Sizes<double> { static constexpr int LOG2P = 12; static constexpr int COEF = 1472; };

// Physical slot of element i of an FFT tile in LDS: one pad slot after every
// 16 elements, so that the strided stores of the Stockham stages fall on
// different banks (offsets of multiples of 16 stay compile-time constants).
FLT_HD int lds_at(int i) { return i + (i >> 4); }
template <typename T> constexpr int tile_alloc() { return (1 << Sizes<T>::LOG2P) + (1 << (Sizes<T>::LOG2P - 4)); }

// One occupied band of the node partition (Def. 3.2 Y_m, or Y_D), or the
// constant band (q = 0) that holds the Z^0 nodes.
struct BandDesc {
    int32_t q;           // columns; 0 for the constant band
    int32_t log2n;       // NFFT grid length n = 2^log2n
    int32_t log2n1;      // first FFT factor (log2n for a one-pass band)
    int32_t log2n2;      // second factor, log2n - log2n1 (0 for one pass)
    int32_t log2b;       // pass A: sub-transforms per workgroup
    int32_t log2B;       // pass B: sub-transforms per workgroup = width of the blocked layout
    int32_t ell_lo;      // interpolated frequency blocks ell_lo..ell_hi (ell_hi < ell_lo: none)
    int32_t ell_hi;
    int32_t n_xi;        // xi_1 = 2^n_xi
    int32_t coef_off;    // first coefficient of block ell_lo in the Chebyshev table (q*q per block)
    int32_t deconv_off;  // deconvolution table of this n: entries |k'| = 0..n/4
    int32_t ycheb_off;   // q (node, weight) pairs of the y interpolation in the ycheb table
    int32_t direct;      // 1: the band's nodes are evaluated by the direct sum (no grids)
    int64_t k0;          // centre of the frequency support
    int64_t kmax;        // support is k = 1..kmax
    int64_t grid_off;    // complex offset of the band's q grids (column-major, n each)
    int64_t scratch_off; // complex offset of the band's pass-A output (two-pass bands)
    int64_t node_start;  // first node of the band in the sorted node arrays
    int64_t node_count;
    int64_t cs_off;      // cell-start table of the band (n + 1 entries) for the adjoint
    int64_t mask_off;    // two-pass bands: first 32-bit word of the cell mask (bit per grid address)
    int64_t base_off;    // FP64 pass A: complex offset of the band's per-point c_k / (n phi_hat) slots
    int64_t cells;       // grid cells per column that some node's window reads
    int64_t c_off;       // first coefficient of the band's instance in the packed c (and adjoint output)
};

// Address of natural grid index l in a band's blocked layout
// [l1 / B][l2][l1 mod B], l = l1 + n1 l2  (one-pass bands: address = l).
FLT_HD int64_t grid_addr(const BandDesc& B, int64_t l)
{
    const int64_t l1 = l & (((int64_t)1 << B.log2n1) - 1);
    const int64_t l2 = l >> B.log2n1;
    return ((l1 >> B.log2B) << (B.log2n2 + B.log2B)) + (l2 << B.log2B) + (l1 & (((int64_t)1 << B.log2B) - 1));
}

// Work item of an FFT kernel: band, first column, and a block index.
struct FftItem {
    int32_t band;
    int32_t s0;          // first column
    int32_t ns;          // columns in this item (one-pass kernel) / unused
    int32_t blk;         // j2-block (pass A) or l1-block (pass B)
};

// A run of work items that share the FFT length 2^log2 (one kernel instance).
struct LaunchGroup {
    int32_t log2;
    int32_t start;
    int32_t count;
    int32_t pad;
};

// Work item of the node kernels: up to GATHER_THREADS consecutive sorted nodes of one band.
struct NodeItem {
    int32_t band;
    int32_t count;
    int64_t start;
};

// Work item of the adjoint's grid side: 256 >> log2tpc cells of a band, each
// summed by a group of 2^log2tpc threads: consecutive cells from cell0, or
// (listed) the entries clist[cell0 ..] of the plan's list of touched cells
// (-1: none).
struct CellItem {
    int32_t band;
    int32_t cell0;
    int32_t log2tpc;
    int32_t listed;
};

// Work item of the direct-sum kernels: a run of the direct-node list and a chunk of k.
struct DirectItem {
    int32_t first;       // first entry of the run in the direct-node list
    int16_t count;       // nodes in the run
    int16_t nch;         // forward: chunks of 2^log2tpg * DIRECT_TPT terms, from `chunk` on
    int32_t chunk;
    int32_t inst;        // instance whose coefficients the chunks cover
    int32_t log2tpg;     // forward: threads per group of DIRECT_NG nodes (8: the whole workgroup;
                         // fewer for short sums, the groups then splitting the workgroup)
};

// One instance of a plan (a single plan has one; a batched plan one per
// member): where its coefficients and nodes sit in the packed arrays.
struct InstDesc {
    int64_t c_off, N;    // coefficients c_off .. c_off + N - 1
    int64_t f_off, M;    // nodes (caller order) f_off .. f_off + M - 1
};

// Work item of the adjoint's k = 0 sum: a run of one instance's g.
struct SumItem {
    int32_t inst;
    int32_t pad;
    int64_t start;       // caller index of the run's first node
};

// Everything a kernel needs to read from the plan (device or host pointers).
template <typename T> struct PlanView {
    const BandDesc* bands;
    const T* coef;           // Chebyshev coefficients a[s][i] per (band, block)
    const T* deconv;         // 1 / (n phi_hat(k')) per distinct n
    const double* ycheb;     // per band: q pairs (y_s, lambda_s)
    const cplx<T>* tw_stage; // e^{-2 pi i t / 2^13}
    const cplx<T>* tw_lo;    // e^{-2 pi i t / 2^22},        t < 2^11
    const cplx<T>* tw_hi;    // e^{-2 pi i t 2^11 / 2^22},   t < 2^11
    const double* nx;        // sorted nodes: x in [0,1)
    const double* ny;        //               y = 2 pi Im z
    const int32_t* perm;     //               caller index
    const uint32_t* mask;    // cell masks of the two-pass bands (bit set: some window reads the cell)
    const InstDesc* inst;    // instances (one for a single plan)
    int32_t mw;              // window half-width
    T kb_b;                  // Kaiser-Bessel shape b = pi (2 - 1/sigma)
};

}  // namespace flt
