// Host planner: parameters (Def. 3.2, Lemma 4.1), node partition and sort,
// interpolation / window / twiddle tables, work lists and workspace layout.
// Pure C++ (FP64); the HIP library uploads what it builds.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "flt_types.h"

namespace flt {

struct HostPlan {
    // parameters
    int64_t N = 0, M = 0;
    int dtype = 0;
    double eps = 0, eps_K = 0, eps_A = 0, y1 = 0;
    int q = 0, D = 0, n_xi = 0, mw = 0;
    double kb_b = 0;
    int64_t nodes_z0 = 0;

    // bands: occupied Y_m / Y_D first (ascending m), then the constant band (Z^0) if any
    std::vector<BandDesc> bands;
    std::vector<int32_t> band_m;      // paper index m of each band (D for Y_D, 0 for Z^0)
    std::vector<int32_t> node_band;   // caller order: 0 = Z^0, m, D

    // sorted nodes
    std::vector<double> nx, ny;
    std::vector<int32_t> perm;

    // tables in FP64 (rounded to the working type on upload)
    std::vector<double> coef, deconv, ycheb;
    std::vector<double> tw_stage, tw_lo, tw_hi;   // interleaved complex

    uint32_t flags = 0;
    double direct_scale = 1.0;          // factor on the direct-sum rate of the band policy

    // work lists
    std::vector<FftItem> onepass_fwd, passA_fwd, passB, onepass_adj, passA_adj;
    // forward + derivative in one pass: the lists over 2q columns per band
    // (the derivative's column s is column q + s; pass A's list serves both)
    std::vector<FftItem> onepass_fused, passB_fused;
    std::vector<CellItem> cells;        // adjoint grid side: cell groups of the NFFT bands
    // FFT item lists are sorted by transform length; one group per length
    std::vector<LaunchGroup> g_onepass_fwd, g_passA_fwd, g_passB, g_onepass_adj, g_passA_adj;
    std::vector<LaunchGroup> g_onepass_fused, g_passB_fused;
    // gather: items whose nodes' windows cover a run of at most GATHER_STAGE
    // cells (staged in LDS), and the rest (the constant band's included)
    std::vector<NodeItem> gather_st, gather_ln;
    std::vector<NodeItem> nfft_nodes;   // adjoint node side: NFFT bands only
    std::vector<int32_t> dlist;         // sorted indices of the nodes of direct bands
    std::vector<DirectItem> direct_fwd, direct_adj;
    std::vector<DirectItem> direct_short;   // the forward's short sums (log2tpg < 8)
    std::vector<int32_t> cstart;        // per NFFT band: first sorted node with cell >= c, c = 0..n
    std::vector<int32_t> clist;         // touched cells of the listed cell items (-1 pads)
    std::vector<uint32_t> mask;         // per two-pass band: bit per grid address read by some window
    std::vector<InstDesc> inst;         // instances: one, or the members of a batched plan
    std::vector<SumItem> sum_items;     // adjoint k = 0 sums: runs of one instance's g

    // workspace layout (bytes)
    int qs = 1;                         // stride of the per-node column values (max q, rounded up to even)
    int64_t grid_elems = 0, scratch_elems = 0, base_elems = 0;   // base: FP64 plans only
    size_t off_grid = 0, off_scratch = 0, off_acc = 0, off_U = 0, off_phi = 0, off_l0 = 0, off_dacc = 0;
    size_t off_base = 0;
    size_t ws_bytes = 0;
    // the forward alone (one column set per band): grids, pass-A output,
    // direct-sum accumulator and FP64 base slots, packed; what a forward
    // without a registered workspace needs
    size_t fwd_off_scratch = 0, fwd_off_dacc = 0, fwd_off_base = 0, fwd_ws_bytes = 0;

    // algorithmic model
    double bytes_forward = 0, flops_forward = 0;

    size_t elem_bytes() const { return dtype == 1 ? 8 : 16; }   // complex element
};

// Planner-internal flag (never accepted from callers): accept eps below the
// dtype's floor.  The real-exponent plan's inner integer sums need it: their
// error is amplified by the frequency window, and FP32 sums of unit-modulus
// terms still reach well below 1e-6 in practice.
constexpr uint32_t PLAN_FLAG_NO_FLOOR = 1u << 30;

// Returns FLT_OK or a negative FLT_E* code (see flt.h).
// Tunable shape of a plan (the autotuner's search space): the band policy's
// direct-sum rate factor.
struct PlanShape {
    double direct_scale = 1.0;
};

int build_host_plan(HostPlan& hp, int64_t N, int64_t M, const double* z, double eps, int dtype,
                    uint32_t flags = 0, PlanShape shape = PlanShape());

// One plan for `count` independent instances (N[i] coefficients, M[i] nodes,
// z packed instance after instance): the members' bands, nodes and work lists
// side by side, with shared interpolation / window / twiddle tables.  The
// packed c (and adjoint output) holds instance i at sum_{i' < i} N[i'], the
// packed f (and adjoint input) at sum_{i' < i} M[i'].
int build_batch_plan(HostPlan& hp, int32_t count, const int64_t* N, const int64_t* M, const double* z, double eps,
                     int dtype, uint32_t flags = 0, PlanShape shape = PlanShape());

// Modified Bessel function I_0 by its power series (host, FP64).
double bessel_i0(double x);

}  // namespace flt
