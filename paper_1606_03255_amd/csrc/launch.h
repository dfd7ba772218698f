// Launch sequences of the transform (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include <vector>

#include "flt_types.h"
#include "laplace.h"
#include "xi_plan.h"

namespace flt {

// The first failure of a launch sequence.  The sequence starts by clearing
// any error an earlier, unrelated call left behind, and the error state is
// read right after every launch, so a later successful launch can neither
// hide a failed one nor can a stale error be reported as this call's.
struct LaunchStatus {
    hipError_t first = hipSuccess;
    LaunchStatus() { (void)hipGetLastError(); }
    void note(hipError_t e)
    {
        if (first == hipSuccess && e != hipSuccess) first = e;
    }
    void launched() { note(hipGetLastError()); }
};

// Device copies of a plan's work lists and index tables.
struct DevLists {
    const FftItem* onepass_fwd = nullptr;
    const FftItem* passA_fwd = nullptr;
    const FftItem* passB = nullptr;
    const FftItem* onepass_adj = nullptr;
    const FftItem* passA_adj = nullptr;
    const FftItem* onepass_fused = nullptr;   // forward + derivative: 2q columns per band
    const FftItem* passB_fused = nullptr;
    const CellItem* cells = nullptr;
    const NodeItem* gather_st = nullptr;   // gather items staged through LDS
    const NodeItem* gather_ln = nullptr;   // gather items read per lane
    const NodeItem* nfft_nodes = nullptr;
    const DirectItem* direct_fwd = nullptr;
    const DirectItem* direct_short = nullptr;   // forward direct sums of short instances (thread groups)
    int n_direct_short = 0;
    const DirectItem* direct_adj = nullptr;
    const int32_t* dlist = nullptr;
    const int32_t* cstart = nullptr;
    const int32_t* clist = nullptr;
    const SumItem* sum_items = nullptr;
    int n_sum = 0;
    int persist_blocks = 512;   // workgroups of the persistent FFT kernels (two per compute unit)
    int n_onepass_fwd = 0, n_passA_fwd = 0, n_passB = 0, n_onepass_adj = 0, n_passA_adj = 0, n_cells = 0;
    int n_onepass_fused = 0, n_passB_fused = 0;
    int n_gather_st = 0, n_gather_ln = 0, n_nfft_nodes = 0, n_direct_fwd = 0, n_direct_adj = 0;
    int64_t n_dlist = 0;
    // host copies of the FFT launch groups (one kernel instance per transform length)
    std::vector<LaunchGroup> g_onepass_fwd, g_passA_fwd, g_passB, g_onepass_adj, g_passA_adj;
};

// Where a call's scratch lives inside the caller's workspace.
struct WsLayout {
    char* ws = nullptr;
    size_t off_grid = 0, off_scratch = 0, off_acc = 0, off_U = 0, off_phi = 0, off_l0 = 0, off_dacc = 0;
    size_t off_base = 0;
    int qs = 1;
    int64_t N = 0, M = 0, grid_elems = 0;
};

// Every launch sequence returns the first error among its launches (and
// event records), or hipSuccess.
//
// a2-a6 (forward, or derivative when deriv != 0): c -> f on stream st; with
// f2 not null, the forward into f and the derivative into f2 in one pass (2q
// columns per band).  If ev is not null, ev[0..5] are recorded on st before
// the first launch and after each stage (one-pass FFTs, pass A, pass B,
// gather, direct bands).
template <typename T>
hipError_t launch_forward(const DevLists& L, const PlanView<T>& pv, const WsLayout& W, const void* c, void* f,
                          void* f2, int deriv, hipStream_t st, hipEvent_t* ev = nullptr);

// Device address of the static scratch array of the forward without a
// workspace on `device` (FLT_NOALLOC_MAX_BYTES bytes), looked up once per
// device with it current (the caller's current device is restored).
hipError_t noalloc_scratch_address(int device, char** out);

// The discrete Laplace transform: fhat -> f on stream st (laplace.hip).
template <typename T>
hipError_t launch_laplace(const LapView& V, const LapItem* items, int nitems, int64_t M, const void* fhat, void* f,
                          hipStream_t st);

// Real exponents (xi.hip), on stream st: the frequency-side spread of c into
// the inner plan's coefficients cin; the node-side combination of the inner
// sums hin into f; the node-side weights of g for the inner transposed sums
// (conj_in: g conjugated); the frequency-side gather of the inner transposed
// sums vin into h through the FP64 accumulator hacc (2N doubles; conj_out: h
// conjugated).  q: the largest band rank (selects the kernel instance).
template <typename T>
hipError_t launch_xi_spread(const XiView<T>& xv, int q, const XiItem* items, int nitems, const void* c, void* cin,
                            hipStream_t st);
template <typename T>
hipError_t launch_xi_combine(const XiView<T>& xv, const NodeItem* items, int nitems, const void* hin, void* f,
                             hipStream_t st);
template <typename T>
hipError_t launch_xi_prep(const XiView<T>& xv, const NodeItem* items, int nitems, const void* g, int conj_in,
                          void* uin, hipStream_t st);
template <typename T>
hipError_t launch_xi_gather(const XiView<T>& xv, int q, const XiItem* items, int nitems, const void* vin,
                            double* hacc, int64_t N, int conj_out, void* h, hipStream_t st);

// a7 (adjoint): g -> c_out on stream st.  If ev is not null, ev[0..8] are
// recorded before the first launch and after each stage (clearing and the
// sum of g, node-side weights, cell spread, pass B, pass A, one-pass bands,
// direct bands, conversion of the FP64 accumulator).
template <typename T>
hipError_t launch_adjoint(const DevLists& L, const PlanView<T>& pv, const WsLayout& W, const void* g, void* c_out,
                          hipStream_t st, hipEvent_t* ev = nullptr);

}  // namespace flt
