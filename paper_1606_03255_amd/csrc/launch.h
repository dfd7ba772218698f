// Launch sequences of the transform (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include "flt_types.h"

namespace flt {

// Device copies of a plan's work lists.
struct DevLists {
    const FftItem* onepass_fwd = nullptr;
    const FftItem* passA_fwd = nullptr;
    const FftItem* passB = nullptr;
    const FftItem* onepass_adj = nullptr;
    const FftItem* passA_adj = nullptr;
    const NodeItem* nodes = nullptr;
    int n_onepass_fwd = 0, n_passA_fwd = 0, n_passB = 0, n_onepass_adj = 0, n_passA_adj = 0, n_nodes = 0;
};

// a2-a6 (forward, or derivative when deriv != 0): c -> f on stream st.
// If ev is not null, ev[0..4] are recorded on st before the first launch and
// after each of the four stages (one-pass FFTs, pass A, pass B, gather).
template <typename T>
hipError_t launch_forward(const DevLists& L, const PlanView<T>& pv, const void* c, void* f, char* ws,
                          size_t off_grid, size_t off_scratch, int deriv, hipStream_t st,
                          hipEvent_t* ev = nullptr);

// a7 (adjoint): g -> c_out on stream st.
template <typename T>
hipError_t launch_adjoint(const DevLists& L, const PlanView<T>& pv, int64_t N, int64_t grid_elems, const void* g,
                          void* c_out, char* ws, size_t off_grid, size_t off_scratch, size_t off_acc,
                          hipStream_t st);

}  // namespace flt
