// gfx950 kernels of the discrete Laplace transform (Sect. 3, Algorithm 1) and
// their launch sequence; the bodies are in laplace.h.
#include <hip/hip_runtime.h>

#include "laplace.h"
#include "launch.h"

namespace flt {

struct LapCtx {
    __device__ __forceinline__ int tid() const { return (int)threadIdx.x; }
    __device__ __forceinline__ int ntid() const { return (int)blockDim.x; }
    __device__ __forceinline__ int bid() const { return (int)blockIdx.x; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
};

template <typename T, int QB>
__global__ __launch_bounds__(LAP_THREADS) void k_lap_moments(LapView V, const LapItem* items, const cplx<T>* fhat)
{
    __shared__ double red[8 * LAP_THREADS], red2[LAP_THREADS];
    lap_body_moments<LapCtx, T, QB>(LapCtx(), V, items, fhat, red, red2);
}

__global__ __launch_bounds__(LAP_THREADS) void k_lap_reduce(LapView V)
{
    __shared__ double red[LAP_THREADS];
    lap_body_reduce(LapCtx(), V, red);
}

template <int QB>
__global__ __launch_bounds__(LAP_THREADS) void k_lap_bands(LapView V)
{
    __shared__ double red[4 * LAP_THREADS];
    lap_body_bands<LapCtx, QB>(LapCtx(), V, red);
}

template <typename T, int QB>
__global__ __launch_bounds__(LAP_THREADS) void k_lap_nodes(LapView V, int64_t M, cplx<T>* f, int staged,
                                                             const cplx<T>* fhat)
{
    extern __shared__ double sb[];   // lap_node_stage(L, q) doubles when staged
    lap_body_nodes<LapCtx, T, QB>(LapCtx(), V, M, f, staged ? sb : nullptr, fhat);
}

// Item partials of the block moments, their sum per block, band side, node
// side, at one rank bucket.  Every accumulator is written in full by each call.
template <typename T, int QB>
static void launch_all(LaunchStatus& ls, const LapView& V, const LapItem* items, int nitems, int64_t M,
                       const void* fhat, void* f, hipStream_t st)
{
    hipLaunchKernelGGL((k_lap_moments<T, QB>), dim3(nitems), dim3(LAP_THREADS), 0, st, V, items, (const cplx<T>*)fhat);
    ls.launched();
    hipLaunchKernelGGL(k_lap_reduce, dim3((unsigned)V.L), dim3(LAP_THREADS), 0, st, V);
    ls.launched();
    hipLaunchKernelGGL(k_lap_bands<QB>, dim3((unsigned)V.L), dim3(LAP_THREADS), 0, st, V);
    ls.launched();
    const int64_t per = (int64_t)LAP_THREADS * LAP_NODE_PER, ns = lap_node_stage(V.L, V.q);
    hipLaunchKernelGGL((k_lap_nodes<T, QB>), dim3((unsigned)((M + per - 1) / per)), dim3(LAP_THREADS),
                       (unsigned)(ns * sizeof(double)), st, V, M, (cplx<T>*)f, ns > 0 ? 1 : 0,
                       (const cplx<T>*)fhat);
    ls.launched();
}

template <typename T>
hipError_t launch_laplace(const LapView& V, const LapItem* items, int nitems, int64_t M, const void* fhat, void* f,
                          hipStream_t st)
{
    LaunchStatus ls;
    switch (lap_qbucket(V.q)) {
    case 8: launch_all<T, 8>(ls, V, items, nitems, M, fhat, f, st); break;
    case 12: launch_all<T, 12>(ls, V, items, nitems, M, fhat, f, st); break;
    case 16: launch_all<T, 16>(ls, V, items, nitems, M, fhat, f, st); break;
    case 24: launch_all<T, 24>(ls, V, items, nitems, M, fhat, f, st); break;
    default: launch_all<T, 32>(ls, V, items, nitems, M, fhat, f, st); break;
    }
    return ls.first;
}

template hipError_t launch_laplace<float>(const LapView&, const LapItem*, int, int64_t, const void*, void*,
                                          hipStream_t);
template hipError_t launch_laplace<double>(const LapView&, const LapItem*, int, int64_t, const void*, void*,
                                           hipStream_t);

}  // namespace flt
