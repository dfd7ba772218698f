// gfx950 kernels of the discrete Laplace transform (Sect. 3, Algorithm 1) and
// their launch sequence; the bodies are in laplace.h.
#include <hip/hip_runtime.h>

#include "laplace.h"

namespace flt {

struct LapCtx {
    __device__ __forceinline__ int tid() const { return (int)threadIdx.x; }
    __device__ __forceinline__ int ntid() const { return (int)blockDim.x; }
    __device__ __forceinline__ int bid() const { return (int)blockIdx.x; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
    __device__ __forceinline__ void atomic_add(double* p, double v) const { unsafeAtomicAdd(p, v); }
};

__global__ __launch_bounds__(LAP_THREADS) void k_lap_zero(double* acc, int64_t n)
{
    lap_body_zero(LapCtx(), acc, n);
}

template <typename T>
__global__ __launch_bounds__(LAP_THREADS) void k_lap_moments(LapView V, const LapItem* items, const cplx<T>* fhat)
{
    __shared__ double sden[LAP_CHUNK], sf[2 * LAP_CHUNK], red[4 * LAP_THREADS];
    __shared__ int32_t shit[LAP_CHUNK];
    lap_body_moments<LapCtx, T>(LapCtx(), V, items, fhat, sden, shit, sf, red);
}

__global__ __launch_bounds__(LAP_THREADS) void k_lap_bands(LapView V)
{
    lap_body_bands(LapCtx(), V);
}

template <typename T>
__global__ __launch_bounds__(LAP_THREADS) void k_lap_nodes(LapView V, int64_t M, cplx<T>* f)
{
    lap_body_nodes<LapCtx, T>(LapCtx(), V, M, f);
}

// Clear the accumulators, block moments and sums, band side, node side.
template <typename T>
hipError_t launch_laplace(const LapView& V, const LapItem* items, int nitems, int64_t M, const void* fhat, void* f,
                          hipStream_t st)
{
    const int64_t n = lap_acc_doubles(V.L, V.q);
    hipLaunchKernelGGL(k_lap_zero, dim3((unsigned)((n + LAP_THREADS - 1) / LAP_THREADS)), dim3(LAP_THREADS), 0, st,
                       V.acc, n);
    hipLaunchKernelGGL(k_lap_moments<T>, dim3(nitems), dim3(LAP_THREADS), 0, st, V, items, (const cplx<T>*)fhat);
    hipLaunchKernelGGL(k_lap_bands, dim3(1), dim3(LAP_THREADS), 0, st, V);
    hipLaunchKernelGGL(k_lap_nodes<T>, dim3((unsigned)((M + LAP_THREADS - 1) / LAP_THREADS)), dim3(LAP_THREADS), 0,
                       st, V, M, (cplx<T>*)f);
    return hipGetLastError();
}

template hipError_t launch_laplace<float>(const LapView&, const LapItem*, int, int64_t, const void*, void*,
                                          hipStream_t);
template hipError_t launch_laplace<double>(const LapView&, const LapItem*, int, int64_t, const void*, void*,
                                           hipStream_t);

}  // namespace flt
