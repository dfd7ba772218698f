// gfx950 kernels of the real-exponent transform and the frequency- and
// node-side launch sequences around the inner integer sums; the bodies are in
// xi_impl.h.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "xi_impl.h"

namespace flt {

struct XiCtx {
    __device__ __forceinline__ int tid() const { return (int)threadIdx.x; }
    __device__ __forceinline__ int ntid() const { return (int)blockDim.x; }
    __device__ __forceinline__ int bid() const { return (int)blockIdx.x; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
    __device__ __forceinline__ void atomic_add(double* p, double v) const { unsafeAtomicAdd(p, v); }
};

// LDS of the staged interpolated blocks: XI_NBLK blocks of q x q coefficients.
template <typename T, int QM> constexpr int xi_lc() { return XI_NBLK * QM * QM; }
static_assert(xi_lc<double, 32>() * sizeof(double) <= 64 * 1024, "staged blocks of the real-exponent kernels");

template <typename T, int QM>
__global__ __launch_bounds__(XI_THREADS) void k_xi_spread(XiView<T> xv, const XiItem* items, const cplx<T>* c,
                                                          cplx<T>* cin)
{
    __shared__ T lc[xi_lc<T, QM>()];
    __shared__ cplx<T> ct[xi_kcap<T, QM>() * QM];
    body_xi_spread<XiCtx, T, QM>(XiCtx(), xv, items, c, cin, lc, ct);
}

template <typename T>
__global__ __launch_bounds__(GATHER_THREADS) void k_xi_combine(XiView<T> xv, const NodeItem* items,
                                                               const cplx<T>* hin, cplx<T>* f)
{
    body_xi_combine<XiCtx, T>(XiCtx(), xv, items, hin, f);
}

template <typename T>
__global__ __launch_bounds__(GATHER_THREADS) void k_xi_prep(XiView<T> xv, const NodeItem* items, const cplx<T>* g,
                                                            int conj_in, cplx<T>* uin)
{
    body_xi_prep<XiCtx, T>(XiCtx(), xv, items, g, conj_in, uin);
}

template <typename T, int QM>
__global__ __launch_bounds__(XI_THREADS) void k_xi_gather(XiView<T> xv, const XiItem* items, const cplx<T>* vin,
                                                          double* hacc)
{
    __shared__ T lc[xi_lc<T, QM>()];
    body_xi_gather<XiCtx, T, QM>(XiCtx(), xv, items, vin, hacc, lc);
}

template <typename T>
__global__ __launch_bounds__(XI_THREADS) void k_xi_finalize(XiView<T> xv, int64_t N, const double* hacc,
                                                            int conj_out, cplx<T>* h)
{
    body_xi_finalize<XiCtx, T>(XiCtx(), xv, N, hacc, conj_out, h);
}

__global__ __launch_bounds__(XI_THREADS) void k_xi_zero(double* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * XI_THREADS + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <typename T>
hipError_t launch_xi_spread(const XiView<T>& xv, int q, const XiItem* items, int nitems, const void* c, void* cin,
                            hipStream_t st)
{
    LaunchStatus ls;
    if (nitems > 0) {
        if (q <= 16)
            hipLaunchKernelGGL((k_xi_spread<T, 16>), dim3(nitems), dim3(XI_THREADS), 0, st, xv, items,
                               (const cplx<T>*)c, (cplx<T>*)cin);
        else if (q <= 24)
            hipLaunchKernelGGL((k_xi_spread<T, 24>), dim3(nitems), dim3(XI_THREADS), 0, st, xv, items,
                               (const cplx<T>*)c, (cplx<T>*)cin);
        else
            hipLaunchKernelGGL((k_xi_spread<T, 32>), dim3(nitems), dim3(XI_THREADS), 0, st, xv, items,
                               (const cplx<T>*)c, (cplx<T>*)cin);
        ls.launched();
    }
    return ls.first;
}

template <typename T>
hipError_t launch_xi_combine(const XiView<T>& xv, const NodeItem* items, int nitems, const void* hin, void* f,
                             hipStream_t st)
{
    LaunchStatus ls;
    if (nitems > 0) {
        hipLaunchKernelGGL(k_xi_combine<T>, dim3(nitems), dim3(GATHER_THREADS), 0, st, xv, items,
                           (const cplx<T>*)hin, (cplx<T>*)f);
        ls.launched();
    }
    return ls.first;
}

template <typename T>
hipError_t launch_xi_prep(const XiView<T>& xv, const NodeItem* items, int nitems, const void* g, int conj_in,
                          void* uin, hipStream_t st)
{
    LaunchStatus ls;
    if (nitems > 0) {
        hipLaunchKernelGGL(k_xi_prep<T>, dim3(nitems), dim3(GATHER_THREADS), 0, st, xv, items, (const cplx<T>*)g,
                           conj_in, (cplx<T>*)uin);
        ls.launched();
    }
    return ls.first;
}

template <typename T>
hipError_t launch_xi_gather(const XiView<T>& xv, int q, const XiItem* items, int nitems, const void* vin,
                            double* hacc, int64_t N, int conj_out, void* h, hipStream_t st)
{
    LaunchStatus ls;
    const unsigned nz = (unsigned)((2 * N + XI_THREADS - 1) / XI_THREADS);
    hipLaunchKernelGGL(k_xi_zero, dim3(nz), dim3(XI_THREADS), 0, st, hacc, 2 * N);
    ls.launched();
    if (nitems > 0) {
        if (q <= 16)
            hipLaunchKernelGGL((k_xi_gather<T, 16>), dim3(nitems), dim3(XI_THREADS), 0, st, xv, items,
                               (const cplx<T>*)vin, hacc);
        else if (q <= 24)
            hipLaunchKernelGGL((k_xi_gather<T, 24>), dim3(nitems), dim3(XI_THREADS), 0, st, xv, items,
                               (const cplx<T>*)vin, hacc);
        else
            hipLaunchKernelGGL((k_xi_gather<T, 32>), dim3(nitems), dim3(XI_THREADS), 0, st, xv, items,
                               (const cplx<T>*)vin, hacc);
        ls.launched();
    }
    const unsigned nf = (unsigned)((N + XI_THREADS - 1) / XI_THREADS);
    hipLaunchKernelGGL(k_xi_finalize<T>, dim3(nf), dim3(XI_THREADS), 0, st, xv, N, (const double*)hacc, conj_out,
                       (cplx<T>*)h);
    ls.launched();
    return ls.first;
}

#define FLT_XI_INST(T)                                                                                          \
    template hipError_t launch_xi_spread<T>(const XiView<T>&, int, const XiItem*, int, const void*, void*,      \
                                            hipStream_t);                                                       \
    template hipError_t launch_xi_combine<T>(const XiView<T>&, const NodeItem*, int, const void*, void*,        \
                                             hipStream_t);                                                      \
    template hipError_t launch_xi_prep<T>(const XiView<T>&, const NodeItem*, int, const void*, int, void*,      \
                                          hipStream_t);                                                         \
    template hipError_t launch_xi_gather<T>(const XiView<T>&, int, const XiItem*, int, const void*, double*,    \
                                            int64_t, int, void*, hipStream_t);
FLT_XI_INST(float)
FLT_XI_INST(double)
#undef FLT_XI_INST

}  // namespace flt
