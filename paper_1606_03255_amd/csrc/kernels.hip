// gfx950 kernels of the fast Fourier-Laplace transform and their launch
// sequences.  The bodies live in kernels_impl.h; this file binds them to the
// HIP execution model (one workgroup per item of a precomputed work list,
// 64 KB LDS tiles for the FFT kernels) and orders them on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "flt.h"

#include "kernels_impl.h"
#include "launch.h"

namespace flt {

struct DevCtx {
    __device__ __forceinline__ int tid() const { return (int)threadIdx.x; }
    __device__ __forceinline__ int ntid() const { return (int)blockDim.x; }
    __device__ __forceinline__ int bid() const { return (int)blockIdx.x; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
    __device__ __forceinline__ void atomic_add(double* p, double v) const { unsafeAtomicAdd(p, v); }
    __device__ __forceinline__ void atomic_add(float* p, float v) const { unsafeAtomicAdd(p, v); }
};

// Static LDS of the kernels, against gfx950's 160 KB per workgroup (the
// compiler rejects more) and the 80 KB that lets two 512-thread workgroups
// share a compute unit, which the FFT kernels other than the FP32 pass A are
// laid out for (that one runs a workgroup per CU with two tiles).
constexpr size_t LDS_LIMIT = 160 * 1024, LDS_TWO_PER_CU = 80 * 1024;
template <typename T> constexpr size_t lds_fft_bytes() { return sizeof(cplx<T>) * tile_alloc<T>(); }
template <typename T> constexpr int passA_omega_alloc() { return sizeof(T) == 4 ? PASSA_OMEGA_MAX : 0; }
constexpr size_t lds_passA_f32_bytes()
{
    return 2 * lds_fft_bytes<float>() + 2 * sizeof(float) * Sizes<float>::COEF +
           sizeof(cplx<float>) * passA_omega_alloc<float>();
}
constexpr size_t lds_passA_f64_bytes() { return lds_fft_bytes<double>() + sizeof(double) * Sizes<double>::COEF; }
static_assert(lds_passA_f32_bytes() <= LDS_LIMIT, "LDS per workgroup");
static_assert(lds_passA_f64_bytes() <= LDS_TWO_PER_CU, "two FP64 pass-A workgroups per CU");
static_assert(lds_fft_bytes<float>() + sizeof(float) * Sizes<float>::COEF <= LDS_TWO_PER_CU &&
                  lds_fft_bytes<double>() + sizeof(double) * Sizes<double>::COEF <= LDS_TWO_PER_CU,
              "a tile and a coefficient buffer leave room for a second workgroup per CU");
static_assert(lds_fft_bytes<float>() + sizeof(float) * onepass_coef<float>() <= LDS_TWO_PER_CU &&
                  lds_fft_bytes<double>() + sizeof(double) * onepass_coef<double>() <= LDS_TWO_PER_CU &&
                  onepass_coef<double>() >= 2 * MAX_Q * 16,
              "one-pass FFT: tile and staged coefficients, two workgroups per CU");
static_assert(lds_fft_bytes<float>() + sizeof(cplx<float>) * lds_tw_half<Log2Range<float>::B_HI>() <= LDS_TWO_PER_CU,
              "persistent pass B: tile and twiddle half table, two workgroups per CU");

// One launch per FFT kind; each workgroup picks the compile-time instance of
// its band's transform length.
template <typename T>
__global__ __launch_bounds__(FFT_THREADS, 2) void k_onepass_fwd(PlanView<T> pv, const FftItem* items,
                                                                const cplx<T>* c, cplx<T>* grids, int deriv,
                                                                int cols)
{
    __shared__ cplx<T> lds[tile_alloc<T>()];
    __shared__ alignas(16) T lc[onepass_coef<T>()];
    using RG = Log2Range<T>;
    with_log2<RG::ONE_LO, RG::ONE_HI>(pv.bands[items[blockIdx.x].band].log2n, [&](auto LG) {
        body_onepass_fwd<DevCtx, T, decltype(LG)::value>(DevCtx(), pv, items, c, grids, deriv, cols, lds, lc);
    });
}

// FP32: two waves per SIMD (one workgroup per CU): the bases, the first-stage
// butterfly and the stage twiddles of a thread stay in registers (measured
// faster than four waves per SIMD with spills).
__global__ __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_passA_fwd_f32(
    PlanView<float> pv, const FftItem* items, const cplx<float>* c, cplx<float>* scratch, int deriv, int cols)
{
    __shared__ cplx<float> lds[2 * tile_alloc<float>()];
    __shared__ alignas(16) float lc[2 * Sizes<float>::COEF];
    __shared__ cplx<float> omega[passA_omega_alloc<float>()];
    using RG = Log2Range<float>;
    with_log2<RG::TWO_LO, RG::TWO_HI>(pv.bands[items[blockIdx.x].band].log2n, [&](auto LG) {
        body_passA_fwd<DevCtx, float, decltype(LG)::value>(DevCtx(), pv, items, c, scratch, deriv, cols, lds, lc,
                                                           omega);
    });
}

// FP64: four waves per SIMD (two workgroups per CU, as the LDS allows); the
// bases in the workspace slots
__global__ __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_passA_fwd_f64(
    PlanView<double> pv, const FftItem* items, const cplx<double>* c, cplx<double>* scratch, cplx<double>* basebuf,
    int deriv, int cols)
{
    __shared__ cplx<double> lds[tile_alloc<double>()];
    __shared__ alignas(16) double lc[Sizes<double>::COEF];
    using RG = Log2Range<double>;
    with_log2<RG::TWO_LO, RG::TWO_HI>(pv.bands[items[blockIdx.x].band].log2n, [&](auto LG) {
        body_passA_fwd_slot<DevCtx, double, decltype(LG)::value>(DevCtx(), pv, items, c, scratch, basebuf, deriv,
                                                                 cols, lds, lc);
    });
}

template <typename T, int SIGN>
// four waves per SIMD (two workgroups per CU, as the LDS allows): the
// register budget the prefetched tile has to fit in
__global__ __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_passB(PlanView<T> pv, const FftItem* items, int nitems,
                                                          const cplx<T>* src, cplx<T>* dst, int cols)
{
    __shared__ cplx<T> lds[tile_alloc<T>()];
    // the prefetching variant's twiddle half table (the longest pass-B transform)
    __shared__ cplx<T> twl[passB_prefetch<T, SIGN>() ? lds_tw_half<Log2Range<T>::B_HI>() : 1];
    body_passB<DevCtx, T, SIGN>(DevCtx(), pv, items, nitems, (int)gridDim.x, src, dst, cols, lds, twl);
}

template <typename T, int MW>
__global__ __launch_bounds__(GATHER_THREADS) void k_gather_staged(PlanView<T> pv, const NodeItem* items,
                                                                  const cplx<T>* c, const cplx<T>* grids,
                                                                  cplx<T>* f, int with_c0, cplx<T>* f2)
{
    __shared__ cplx<T> stage[GATHER_STAGE];
    body_gather<DevCtx, T, MW, true>(DevCtx(), pv, items, c, grids, f, with_c0, f2, stage);
}

template <typename T, int MW>
__global__ __launch_bounds__(GATHER_THREADS) void k_gather_lane(PlanView<T> pv, const NodeItem* items,
                                                                const cplx<T>* c, const cplx<T>* grids, cplx<T>* f,
                                                                int with_c0, cplx<T>* f2)
{
    body_gather<DevCtx, T, MW, false>(DevCtx(), pv, items, c, grids, f, with_c0, f2, nullptr);
}

template <typename T, int MW>
__global__ __launch_bounds__(GATHER_THREADS) void k_adj_prep(PlanView<T> pv, const NodeItem* items,
                                                             const cplx<T>* g, int qs, cplx<T>* U, T* Phi,
                                                             int32_t* L0)
{
    body_adj_prep<DevCtx, T, MW>(DevCtx(), pv, items, g, qs, U, Phi, L0);
}

template <typename T, int MW>
__global__ __launch_bounds__(GATHER_THREADS) void k_adj_cells(PlanView<T> pv, const CellItem* items, int qs,
                                                              const cplx<T>* U, const T* Phi, const int32_t* L0,
                                                              const int32_t* cstart, const int32_t* clist,
                                                              cplx<T>* grids)
{
    __shared__ T red[2 * ADJ_RC * GATHER_THREADS];
    body_adj_cells<DevCtx, T, MW>(DevCtx(), pv, items, qs, U, Phi, L0, cstart, clist, grids, red);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sum_g(PlanView<T> pv, const SumItem* items, const cplx<T>* g, double* acc)
{
    __shared__ double red[2 * 256];
    body_sum_g<DevCtx, T>(DevCtx(), pv, items, g, acc, red);
}

template <typename T>
__global__ __launch_bounds__(FFT_THREADS, 2) void k_onepass_adj(PlanView<T> pv, const FftItem* items,
                                                                const cplx<T>* grids, double* acc)
{
    __shared__ cplx<T> lds[tile_alloc<T>()];
    using RG = Log2Range<T>;
    with_log2<RG::ONE_LO, RG::ONE_HI>(pv.bands[items[blockIdx.x].band].log2n, [&](auto LG) {
        body_onepass_adj<DevCtx, T, decltype(LG)::value>(DevCtx(), pv, items, grids, acc, lds);
    });
}

// FP32: the adjoint pass A with a workgroup per CU (two waves per SIMD, two
// LDS tiles); FP64: the one-tile variant, compiler's register choice.
__global__ __launch_bounds__(FFT_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_passA_adj_f32(
    PlanView<float> pv, const FftItem* items, const cplx<float>* scratch, double* acc)
{
    __shared__ cplx<float> lds[2 * tile_alloc<float>()];
    __shared__ alignas(16) float lc[2 * Sizes<float>::COEF];
    __shared__ cplx<float> omega[passA_omega_alloc<float>()];
    using RG = Log2Range<float>;
    with_log2<RG::TWO_LO, RG::TWO_HI>(pv.bands[items[blockIdx.x].band].log2n, [&](auto LG) {
        body_passA_adj<DevCtx, float, decltype(LG)::value>(DevCtx(), pv, items, scratch, acc, lds, lc, omega);
    });
}

__global__ __launch_bounds__(FFT_THREADS, 2) void k_passA_adj_f64(PlanView<double> pv, const FftItem* items,
                                                                  const cplx<double>* scratch, double* acc)
{
    __shared__ cplx<double> lds[tile_alloc<double>()];
    __shared__ alignas(16) double lc[Sizes<double>::COEF];
    using RG = Log2Range<double>;
    with_log2<RG::TWO_LO, RG::TWO_HI>(pv.bands[items[blockIdx.x].band].log2n, [&](auto LG) {
        body_passA_adj_1tile<DevCtx, double, decltype(LG)::value>(DevCtx(), pv, items, scratch, acc, lds, lc);
    });
}

template <typename T, bool DERIV, bool GROUPED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_direct_fwd(PlanView<T> pv, const DirectItem* items, const int32_t* dlist,
                                                    const cplx<T>* c, double* dacc)
{
    __shared__ double red[2 * DIRECT_NG * 256];
    static_assert(256 / 8 == DIRECT_GMAX, "groups of at least 8 threads fill DIRECT_GMAX groups");
    __shared__ cplx<T> nw[DIRECT_NG * DIRECT_GMAX];
    body_direct_fwd<DevCtx, T, DERIV, GROUPED>(DevCtx(), pv, items, dlist, c, dacc, red, nw);
}

template <typename T>
__global__ __launch_bounds__(256) void k_direct_io(PlanView<T> pv, const int32_t* dlist, int64_t nd, double* dacc,
                                                   cplx<T>* f, int op)
{
    body_direct_io<DevCtx, T>(DevCtx(), pv, dlist, nd, dacc, f, op);
}

template <typename T>
__global__ __launch_bounds__(256) void k_direct_adj(PlanView<T> pv, const DirectItem* items, const int32_t* dlist,
                                                    const cplx<T>* g, double* acc)
{
    __shared__ cplx<T> nw[DIRECT_ANG], ng[DIRECT_ANG], red[256 * ADJ_TS];
    body_direct_adj<DevCtx, T>(DevCtx(), pv, items, dlist, g, acc, nw, ng, red);
}

// Clear `n` 16-byte words (a fill kernel, so the sequence stays capturable).
__global__ __launch_bounds__(256) void k_zero16(double2* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_finalize_adj(const double* acc, cplx<T>* out, int64_t N)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = mk<T>((T)acc[2 * k], (T)acc[2 * k + 1]);
}

static int grid_for(int64_t work, int per_block)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

// A HIP event on the stream between stages (measurement calls only).
static void mark(LaunchStatus& ls, hipEvent_t* ev, int i, hipStream_t st)
{
    if (ev) ls.note(hipEventRecord(ev[i], st));
}

template <typename T>
static void fft_forward_stages(LaunchStatus& ls, const DevLists& L, const PlanView<T>& pv, const WsLayout& W,
                               const cplx<T>* c, int deriv, int cols, hipStream_t st, hipEvent_t* ev)
{
    cplx<T>* grids = (cplx<T>*)(W.ws + W.off_grid);
    cplx<T>* scratch = (cplx<T>*)(W.ws + W.off_scratch);
    // cols = 2: the item lists over 2q columns per band
    const FftItem* one = cols == 2 ? L.onepass_fused : L.onepass_fwd;
    const int n_one = cols == 2 ? L.n_onepass_fused : L.n_onepass_fwd;
    const FftItem* pb = cols == 2 ? L.passB_fused : L.passB;
    const int n_pb = cols == 2 ? L.n_passB_fused : L.n_passB;
    if (n_one) {
        hipLaunchKernelGGL(k_onepass_fwd<T>, dim3(n_one), dim3(FFT_THREADS), 0, st, pv, one, c, grids, deriv, cols);
        ls.launched();
    }
    mark(ls, ev, 1, st);
    if (L.n_passA_fwd) {
        if constexpr (std::is_same<T, float>::value)
            hipLaunchKernelGGL(k_passA_fwd_f32, dim3(L.n_passA_fwd), dim3(FFT_THREADS), 0, st, pv, L.passA_fwd, c,
                               scratch, deriv, cols);
        else
            hipLaunchKernelGGL(k_passA_fwd_f64, dim3(L.n_passA_fwd), dim3(FFT_THREADS), 0, st, pv, L.passA_fwd, c,
                               scratch, (cplx<T>*)(W.ws + W.off_base), deriv, cols);
        ls.launched();
    }
    mark(ls, ev, 2, st);
    if (n_pb) {
        hipLaunchKernelGGL((k_passB<T, +1>),
                           dim3(passB_prefetch<T, +1>() ? std::min(n_pb, L.persist_blocks) : n_pb),
                           dim3(FFT_THREADS), 0, st, pv, pb, n_pb, (const cplx<T>*)scratch, grids, cols);
        ls.launched();
    }
    mark(ls, ev, 3, st);
}

template <typename T>
static void fft_adjoint_stages(LaunchStatus& ls, const DevLists& L, const PlanView<T>& pv, cplx<T>* grids,
                               cplx<T>* scratch, double* acc, hipStream_t st, hipEvent_t* ev)
{
    if (L.n_passB) {
        hipLaunchKernelGGL((k_passB<T, -1>),
                           dim3(passB_prefetch<T, -1>() ? std::min(L.n_passB, L.persist_blocks) : L.n_passB),
                           dim3(FFT_THREADS), 0, st,
                           pv, L.passB, L.n_passB, (const cplx<T>*)grids, scratch, 1);
        ls.launched();
    }
    mark(ls, ev, 4, st);
    if (L.n_passA_adj) {
        if constexpr (std::is_same<T, float>::value)
            hipLaunchKernelGGL(k_passA_adj_f32, dim3(L.n_passA_adj), dim3(FFT_THREADS), 0, st, pv, L.passA_adj,
                               (const cplx<T>*)scratch, acc);
        else
            hipLaunchKernelGGL(k_passA_adj_f64, dim3(L.n_passA_adj), dim3(FFT_THREADS), 0, st, pv, L.passA_adj,
                               (const cplx<T>*)scratch, acc);
        ls.launched();
    }
    mark(ls, ev, 5, st);
    if (L.n_onepass_adj) {
        hipLaunchKernelGGL(k_onepass_adj<T>, dim3(L.n_onepass_adj), dim3(FFT_THREADS), 0, st, pv, L.onepass_adj,
                           (const cplx<T>*)grids, acc);
        ls.launched();
    }
    mark(ls, ev, 6, st);
}

template <typename T, int MW>
static void mw_forward_nodes(LaunchStatus& ls, const DevLists& L, const PlanView<T>& pv, const cplx<T>* c,
                             const cplx<T>* grids, cplx<T>* f, int with_c0, cplx<T>* f2, hipStream_t st)
{
    if (L.n_gather_st) {
        hipLaunchKernelGGL((k_gather_staged<T, MW>), dim3(L.n_gather_st), dim3(GATHER_THREADS), 0, st, pv,
                           L.gather_st, c, grids, f, with_c0, f2);
        ls.launched();
    }
    if (L.n_gather_ln) {
        hipLaunchKernelGGL((k_gather_lane<T, MW>), dim3(L.n_gather_ln), dim3(GATHER_THREADS), 0, st, pv,
                           L.gather_ln, c, grids, f, with_c0, f2);
        ls.launched();
    }
}

template <typename T, int MW>
static void mw_adjoint_nodes(LaunchStatus& ls, const DevLists& L, const PlanView<T>& pv, const WsLayout& W,
                             const cplx<T>* g, cplx<T>* grids, hipStream_t st, hipEvent_t* ev)
{
    cplx<T>* U = (cplx<T>*)(W.ws + W.off_U);
    T* Phi = (T*)(W.ws + W.off_phi);
    int32_t* L0 = (int32_t*)(W.ws + W.off_l0);
    if (L.n_nfft_nodes) {
        hipLaunchKernelGGL((k_adj_prep<T, MW>), dim3(L.n_nfft_nodes), dim3(GATHER_THREADS), 0, st, pv,
                           L.nfft_nodes, g, W.qs, U, Phi, L0);
        ls.launched();
    }
    mark(ls, ev, 2, st);
    if (L.n_cells) {
        hipLaunchKernelGGL((k_adj_cells<T, MW>), dim3(L.n_cells), dim3(GATHER_THREADS), 0, st, pv, L.cells, W.qs,
                           (const cplx<T>*)U, (const T*)Phi, (const int32_t*)L0, L.cstart, L.clist, grids);
        ls.launched();
    }
    mark(ls, ev, 3, st);
}

template <typename T>
hipError_t launch_forward(const DevLists& L, const PlanView<T>& pv, const WsLayout& W, const void* cv, void* fv,
                          void* f2v, int deriv, hipStream_t st, hipEvent_t* ev)
{
    LaunchStatus ls;
    const cplx<T>* c = (const cplx<T>*)cv;
    cplx<T>* f = (cplx<T>*)fv;
    cplx<T>* f2 = (cplx<T>*)f2v;   // non-null: the derivative too, in the same pass (2q columns per band)
    const int cols = f2 ? 2 : 1;
    if (f2) deriv = 0;
    if (pv.mw < 2 || pv.mw > MAX_MW) return hipErrorInvalidValue;
    cplx<T>* grids = (cplx<T>*)(W.ws + W.off_grid);
    double* dacc = (double*)(W.ws + W.off_dacc);
    mark(ls, ev, 0, st);
    fft_forward_stages<T>(ls, L, pv, W, c, deriv, cols, st, ev);
    if (L.n_gather_st + L.n_gather_ln) {
        switch (pv.mw) {
#define G(MWV) case MWV: mw_forward_nodes<T, MWV>(ls, L, pv, c, grids, f, !deriv, f2, st); break;
            G(2) G(3) G(4) G(5) G(6) G(7) G(8) G(9) G(10)
#undef G
        }
    }
    mark(ls, ev, 4, st);
    if (L.n_dlist) {
        const int gb = (int)((L.n_dlist + 255) / 256);
        for (int d = 0; d < cols; ++d) {   // direct bands: exact sums, of c and (cols = 2) of c'
            cplx<T>* out = d ? f2 : f;
            hipLaunchKernelGGL(k_direct_io<T>, dim3(gb), dim3(256), 0, st, pv, L.dlist, L.n_dlist, dacc, out, 0);
            ls.launched();
            // long sums, then short ones (thread groups), both adding into dacc
            if (L.n_direct_fwd) {
                if (deriv || d)
                    hipLaunchKernelGGL((k_direct_fwd<T, true, false>), dim3(L.n_direct_fwd), dim3(256), 0, st, pv,
                                       L.direct_fwd, L.dlist, c, dacc);
                else
                    hipLaunchKernelGGL((k_direct_fwd<T, false, false>), dim3(L.n_direct_fwd), dim3(256), 0, st, pv,
                                       L.direct_fwd, L.dlist, c, dacc);
                ls.launched();
            }
            if (L.n_direct_short) {
                if (deriv || d)
                    hipLaunchKernelGGL((k_direct_fwd<T, true, true>), dim3(L.n_direct_short), dim3(256), 0, st, pv,
                                       L.direct_short, L.dlist, c, dacc);
                else
                    hipLaunchKernelGGL((k_direct_fwd<T, false, true>), dim3(L.n_direct_short), dim3(256), 0, st, pv,
                                       L.direct_short, L.dlist, c, dacc);
                ls.launched();
            }
            hipLaunchKernelGGL(k_direct_io<T>, dim3(gb), dim3(256), 0, st, pv, L.dlist, L.n_dlist, dacc, out, 1);
            ls.launched();
        }
    }
    mark(ls, ev, 5, st);
    return ls.first;
}

template <typename T>
hipError_t launch_adjoint(const DevLists& L, const PlanView<T>& pv, const WsLayout& W, const void* gv, void* outv,
                          hipStream_t st, hipEvent_t* ev)
{
    LaunchStatus ls;
    const cplx<T>* g = (const cplx<T>*)gv;
    cplx<T>* out = (cplx<T>*)outv;
    cplx<T>* grids = (cplx<T>*)(W.ws + W.off_grid);
    cplx<T>* scratch = (cplx<T>*)(W.ws + W.off_scratch);
    double* acc = (double*)(W.ws + W.off_acc);
    if (pv.mw < 2 || pv.mw > MAX_MW) return hipErrorInvalidValue;
    mark(ls, ev, 0, st);
    hipLaunchKernelGGL(k_zero16, dim3(grid_for(W.N, 256 * 8)), dim3(256), 0, st, (double2*)acc, W.N);
    ls.launched();
    hipLaunchKernelGGL(k_sum_g<T>, dim3(L.n_sum), dim3(256), 0, st, pv, L.sum_items, g, acc);
    ls.launched();
    mark(ls, ev, 1, st);
    switch (pv.mw) {
#define S(MWV) case MWV: mw_adjoint_nodes<T, MWV>(ls, L, pv, W, g, grids, st, ev); break;
        S(2) S(3) S(4) S(5) S(6) S(7) S(8) S(9) S(10)
#undef S
    }
    fft_adjoint_stages<T>(ls, L, pv, grids, scratch, acc, st, ev);
    if (L.n_direct_adj) {
        hipLaunchKernelGGL(k_direct_adj<T>, dim3(L.n_direct_adj), dim3(256), 0, st, pv, L.direct_adj, L.dlist, g,
                           acc);
        ls.launched();
    }
    mark(ls, ev, 7, st);
    hipLaunchKernelGGL(k_finalize_adj<T>, dim3(grid_for(W.N, 256 * 4)), dim3(256), 0, st, acc, out, W.N);
    ls.launched();
    mark(ls, ev, 8, st);
    return ls.first;
}

// The scratch of the forward without a workspace (flt_forward_noalloc): one
// static array, of which every device the library runs that call on holds
// its own copy at its own address while the library is loaded.  In host code
// this name is only a handle for the address lookup below, never a device
// address: kernels and copies are given the looked-up address.
static __device__ __align__(256) char noalloc_scratch[FLT_NOALLOC_MAX_BYTES];

namespace {
std::mutex g_noalloc_mu;
std::map<int, char*> g_noalloc_at;   // device -> address of its noalloc_scratch
}  // namespace

hipError_t noalloc_scratch_address(int device, char** out)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    const auto it = g_noalloc_at.find(device);
    if (it != g_noalloc_at.end()) {
        *out = it->second;
        return hipSuccess;
    }
    // the lookup with that device current, the caller's device restored after
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
    if (cur != device) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_noalloc_at[device] = (char*)ptr;
    *out = (char*)ptr;
    return hipSuccess;
}

template hipError_t launch_forward<float>(const DevLists&, const PlanView<float>&, const WsLayout&, const void*,
                                          void*, void*, int, hipStream_t, hipEvent_t*);
template hipError_t launch_forward<double>(const DevLists&, const PlanView<double>&, const WsLayout&, const void*,
                                           void*, void*, int, hipStream_t, hipEvent_t*);
template hipError_t launch_adjoint<float>(const DevLists&, const PlanView<float>&, const WsLayout&, const void*,
                                          void*, hipStream_t, hipEvent_t*);
template hipError_t launch_adjoint<double>(const DevLists&, const PlanView<double>&, const WsLayout&, const void*,
                                           void*, hipStream_t, hipEvent_t*);

}  // namespace flt
