/*
 * flt.h -- fast Fourier-Laplace transform on AMD MI355X (gfx950).
 *
 * Evaluates the exponential sums of Kunis & Melzer, "Fast evaluation of real
 * and complex exponential sums", Sect. 4, eq. 4.1 with integer exponents:
 *
 *     f(z_j) = sum_{k=0}^{N-1} c_k e^{2 pi i k z_j},   Im z_j >= 0,   j < M,
 *
 * i.e. a polynomial with monomial coefficients c_k at w_j = e^{2 pi i z_j} in
 * the closed unit disk, by the paper's Algorithm 2: dyadic bands of
 * y = 2 pi Im z (Def. 3.2), rank-q Chebyshev interpolation of every admissible
 * Laplace block (Lemma A.1/A.2), the Hadamard-product identity of Lemma 4.2,
 * and one oversampled Kaiser-Bessel NFFT per band column as the Fourier black
 * box.  The result satisfies max_j |f~_j - f_j| <= eps * sum_k |c_k|
 * (Thm 4.3).  All work after plan creation runs in HIP kernels on the GPU.
 *
 * Conventions for every entry point
 *   - Complex arrays are interleaved (re, im): complex64 = 2 x float,
 *     complex128 = 2 x double, contiguous, element stride 1.
 *   - "device" pointers are HIP device (or managed) memory of the device that
 *     was current when the plan was created; "host" pointers are ordinary host
 *     memory.  The caller owns every pointer it passes; the library never
 *     frees caller memory and keeps no pointer to caller memory after a call
 *     returns, except the workspace registered with flt_plan_set_workspace.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Transform
 *     calls only enqueue work on it and return; results are ready when the
 *     stream reaches that point.  Inputs are read-only.
 *   - Every call returns FLT_OK (0) or a negative FLT_E* code; no exception
 *     crosses the boundary and nothing aborts.  Argument checks happen before
 *     any device work, so a failed call enqueues nothing.
 *   - A plan is immutable after creation apart from its workspace binding and
 *     may be used from one stream at a time.
 */
#ifndef FLT_H
#define FLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct flt_plan flt_plan;

/* dtype: the arithmetic form of a plan */
#define FLT_C64  1 /* c, f complex64; FP32 bulk arithmetic, FP64 phase reduction and final per-node sums */
#define FLT_C128 2 /* c, f complex128; FP64 throughout */

/* flags for flt_plan_create */
#define FLT_FLAG_HOST_ONLY (1u << 0) /* plan on the host only (parameters, partition, byte model); no device */
#define FLT_FLAG_NFFT_ONLY (1u << 1) /* every band by Alg. 2's NFFT path; by default a band whose grids would
                                        cost more than summing its few nodes directly is summed exactly */
#define FLT_FLAG_GRAPH     (1u << 2) /* capture each operation's launch sequence into a hipGraph on its first call
                                        (and again whenever the buffers or the workspace change) and replay it */
#define FLT_FLAG_AUTOTUNE  (1u << 3) /* choose the plan's shape by timing forward + adjoint of candidates on the
                                        device during creation, one dimension after the other: the band policy
                                        (direct-sum rate scaled by 0, 1/2, 1, 2, 4, 8; distinct band choices
                                        only), then workgroups per CU of the persistent pass B (2, 1, 3, 4).
                                        All candidates are timed twice (the first pass a warm-up); in that
                                        order each replaces the choice only when at least 2% faster.  The
                                        choice is cached per (objective, dtype, eps, instances, size class) for
                                        the process.  Ignored with FLT_FLAG_NFFT_ONLY or FLT_FLAG_HOST_ONLY */
#define FLT_FLAG_TUNE_FORWARD (1u << 4) /* with FLT_FLAG_AUTOTUNE: time the forward alone (plans used for
                                        evaluation only); without it forward + adjoint (training steps) */

/* return codes */
#define FLT_OK            0
#define FLT_EINVAL       -1 /* null pointer, N < 1, M < 1, unknown dtype/flags, band index out of range */
#define FLT_EDOMAIN      -2 /* eps outside (0,1); Im z < 0 (|w| > 1) or NaN/inf in Re z, NaN in Im z */
#define FLT_EPRECISION   -3 /* eps below what the dtype can deliver (c64: 1e-6, c128: 1e-14) */
#define FLT_ENOWORKSPACE -4 /* no workspace registered, or the one given is too small */
#define FLT_EHIP         -5 /* a HIP runtime call failed; see flt_last_hip_error() */
#define FLT_ESTATE       -6 /* plan created with FLT_FLAG_HOST_ONLY used for device work */
#define FLT_ENOMEM       -7 /* host allocation failed */
#define FLT_ERANGE       -8 /* N beyond the largest supported size (2^21 + 1 coefficients) */

/* Plan-wide figures (Def. 3.2, Alg. 2, Lemma 4.1). */
typedef struct flt_info {
    int64_t N, M;            /* coefficients, nodes */
    int32_t dtype;           /* FLT_C64 or FLT_C128 */
    int32_t q;               /* Chebyshev rank, ceil(1/2 + log4(1/eps_K)) */
    int32_t D;               /* dyadic levels (the paper's M), ceil(log2(y1 xi1 / eps_K)) + 1 */
    int32_t n_xi;            /* xi_1 = 2^n_xi >= N - 1 */
    int32_t mw;              /* Kaiser-Bessel window half-width (2 mw taps) */
    int32_t num_bands;       /* occupied bands, Y_D included, Z^0 excluded */
    double eps, eps_K, eps_A;/* target accuracy and its Laplace / Fourier shares */
    double y1;               /* ln(1/eps_K): nodes with y = 2 pi Im z > y1 form Z^0 */
    int64_t nodes_z0;        /* nodes in Z^0 (f = c_0 there) */
    size_t workspace_bytes;  /* device workspace every transform call needs (the fused one included) */
    double bytes_forward;    /* algorithmic HBM bytes of one forward call */
    double flops_forward;    /* algorithmic flops of one forward call */
    double direct_scale;     /* factor on the direct-sum rate the band policy used (1, or the tuned choice) */
    size_t forward_scratch_bytes; /* device scratch of one forward call alone (see flt_forward_noalloc) */
    int32_t passB_blocks;    /* workgroups of the persistent pass B (0 for a host-only plan) */
    int32_t pad;
} flt_info;

/* One occupied band (Def. 3.2 Y_m, or Y_D). */
typedef struct flt_band_info {
    int32_t m;               /* 1..D-1 for Y_m, D for Y_D */
    int32_t q;               /* columns: the rank q, or 1 for Y_D */
    int32_t ell_lo, ell_hi;  /* interpolated frequency blocks Omega_l, l_m <= l <= L_m (none for Y_D) */
    int64_t K;               /* support: frequencies 1..min(K, N-1) */
    int64_t n;               /* NFFT grid length (2K, at least 16) */
    int64_t k0;              /* centre of the support, floor(K/2) */
    int64_t nodes;           /* nodes in the band */
    int32_t passes;          /* FFT passes through HBM (1 or 2); 0 for a direct band */
    int32_t direct;          /* 1: the band's nodes are summed directly (exact), not by NFFT */
    int64_t cells;           /* grid cells per column that some node's window reads (0 for a direct band) */
} flt_band_info;

/* Build a plan for N coefficients and M nodes z (host, 2*M doubles,
 * complex128 layout; copied, the caller keeps ownership).  Host work in FP64:
 * parameters, node classification and sorting, interpolation and window
 * tables; then an upload to the current device (unless FLT_FLAG_HOST_ONLY).
 * Im z = +inf is accepted (w = 0, f = c_0).  *out receives the plan or NULL. */
int flt_plan_create(flt_plan** out, int64_t N, int64_t M, const double* z,
                    double eps, int dtype, uint32_t flags);

/* As flt_plan_create, with the band policy's factor on the direct-sum rate
 * given.  The band policy decides which bands of the partition (Def. 3.2) are
 * summed directly and exactly instead of by Alg. 2's NFFT (few nodes, large
 * grids; FLT_FLAG_NFFT_ONLY turns it off): its default factor is 1, and
 * FLT_FLAG_AUTOTUNE chooses among 0, 1/2, 1, 2, 4, 8 and reports the choice in
 * flt_info.direct_scale.  This call rebuilds a tuned plan's shape without
 * timing, e.g. in another process.  The result meets the same bar (Thm 4.3;
 * direct bands are exact); only which bands are summed directly changes.
 * direct_scale must be finite and >= 0, and flags may not hold
 * FLT_FLAG_AUTOTUNE (FLT_EINVAL otherwise). */
int flt_plan_create_policy(flt_plan** out, int64_t N, int64_t M, const double* z,
                           double eps, int dtype, uint32_t flags, double direct_scale);

/* One plan for `count` independent instances of Alg. 2 at one eps and dtype
 * (instance i: N[i] coefficients, M[i] nodes; N, M host arrays of count
 * entries).  z (host) holds the nodes instance after instance, sum M[i]
 * complex128 values.  The plan's transforms act on packed arrays: c (and the
 * adjoint's output) holds instance i's coefficients from sum_{i'<i} N[i'],
 * f (and the adjoint's input) its nodes from sum_{i'<i} M[i'].  Every
 * instance gets exactly what its own flt_plan_create plan would compute, with
 * each transform kind of all instances in a single launch.  Errors as for
 * flt_plan_create (the first failing instance decides); count < 1 or a null
 * array is FLT_EINVAL. */
int flt_plan_create_batch(flt_plan** out, int32_t count, const int64_t* N, const int64_t* M,
                          const double* z, double eps, int dtype, uint32_t flags);

/* Release the plan's device and host memory; NULL is a no-op.  The caller
 * must ensure no enqueued work of the plan is still pending. */
void flt_plan_destroy(flt_plan* plan);

/* Host queries (valid for every plan). */
int flt_plan_info(const flt_plan* plan, flt_info* out);
int flt_plan_band(const flt_plan* plan, int32_t i, flt_band_info* out);   /* 0 <= i < num_bands */
/* out (host, M int32): band of each node in caller order: 0 = Z^0, m = Y_m, D = Y_D */
int flt_plan_node_bands(const flt_plan* plan, int32_t* out);

/* Device workspace: the caller allocates at least flt_plan_workspace_size()
 * bytes of device memory (256-byte aligned) and registers it; it must stay
 * valid while transforms that use it are pending.  The plan does not own it. */
int flt_plan_workspace_size(const flt_plan* plan, size_t* bytes);
int flt_plan_set_workspace(flt_plan* plan, void* dev, size_t bytes);

/* Forward (Alg. 2): f[j] ~ sum_{k<N} c_k w_j^k.
 * c: device complex[N] of the plan's dtype; f: device complex[M], overwritten.
 * Error <= eps * sum|c_k| (Thm 4.3). */
int flt_forward(flt_plan* plan, const void* c, void* f, void* stream);

/* The most device scratch flt_forward_noalloc can use (128 MiB). */
#define FLT_NOALLOC_MAX_BYTES ((size_t)128 << 20)

/* Forward without a workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels and result as flt_forward, with their
 * scratch (band grids, pass-A output, direct-sum accumulator, base slots) in
 * one static device array of FLT_NOALLOC_MAX_BYTES that the library holds on
 * each device it runs this call on, until the process ends.  The call
 * allocates nothing and needs no registered workspace; its address is looked
 * up once per device on the first call there.
 * c: device complex[N], f: device complex[M] of the plan's dtype, as for
 * flt_forward.  Errors: as flt_forward (no FLT_ENOWORKSPACE); FLT_ERANGE if
 * the plan's forward needs more than FLT_NOALLOC_MAX_BYTES of scratch (its
 * flt_info.forward_scratch_bytes), checked before any device work.  Every
 * call on one device shares that device's array: calls that overlap in time
 * on one device (two streams, two threads, or this and another plan) race
 * and give wrong results; calls one after another on a stream are fine (the
 * forward writes every scratch value it reads before reading it). */
int flt_forward_noalloc(flt_plan* plan, const void* c, void* f, void* stream);

/* Derivative: fp[j] ~ f'(z_j) = sum_{k<N} 2 pi i k c_k w_j^k, i.e. Alg. 2
 * applied to c'_k = 2 pi i k c_k; error <= eps * sum_k |2 pi k c_k|. */
int flt_derivative(flt_plan* plan, const void* c, void* fp, void* stream);

/* Forward and derivative in one pass: f as flt_forward, fp as flt_derivative,
 * with the derivative's q columns per band transformed alongside the
 * forward's (2q columns; the interpolant rows, cell positions, window weights
 * and node-side weights are shared).  f, fp: device complex[M], distinct,
 * overwritten.  The workspace of flt_plan_workspace_size covers this call.
 * Errors as for flt_forward; fp null or equal to f is FLT_EINVAL.  For callers
 * that need both values, e.g. an autograd forward that keeps f' for the
 * gradient with respect to z. */
int flt_forward_derivative(flt_plan* plan, const void* c, void* f, void* fp, void* stream);

/* Adjoint (Sect. 4, closing remarks: C^* by the adjoints of the K and A
 * factors): c_out[k] ~ sum_{j<M} g_j conj(w_j)^k, k < N.
 * g: device complex[M]; c_out: device complex[N], overwritten.
 * Error <= eps * sum|g_j|. */
int flt_adjoint(flt_plan* plan, const void* g, void* c_out, void* stream);

/* Measurement: run one forward on `stream` with HIP events recorded between
 * its stages and wait for it; stage_ms (host, 5 doubles) receives the
 * durations of (one-pass band FFTs, pass A, pass B, window gather, direct-sum
 * bands) in milliseconds.  Same arguments and results as flt_forward. */
int flt_profile_forward(flt_plan* plan, const void* c, void* f, void* stream, double* stage_ms);

/* Measurement: one adjoint, as flt_profile_forward; stage_ms (host, 8 doubles)
 * receives the durations of (clearing the FP64 accumulator and the k = 0 sum
 * of g, node-side weights and window values, cell spread onto the grids,
 * pass B, pass A with the transposed contraction, one-pass bands, direct-sum
 * bands, rounding the accumulator to c_out) in milliseconds.  Same arguments
 * and results as flt_adjoint. */
int flt_profile_adjoint(flt_plan* plan, const void* g, void* c_out, void* stream, double* stage_ms);

/* ------------------------------------------------------------------------
 * The discrete Laplace transform (Sect. 3, Algorithm 1):
 *
 *     f_j = sum_{k<N} fhat_k exp(-y_j xi_k),   xi_k > 0, y_j >= 0,
 *
 * by the dyadic partition of Def. 3.2 (y_1 = max y_j, xi_1 = max xi_k), rank-q
 * Chebyshev interpolation of every admissible block, cumulative sums for the
 * blocks where the kernel is 1, and nothing for those where it is below eps.
 * Error <= eps * sum |fhat_k| (Thm A.3).  All work after plan creation runs in
 * HIP kernels; the arithmetic is FP64 for both dtypes (dtype sets the type of
 * fhat and f: FLT_C64 complex64, FLT_C128 complex128).
 * ------------------------------------------------------------------------ */
typedef struct flt_laplace_plan flt_laplace_plan;

/* Kernels of flt_laplace_plan_create_kernel (Thm 3.3 and its example). */
#define FLT_KERNEL_EXP          0 /* exp(-y xi): Algorithm 1 */
#define FLT_KERNEL_BESSEL_K_HALF 1 /* K_{1/2}(y xi) = sqrt(pi / (2 y xi)) exp(-y xi), asymptotically smooth */

typedef struct flt_laplace_info {
    int64_t N, M;            /* frequencies, nodes */
    int32_t dtype;           /* FLT_C64 or FLT_C128 */
    int32_t q;               /* Chebyshev rank, ceil(1/2 + log4(1/eps)) */
    int32_t levels;          /* the paper's M: ceil(log2(y_1 xi_1 / eps)) + 1 (1 if every y_j = 0) for
                                FLT_KERNEL_EXP, ceil(log2(y_1 xi_1 N / eps)) + 1 for general kernels */
    int32_t kernel;          /* FLT_KERNEL_* */
    double eps, y1, xi1;     /* target accuracy and the interval lengths */
} flt_laplace_info;

/* Plan for N frequencies xi (host, N doubles, > 0, finite) and M nodes y
 * (host, M doubles, >= 0, finite); both copied.  flags: 0 or
 * FLT_FLAG_HOST_ONLY.  The plan owns one device allocation: its tables (about
 * 12 bytes per frequency and per node, plus the band-block matrices) and its
 * scratch (per block and band accumulators, 16q bytes per 2048 frequencies of
 * item partials), all rewritten by every call; transform calls allocate
 * nothing, and calls on one plan must not overlap.
 * Errors: FLT_EINVAL (null, N or M < 1, dtype, flags), FLT_EDOMAIN (eps outside
 * (0,1), xi <= 0, y < 0, non-finite values), FLT_EPRECISION (eps below 1e-6
 * for FLT_C64, 1e-14 for FLT_C128), FLT_ERANGE, FLT_EHIP, FLT_ENOMEM. */
int flt_laplace_plan_create(flt_laplace_plan** out, int64_t N, const double* xi, int64_t M, const double* y,
                            double eps, int dtype, uint32_t flags);
/* General asymptotically smooth kernels (Thm 3.3): f_j = sum_k fhat_k kappa(y_j, xi_k) with
 * kappa = FLT_KERNEL_BESSEL_K_HALF (the paper's example) or FLT_KERNEL_EXP (the same as
 * flt_laplace_plan_create).  For a general kernel every frequency block l < M is interpolated in
 * every band m < M (no blocks dropped or folded: the kernel is neither ~0 nor ~1 there), with
 * M = ceil(log2(y_1 xi_1 N / eps)) + 1 levels; the near fields (frequencies in Omega_M for every
 * node, every frequency for the nodes of Y_M) are summed directly.  The rank q is the smallest
 * whose tensor Chebyshev interpolant of the kernel is within (eps / 2) max(1, max |kappa|) of it
 * on every block, on a 33 x 33 grid per block (the per-block condition of the theorem's proof,
 * taken from the kernel itself rather than from its asymptotic-smoothness constants; relative to
 * the kernel's size where it exceeds 1, near the origin, where no floating-point sum is absolutely
 * within eps).  Error <= (eps / 2) sum_k |fhat_k| max(1, kappa(y_j xi_k / 4)) (the block maximum of
 * a kernel decreasing in y xi is at most its value at y xi / 4).
 * FLT_KERNEL_BESSEL_K_HALF needs y_j > 0 (FLT_EDOMAIN otherwise: the kernel is singular at 0);
 * FLT_EPRECISION if no rank up to 32 is enough.  Other arguments and errors as
 * flt_laplace_plan_create; the forward is flt_laplace_forward. */
int flt_laplace_plan_create_kernel(flt_laplace_plan** out, int32_t kernel, int64_t N, const double* xi, int64_t M,
                                   const double* y, double eps, int dtype, uint32_t flags);
int flt_laplace_plan_info(const flt_laplace_plan* plan, flt_laplace_info* out);
/* f[j] ~ sum_k fhat_k exp(-y_j xi_k).  fhat: device complex[N] of the plan's
 * dtype, in the order xi was given; f: device complex[M], overwritten. */
int flt_laplace_forward(flt_laplace_plan* plan, const void* fhat, void* f, void* stream);
void flt_laplace_plan_destroy(flt_laplace_plan* plan);

/* ------------------------------------------------------------------------
 * Real exponents (eq. 4.1 with xi_k >= 1 real; Sect. 4, closing remarks: the
 * transposed evaluation g(xi) and the adjoint C^*):
 *
 *     forward     f_j = sum_k c_k w_j^{xi_k}
 *     transposed  h_k = sum_j g_j w_j^{xi_k}          (the paper's g(xi_k))
 *     adjoint     h_k = sum_j g_j conj(w_j^{xi_k})
 *
 * with w_j = exp(2 pi i z_j) and the principal power w^xi = exp(xi Log w),
 * Log w = -y + 2 pi i x_p, x_p = Re z reduced to (-1/2, 1/2] (the paper leaves
 * the nonpositive real axis out; this fixes its side).  Nodes with
 * y = 2 pi Im z > ln(3 / eps) give 0 (every term is below eps / 3 there).
 *
 * Method: the Laplace factor as in Algorithm 2 (the integer plan's partition
 * and Chebyshev interpolants, evaluated at real xi), the Fourier factor of
 * each band column by an NNFFT: a Kaiser-Bessel window of half-width mw1
 * spreads the exponents onto the integers l = sigma xi (sigma in [1.9, 2]),
 * one batched integer plan evaluates every (band, column) sum at the nodes
 * x_p / sigma, and a per-node division by the window's Fourier transform
 * undoes the spread.  Error <= eps sum_k |c_k| (eps / 3 Laplace, eps / 6
 * window, eps / 6 for the inner sums after the window's amplification).
 * ------------------------------------------------------------------------ */
typedef struct flt_xi_plan flt_xi_plan;

typedef struct flt_xi_info {
    int64_t N, M;                 /* exponents, nodes */
    int32_t dtype;                /* FLT_C64 (FP32 form) or FLT_C128 */
    int32_t q;                    /* Chebyshev rank of the Laplace factor */
    int32_t mw1;                  /* frequency window half-width */
    int32_t num_bands;            /* node bands with exponents in their support */
    int32_t inner_instances;      /* inner integer sums: one per (band, column) */
    int32_t inner_mw;             /* the inner plan's window half-width (0 for a host-only plan) */
    double eps, eps_w, eps_in;    /* target; window share; inner plans' accuracy */
    double sigma_min, amp;        /* smallest frequency density; inner-error amplification */
    int64_t inner_coefficients;   /* integer frequencies over all inner sums */
    int64_t inner_nodes;          /* nodes over all inner sums (sum of q_b M_b) */
    size_t inner_workspace_bytes; /* the inner plan's workspace (0 for a host-only plan) */
} flt_xi_info;

/* Plan for N exponents xi (host, N doubles, finite, >= 1, any order, at most
 * 2^29) and M nodes z (host, 2M doubles as for flt_plan_create); both copied.
 * flags: 0 or FLT_FLAG_HOST_ONLY.  The plan owns its device memory: tables,
 * the inner batched plan with its workspace, and buffers of
 * inner_coefficients + inner_nodes complex values and N FP64 complex
 * accumulators, all rewritten by every call.  Transform calls allocate
 * nothing; calls on one plan must not overlap.  Errors: FLT_EINVAL (null,
 * N or M < 1, dtype, flags), FLT_EDOMAIN (eps outside (0,1), xi < 1 or not
 * finite, Im z < 0 or NaN), FLT_EPRECISION (eps below 1e-6 for FLT_C64,
 * 1e-14 for FLT_C128, or a window wider than supported), FLT_ERANGE
 * (N > 2^30, xi > 2^29), FLT_EHIP, FLT_ENOMEM. */
int flt_xi_plan_create(flt_xi_plan** out, int64_t N, const double* xi, int64_t M, const double* z, double eps,
                       int dtype, uint32_t flags);
int flt_xi_plan_info(const flt_xi_plan* plan, flt_xi_info* out);
/* c: device complex[N] in the order xi was given; f: device complex[M], overwritten. */
int flt_xi_forward(flt_xi_plan* plan, const void* c, void* f, void* stream);
/* g: device complex[M]; h: device complex[N] (order of xi), overwritten. */
int flt_xi_transposed(flt_xi_plan* plan, const void* g, void* h, void* stream);
int flt_xi_adjoint(flt_xi_plan* plan, const void* g, void* h, void* stream);
void flt_xi_plan_destroy(flt_xi_plan* plan);   /* NULL: no-op */

const char* flt_strerror(int code);
int flt_last_hip_error(void); /* hipError_t of the last failing HIP call in this thread */

#ifdef __cplusplus
}
#endif
#endif /* FLT_H */
