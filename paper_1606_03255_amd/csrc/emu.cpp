// CPU build of the kernel bodies, for tests only: every workgroup runs its
// FFT_THREADS / GATHER_THREADS threads with real barriers, on host copies of
// the plan tables.  It exercises exactly the index arithmetic and
// synchronisation of the GPU kernels, so tests can check it (optionally under
// AddressSanitizer) before anything is launched on a GPU.  Nothing in the
// library or its Python binding loads this file's build.
//
// A workgroup's threads are user-level fibers on one OS thread (ucontext):
// each runs until its next barrier or its end, then the next one, so a
// barrier round is complete before any thread passes it.  Built with
// FLT_EMU_OMP_TEAMS (the sanitizer build: AddressSanitizer does not follow
// context switches) they are an OpenMP team of OS threads instead.
#define _GNU_SOURCE 1
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifndef FLT_EMU_OMP_TEAMS
#include <ucontext.h>
#endif

#include <algorithm>
#include <type_traits>
#include <limits>
#include <vector>

#include "flt.h"
#include "kernels_impl.h"
#include "laplace.h"
#include "plan_host.h"
#include "xi_impl.h"

namespace flt {

#ifndef FLT_EMU_OMP_TEAMS
// The fibers of the workgroup being run on this OS thread.
struct FiberTeam {
    static constexpr size_t STACK = 256 * 1024;
    std::vector<ucontext_t> uc;
    std::vector<char> stacks;
    std::vector<uint8_t> done;
    ucontext_t sched;
    int nt = 0, b = 0, cur = 0;
    const void* body = nullptr;
    void (*call)(const void*, int t, int nt, int b) = nullptr;
    void reserve(int n)
    {
        if ((int)uc.size() >= n) return;
        uc.resize(n);
        done.resize(n);
        stacks.assign((size_t)n * STACK, 0);
    }
};
static thread_local FiberTeam g_team;
static void fiber_barrier()
{
    FiberTeam& T = g_team;
    swapcontext(&T.uc[T.cur], &T.sched);
}
static void fiber_entry()
{
    FiberTeam& T = g_team;
    const int t = T.cur;
    T.call(T.body, t, T.nt, T.b);
    T.done[t] = 1;   // returns to T.sched (uc_link)
}
#endif

struct HostCtx {
    int t, nt, b;
    int tid() const { return t; }
    int ntid() const { return nt; }
    int bid() const { return b; }
    void sync() const {
#ifdef FLT_EMU_OMP_TEAMS
#pragma omp barrier
#else
        fiber_barrier();
#endif
    }
    void atomic_add(double* p, double v) const {
#pragma omp atomic
        *p += v;
    }
    void atomic_add(float* p, float v) const {
#pragma omp atomic
        *p += v;
    }
};

// Workgroups of the persistent kernels here: few, so that every one of them
// takes several items of different transform lengths.
static const int EMU_PERSIST_BLOCKS = 5;

// Scratch and LDS stand-ins start as NaN (device memory and LDS hold whatever
// they held), so a read before the kernels' own write shows in the result.
template <typename T> static cplx<T> nan_c()
{
    return mk<T>(std::numeric_limits<T>::quiet_NaN(), std::numeric_limits<T>::quiet_NaN());
}

template <typename T> static std::vector<T> cast(const std::vector<double>& v)
{
    return std::vector<T>(v.begin(), v.end());
}

// LDS stand-ins of the kernels being run: every workgroup's LDS starts with
// whatever it held, so each is refilled with all-ones bytes (NaN in FP32 and
// FP64) before every workgroup; a read before the workgroup's own write shows
// in the result instead of seeing the previous workgroup's values.
static thread_local std::vector<std::pair<void*, size_t>> g_lds;
struct LdsReg {   // registered while in scope (registrations nest)
    template <class V> explicit LdsReg(V& v) { g_lds.emplace_back((void*)v.data(), v.size() * sizeof(v[0])); }
    ~LdsReg() { g_lds.pop_back(); }
    LdsReg(const LdsReg&) = delete;
    LdsReg& operator=(const LdsReg&) = delete;
};
static void lds_poison()
{
    for (const auto& e : g_lds) memset(e.first, 0xFF, e.second);
}

template <class F> static void run_blocks(size_t nblocks, int nthreads, F&& body)
{
#ifdef FLT_EMU_OMP_TEAMS
    for (size_t b = 0; b < nblocks; ++b) {
        lds_poison();
#pragma omp parallel num_threads(nthreads)
        {
            HostCtx ctx{omp_get_thread_num(), omp_get_num_threads(), (int)b};
            body(ctx);
        }
    }
#else
    using Fn = typename std::remove_reference<F>::type;
    FiberTeam& T = g_team;
    T.reserve(nthreads);
    T.nt = nthreads;
    T.body = &body;
    T.call = [](const void* f, int t, int nt, int b) {
        const HostCtx ctx{t, nt, b};
        (*(const Fn*)f)(ctx);
    };
    for (size_t b = 0; b < nblocks; ++b) {
        lds_poison();
        T.b = (int)b;
        for (int t = 0; t < nthreads; ++t) {
            getcontext(&T.uc[t]);
            T.uc[t].uc_stack.ss_sp = T.stacks.data() + (size_t)t * FiberTeam::STACK;
            T.uc[t].uc_stack.ss_size = FiberTeam::STACK;
            T.uc[t].uc_link = &T.sched;
            makecontext(&T.uc[t], fiber_entry, 0);
            T.done[t] = 0;
        }
        // barrier rounds: every live fiber runs to its next barrier (or end)
        for (int live = nthreads; live > 0;) {
            for (int t = 0; t < nthreads; ++t) {
                if (T.done[t]) continue;
                T.cur = t;
                swapcontext(&T.sched, &T.uc[t]);
                if (T.done[t]) --live;
            }
        }
    }
#endif
}

template <typename T, int MW>
static void nodes_mw(const PlanView<T>& pv, const HostPlan& hp, int adjoint, const cplx<T>* c, cplx<T>* grids,
                     cplx<T>* f, int with_c0, cplx<T>* U, T* Phi, int32_t* L0, cplx<T>* f2)
{
    if (!adjoint) {
        std::vector<cplx<T>> stage(GATHER_STAGE, nan_c<T>());
        const LdsReg r_stage(stage);
        run_blocks(hp.gather_st.size(), GATHER_THREADS, [&](const HostCtx& ctx) {
            body_gather<HostCtx, T, MW, true>(ctx, pv, hp.gather_st.data(), c, grids, f, with_c0, f2, stage.data());
        });
        run_blocks(hp.gather_ln.size(), GATHER_THREADS, [&](const HostCtx& ctx) {
            body_gather<HostCtx, T, MW, false>(ctx, pv, hp.gather_ln.data(), c, grids, f, with_c0, f2, nullptr);
        });
        return;
    }
    run_blocks(hp.nfft_nodes.size(), GATHER_THREADS, [&](const HostCtx& ctx) {
        body_adj_prep<HostCtx, T, MW>(ctx, pv, hp.nfft_nodes.data(), c, hp.qs, U, Phi, L0);
    });
    std::vector<T> red(2 * ADJ_RC * GATHER_THREADS, std::numeric_limits<T>::quiet_NaN());
    const LdsReg r_red(red);
    run_blocks(hp.cells.size(), GATHER_THREADS, [&](const HostCtx& ctx) {
        body_adj_cells<HostCtx, T, MW>(ctx, pv, hp.cells.data(), hp.qs, U, Phi, L0, hp.cstart.data(),
                                       hp.clist.data(), grids, red.data());
    });
}

template <typename T>
static int emu_run(const HostPlan& hp, int op, const void* in, void* out)
{
    const std::vector<T> coef = cast<T>(hp.coef), deconv = cast<T>(hp.deconv);
    const std::vector<T> tws = cast<T>(hp.tw_stage), twl = cast<T>(hp.tw_lo), twh = cast<T>(hp.tw_hi);
    PlanView<T> pv;
    pv.bands = hp.bands.data();
    pv.coef = coef.data();
    pv.deconv = deconv.data();
    pv.ycheb = hp.ycheb.data();
    pv.tw_stage = (const cplx<T>*)tws.data();
    pv.tw_lo = (const cplx<T>*)twl.data();
    pv.tw_hi = (const cplx<T>*)twh.data();
    pv.nx = hp.nx.data();
    pv.ny = hp.ny.data();
    pv.perm = hp.perm.data();
    pv.mask = hp.mask.data();
    pv.inst = hp.inst.data();
    pv.mw = hp.mw;
    pv.kb_b = (T)hp.kb_b;

    // exactly sized buffers, so AddressSanitizer sees any out-of-range access;
    // the workspace and LDS start as NaN, as device memory holds whatever it
    // held: a value read before the kernels write it shows in the result
    const int cols = op == 3 ? 2 : 1;   // op 3: forward and derivative, 2q columns per band
    const T qnan = std::numeric_limits<T>::quiet_NaN();
    const cplx<T> cnan = nan_c<T>();
    std::vector<cplx<T>> grids(std::max<int64_t>(hp.grid_elems * cols, 1), cnan);
    std::vector<cplx<T>> scratch(std::max<int64_t>(hp.scratch_elems * cols, 1), cnan);
    std::vector<cplx<T>> U((size_t)hp.M * hp.qs, cnan);
    std::vector<T> Phi((size_t)hp.M * 2 * hp.mw, qnan);
    std::vector<int32_t> L0(hp.M);
    std::vector<double> dacc(2 * hp.M, 0.0), red(2 * 256 * DIRECT_NG);
    std::vector<cplx<T>> lds(tile_alloc<T>(), cnan);
    std::vector<T> lc(Sizes<T>::COEF, qnan);
    std::vector<T> lc1(onepass_coef<T>(), qnan);   // the one-pass FFT's staged coefficients
    std::vector<cplx<T>> lds2(2 * tile_alloc<T>(), cnan);   // the FP32 pass A's two tiles and coefficient buffers
    std::vector<T> lc2(2 * Sizes<T>::COEF, qnan);
    std::vector<cplx<T>> omega(PASSA_OMEGA_MAX);
    std::vector<cplx<T>> passb_tw(lds_tw_half<Log2Range<T>::B_HI>(), cnan);   // pass B's twiddle half table
    const LdsReg r_red(red), r_lds(lds), r_lc(lc), r_lc1(lc1), r_lds2(lds2), r_lc2(lc2), r_omega(omega), r_pbtw(passb_tw);
    std::vector<cplx<T>> basebuf(std::max<int64_t>(hp.base_elems, 1));
    const int64_t nd = (int64_t)hp.dlist.size();
    auto mwsw = [&](int adjoint, const cplx<T>* c, cplx<T>* f, int with_c0, cplx<T>* f2) {
        switch (hp.mw) {
#define G(MWV) case MWV: nodes_mw<T, MWV>(pv, hp, adjoint, c, grids.data(), f, with_c0, U.data(), Phi.data(), L0.data(), f2); break;
            G(2) G(3) G(4) G(5) G(6) G(7) G(8) G(9) G(10)
#undef G
        }
    };
    if (op == 0 || op == 1 || op == 3) {
        const cplx<T>* c = (const cplx<T>*)in;
        cplx<T>* f = (cplx<T>*)out;
        cplx<T>* f2 = op == 3 ? f + hp.M : nullptr;   // op 3: out holds f, then f'
        const int deriv = op == 1;
        constexpr int LP = Sizes<T>::LOG2P;
        const std::vector<FftItem>& one = cols == 2 ? hp.onepass_fused : hp.onepass_fwd;
        const std::vector<FftItem>& pb = cols == 2 ? hp.passB_fused : hp.passB;
        for (const LaunchGroup& g : (cols == 2 ? hp.g_onepass_fused : hp.g_onepass_fwd))
            with_log2<4, LP>(g.log2, [&](auto LG) {
                run_blocks(g.count, FFT_THREADS, [&](const HostCtx& ctx) {
                    body_onepass_fwd<HostCtx, T, decltype(LG)::value>(ctx, pv, one.data() + g.start, c,
                                                                      grids.data(), deriv, cols, lds.data(),
                                                                      lc1.data());
                });
            });
        for (const LaunchGroup& g : hp.g_passA_fwd)
            with_log2<LP + 1, TW2_LOG2>(g.log2, [&](auto LG) {
                run_blocks(g.count, FFT_THREADS, [&](const HostCtx& ctx) {
                    if constexpr (sizeof(T) == 4)
                        body_passA_fwd<HostCtx, T, decltype(LG)::value>(ctx, pv, hp.passA_fwd.data() + g.start, c,
                                                                        scratch.data(), deriv, cols, lds2.data(),
                                                                        lc2.data(), omega.data());
                    else
                        body_passA_fwd_slot<HostCtx, T, decltype(LG)::value>(ctx, pv, hp.passA_fwd.data() + g.start,
                                                                             c, scratch.data(), basebuf.data(), deriv,
                                                                             cols, lds.data(), lc.data());
                });
            });
        if (!pb.empty()) {
            // persistent: a few workgroups, each taking every nb-th item
            const int n = (int)pb.size();
            const int nb = passB_prefetch<T, +1>() ? std::min(n, EMU_PERSIST_BLOCKS) : n;
            run_blocks(nb, FFT_THREADS, [&](const HostCtx& ctx) {
                body_passB<HostCtx, T, +1>(ctx, pv, pb.data(), n, nb, scratch.data(), grids.data(), cols, lds.data(),
                                           passb_tw.data());
            });
        }
        mwsw(0, c, f, !deriv, f2);
        for (int d = 0; d < cols && nd; ++d) {
            cplx<T>* o = d ? f2 : f;
            run_blocks((nd + 255) / 256, 256, [&](const HostCtx& ctx) {
                body_direct_io<HostCtx, T>(ctx, pv, hp.dlist.data(), nd, dacc.data(), o, 0);
            });
            std::vector<cplx<T>> nw(DIRECT_NG * DIRECT_GMAX, nan_c<T>());
            const LdsReg r_nw(nw);
            run_blocks(hp.direct_fwd.size(), 256, [&](const HostCtx& ctx) {
                if (deriv || d)
                    body_direct_fwd<HostCtx, T, true, false>(ctx, pv, hp.direct_fwd.data(), hp.dlist.data(), c,
                                                             dacc.data(), red.data(), nw.data());
                else
                    body_direct_fwd<HostCtx, T, false, false>(ctx, pv, hp.direct_fwd.data(), hp.dlist.data(), c,
                                                              dacc.data(), red.data(), nw.data());
            });
            run_blocks(hp.direct_short.size(), 256, [&](const HostCtx& ctx) {
                if (deriv || d)
                    body_direct_fwd<HostCtx, T, true, true>(ctx, pv, hp.direct_short.data(), hp.dlist.data(), c,
                                                            dacc.data(), red.data(), nw.data());
                else
                    body_direct_fwd<HostCtx, T, false, true>(ctx, pv, hp.direct_short.data(), hp.dlist.data(), c,
                                                             dacc.data(), red.data(), nw.data());
            });
            run_blocks((nd + 255) / 256, 256, [&](const HostCtx& ctx) {
                body_direct_io<HostCtx, T>(ctx, pv, hp.dlist.data(), nd, dacc.data(), o, 1);
            });
        }
        return FLT_OK;
    }
    if (op == 2) {
        const cplx<T>* g = (const cplx<T>*)in;
        cplx<T>* co = (cplx<T>*)out;
        std::vector<double> acc(2 * hp.N, 0.0);
        run_blocks(hp.sum_items.size(), 256, [&](const HostCtx& ctx) {
            body_sum_g<HostCtx, T>(ctx, pv, hp.sum_items.data(), g, acc.data(), red.data());
        });
        mwsw(1, g, nullptr, 0, nullptr);
        constexpr int LP = Sizes<T>::LOG2P;
        if (!hp.passB.empty()) {
            const int n = (int)hp.passB.size();
            const int nb = passB_prefetch<T, -1>() ? std::min(n, EMU_PERSIST_BLOCKS) : n;
            run_blocks(nb, FFT_THREADS, [&](const HostCtx& ctx) {
                body_passB<HostCtx, T, -1>(ctx, pv, hp.passB.data(), n, nb, grids.data(), scratch.data(), 1, lds.data(),
                                           passb_tw.data());
            });
        }
        for (const LaunchGroup& g : hp.g_passA_adj)
            with_log2<LP + 1, TW2_LOG2>(g.log2, [&](auto LG) {
                run_blocks(g.count, FFT_THREADS, [&](const HostCtx& ctx) {
                    if constexpr (sizeof(T) == 4)
                        body_passA_adj<HostCtx, T, decltype(LG)::value>(ctx, pv, hp.passA_adj.data() + g.start,
                                                                        scratch.data(), acc.data(), lds2.data(),
                                                                        lc2.data(), omega.data());
                    else
                        body_passA_adj_1tile<HostCtx, T, decltype(LG)::value>(ctx, pv, hp.passA_adj.data() + g.start,
                                                                              scratch.data(), acc.data(), lds.data(),
                                                                              lc.data());
                });
            });
        for (const LaunchGroup& g : hp.g_onepass_adj)
            with_log2<4, LP>(g.log2, [&](auto LG) {
                run_blocks(g.count, FFT_THREADS, [&](const HostCtx& ctx) {
                    body_onepass_adj<HostCtx, T, decltype(LG)::value>(ctx, pv, hp.onepass_adj.data() + g.start,
                                                                      grids.data(), acc.data(), lds.data());
                });
            });
        std::vector<cplx<T>> nw(DIRECT_ANG, nan_c<T>()), ngv(DIRECT_ANG, nan_c<T>()), redv(256 * ADJ_TS, nan_c<T>());
        const LdsReg r_nw(nw), r_ngv(ngv), r_redv(redv);
        run_blocks(hp.direct_adj.size(), 256, [&](const HostCtx& ctx) {
            body_direct_adj<HostCtx, T>(ctx, pv, hp.direct_adj.data(), hp.dlist.data(), g, acc.data(), nw.data(),
                                        ngv.data(), redv.data());
        });
        for (int64_t k = 0; k < hp.N; ++k) co[k] = mk<T>((T)acc[2 * k], (T)acc[2 * k + 1]);
        return FLT_OK;
    }
    return FLT_EINVAL;
}

}  // namespace flt

namespace flt {

// The Laplace transform's kernel bodies on the CPU (same plan, same launches).
template <typename T> static int emu_laplace(const LapHost& hp, const void* in, void* out)
{
    // garbage: every call must write each accumulator and partial before reading it
    std::vector<double> acc((size_t)lap_acc_doubles(hp.L, hp.q), 1e300);
    std::vector<double> part(hp.items.size() * 2 * hp.q, 1e300);
    LapView V{};
    V.q = hp.q;
    V.L = hp.L;
    V.kernel = hp.kernel;
    V.near0 = hp.near0;
    V.nnear = hp.nnear;
    V.N = hp.N;
    V.xs = hp.xs.data();
    V.kperm = hp.kperm.data();
    V.bcw = hp.bcw.data();
    V.ycw = hp.ycw.data();
    V.lm = hp.lm.data();
    V.Lm = hp.Lm.data();
    V.koff = hp.koff.data();
    V.K = hp.K.data();
    V.y = hp.y.data();
    V.band = hp.band.data();
    V.bitem = hp.bitem.data();
    V.nitems = (int32_t)hp.items.size();
    V.part = part.data();
    V.acc = acc.data();
    const double dnan = std::numeric_limits<double>::quiet_NaN();
    std::vector<double> red(8 * LAP_THREADS, dnan), red2(LAP_THREADS, dnan), rred(LAP_THREADS, dnan),
        bred(4 * LAP_THREADS, dnan);
    const LdsReg r_red(red), r_red2(red2), r_rred(rred), r_bred(bred);
    auto all = [&](auto qb) {
        constexpr int QB = decltype(qb)::value;
        run_blocks(hp.items.size(), LAP_THREADS, [&](const HostCtx& ctx) {
            lap_body_moments<HostCtx, T, QB>(ctx, V, hp.items.data(), (const cplx<T>*)in, red.data(), red2.data());
        });
        run_blocks((size_t)hp.L, LAP_THREADS, [&](const HostCtx& ctx) { lap_body_reduce(ctx, V, rred.data()); });
        run_blocks((size_t)hp.L, LAP_THREADS, [&](const HostCtx& ctx) { lap_body_bands<HostCtx, QB>(ctx, V, bred.data()); });
        const int64_t per = (int64_t)LAP_THREADS * LAP_NODE_PER, ns = lap_node_stage(hp.L, hp.q);
        std::vector<double> sb((size_t)std::max<int64_t>(ns, 1), dnan);
        const LdsReg r_sb(sb);
        run_blocks((hp.M + per - 1) / per, LAP_THREADS, [&](const HostCtx& ctx) {
            lap_body_nodes<HostCtx, T, QB>(ctx, V, hp.M, (cplx<T>*)out, ns > 0 ? sb.data() : nullptr,
                                           (const cplx<T>*)in);
        });
    };
    switch (lap_qbucket(hp.q)) {
    case 8: all(std::integral_constant<int, 8>()); break;
    case 12: all(std::integral_constant<int, 12>()); break;
    case 16: all(std::integral_constant<int, 16>()); break;
    case 24: all(std::integral_constant<int, 24>()); break;
    default: all(std::integral_constant<int, 32>()); break;
    }
    return FLT_OK;
}

// The real-exponent transform on the CPU: op 0 forward (in c, out f), 1
// transposed, 2 adjoint (in g, out h); the inner sums by emu_run.
template <typename T> static int emu_xi(XiHost& hp, int op, const void* in, void* out)
{
    HostPlan inner;
    int rc = build_batch_plan(inner, (int32_t)hp.in_N.size(), hp.in_N.data(), hp.in_M.data(), hp.in_z.data(),
                              hp.eps_in, hp.dtype, PLAN_FLAG_NO_FLOOR);
    if (rc != FLT_OK) return rc;
    const std::vector<T> coef = cast<T>(hp.outer.coef);
    XiView<T> xv;
    xv.bands = hp.bands.data();
    xv.coef = coef.data();
    xv.ycheb = hp.outer.ycheb.data();
    xv.xi = hp.xi.data();
    xv.xi_perm = hp.xi_perm.data();
    xv.xp = hp.xp.data();
    xv.ny = hp.outer.ny.data();
    xv.perm = hp.outer.perm.data();
    xv.mw1 = hp.mw1;
    int qmax = 1;
    for (const XiBand& X : hp.bands) qmax = std::max(qmax, (int)X.q);
    std::vector<cplx<T>> cin(std::max<int64_t>(hp.cin_elems, 1), nan_c<T>()),
        hout(std::max<int64_t>(hp.hout_elems, 1), nan_c<T>());
    std::vector<T> lc(XI_NBLK * 32 * 32, std::numeric_limits<T>::quiet_NaN());
    std::vector<cplx<T>> ct(32 * 1024 / sizeof(cplx<T>), nan_c<T>());   // xi_kcap * QM for every QM
    const LdsReg r_lc(lc), r_ct(ct);
    if (op == 0) {
        run_blocks(hp.spread.size(), XI_THREADS, [&](const HostCtx& ctx) {
            if (qmax <= 16) body_xi_spread<HostCtx, T, 16>(ctx, xv, hp.spread.data(), (const cplx<T>*)in, cin.data(), lc.data(), ct.data());
            else if (qmax <= 24) body_xi_spread<HostCtx, T, 24>(ctx, xv, hp.spread.data(), (const cplx<T>*)in, cin.data(), lc.data(), ct.data());
            else body_xi_spread<HostCtx, T, 32>(ctx, xv, hp.spread.data(), (const cplx<T>*)in, cin.data(), lc.data(), ct.data());
        });
        rc = emu_run<T>(inner, 0, cin.data(), hout.data());
        if (rc != FLT_OK) return rc;
        run_blocks(hp.nodes.size(), GATHER_THREADS, [&](const HostCtx& ctx) {
            body_xi_combine<HostCtx, T>(ctx, xv, hp.nodes.data(), hout.data(), (cplx<T>*)out);
        });
        return FLT_OK;
    }
    const int conj = op == 2;
    run_blocks(hp.nodes.size(), GATHER_THREADS, [&](const HostCtx& ctx) {
        body_xi_prep<HostCtx, T>(ctx, xv, hp.nodes.data(), (const cplx<T>*)in, conj, hout.data());
    });
    rc = emu_run<T>(inner, 2, hout.data(), cin.data());
    if (rc != FLT_OK) return rc;
    std::vector<double> hacc(2 * hp.N, 0.0);
    run_blocks(hp.gather.size(), XI_THREADS, [&](const HostCtx& ctx) {
        if (qmax <= 16) body_xi_gather<HostCtx, T, 16>(ctx, xv, hp.gather.data(), cin.data(), hacc.data(), lc.data());
        else if (qmax <= 24) body_xi_gather<HostCtx, T, 24>(ctx, xv, hp.gather.data(), cin.data(), hacc.data(), lc.data());
        else body_xi_gather<HostCtx, T, 32>(ctx, xv, hp.gather.data(), cin.data(), hacc.data(), lc.data());
    });
    run_blocks((hp.N + XI_THREADS - 1) / XI_THREADS, XI_THREADS, [&](const HostCtx& ctx) {
        body_xi_finalize<HostCtx, T>(ctx, xv, hp.N, hacc.data(), conj, (cplx<T>*)out);
    });
    return FLT_OK;
}

}  // namespace flt

// The real-exponent transform on the CPU build: op 0 forward, 1 transposed,
// 2 adjoint (see flt_xi_forward / flt_xi_transposed / flt_xi_adjoint).
extern "C" int flt_emu_xi(int64_t N, const double* xi, int64_t M, const double* z, double eps, int dtype, int op,
                          const void* in, void* out)
{
    flt::XiHost hp;
    int rc = flt::build_xi_plan(hp, N, xi, M, z, eps, dtype);
    if (rc != FLT_OK) return rc;
    return dtype == FLT_C64 ? flt::emu_xi<float>(hp, op, in, out) : flt::emu_xi<double>(hp, op, in, out);
}

// The kernel bodies on the CPU for one call: op 0 forward, 1 derivative,
// 2 adjoint, 3 forward and derivative in one pass (out: f, then f', 2M values).
extern "C" int flt_emu_run(int64_t N, int64_t M, const double* z, double eps, int dtype, uint32_t flags, int op,
                           const void* in, void* out)
{
    flt::HostPlan hp;
    int rc = flt::build_host_plan(hp, N, M, z, eps, dtype, flags);
    if (rc != FLT_OK) return rc;
    return dtype == FLT_C64 ? flt::emu_run<float>(hp, op, in, out) : flt::emu_run<double>(hp, op, in, out);
}

// The same for a batched plan (packed in / out, see flt_plan_create_batch).
extern "C" int flt_emu_run_batch(int32_t count, const int64_t* N, const int64_t* M, const double* z, double eps,
                                 int dtype, uint32_t flags, int op, const void* in, void* out)
{
    flt::HostPlan hp;
    int rc = flt::build_batch_plan(hp, count, N, M, z, eps, dtype, flags);
    if (rc != FLT_OK) return rc;
    return dtype == FLT_C64 ? flt::emu_run<float>(hp, op, in, out) : flt::emu_run<double>(hp, op, in, out);
}

// The Laplace transform on the CPU build (in: fhat, out: f, the plan's dtype).
extern "C" int flt_emu_laplace(int64_t N, const double* xi, int64_t M, const double* y, double eps, int dtype,
                               const void* in, void* out)
{
    flt::LapHost hp;
    int rc = flt::build_laplace_plan(hp, N, xi, M, y, eps, dtype);
    if (rc != FLT_OK) return rc;
    return dtype == FLT_C64 ? flt::emu_laplace<float>(hp, in, out) : flt::emu_laplace<double>(hp, in, out);
}

// The same for a chosen kernel (FLT_KERNEL_*, see flt_laplace_plan_create_kernel).
extern "C" int flt_emu_laplace_kernel(int kernel, int64_t N, const double* xi, int64_t M, const double* y,
                                      double eps, int dtype, const void* in, void* out)
{
    flt::LapHost hp;
    int rc = flt::build_laplace_plan(hp, N, xi, M, y, eps, dtype, kernel);
    if (rc != FLT_OK) return rc;
    return dtype == FLT_C64 ? flt::emu_laplace<float>(hp, in, out) : flt::emu_laplace<double>(hp, in, out);
}
