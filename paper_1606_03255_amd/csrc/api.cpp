// C-ABI of the fast Fourier-Laplace transform (see include/flt.h).
#include <hip/hip_runtime_api.h>
#include <string.h>

#include <exception>
#include <map>
#include <mutex>
#include <new>
#include <system_error>
#include <thread>
#include <tuple>
#include <vector>

#include "flt.h"
#include "launch.h"
#include "plan_host.h"

using namespace flt;

static thread_local int g_last_hip = 0;

// A captured launch sequence (FLT_FLAG_GRAPH): valid for one operation and
// one set of buffers; a call with other buffers captures anew.
struct GraphSlot {
    const void* in = nullptr;
    void* out = nullptr;
    void* out2 = nullptr;
    char* ws = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct flt_plan {
    HostPlan hp;
    bool host_only = true;
    int device = -1;
    void* dev = nullptr;     // one allocation holding every table and list
    PlanView<float> pv32{};
    PlanView<double> pv64{};
    DevLists lists{};
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t capture = nullptr;   // FLT_FLAG_GRAPH: stream the sequences are captured on
    GraphSlot graphs[4];             // forward, derivative, adjoint, forward + derivative
};

static int hip_fail(hipError_t e)
{
    g_last_hip = (int)e;
    return FLT_EHIP;
}

namespace {
struct Packer {
    std::vector<char> buf;
    size_t add(const void* p, size_t bytes)
    {
        size_t off = (buf.size() + 255) & ~(size_t)255;
        buf.resize(off + (bytes ? bytes : 1));
        if (bytes) memcpy(buf.data() + off, p, bytes);
        return off;
    }
    template <typename T> size_t add_cast(const std::vector<double>& v)
    {
        std::vector<T> t(v.begin(), v.end());
        return add(t.data(), t.size() * sizeof(T));
    }
};
}  // namespace

template <typename T> static PlanView<T> make_view(const HostPlan& hp, char* base, size_t o_bands, size_t o_coef,
                                                   size_t o_deconv, size_t o_ycheb, size_t o_tws, size_t o_twl,
                                                   size_t o_twh, size_t o_nx, size_t o_ny, size_t o_perm,
                                                   size_t o_mask, size_t o_inst)
{
    PlanView<T> pv;
    pv.bands = (const BandDesc*)(base + o_bands);
    pv.coef = (const T*)(base + o_coef);
    pv.deconv = (const T*)(base + o_deconv);
    pv.ycheb = (const double*)(base + o_ycheb);
    pv.tw_stage = (const cplx<T>*)(base + o_tws);
    pv.tw_lo = (const cplx<T>*)(base + o_twl);
    pv.tw_hi = (const cplx<T>*)(base + o_twh);
    pv.nx = (const double*)(base + o_nx);
    pv.ny = (const double*)(base + o_ny);
    pv.perm = (const int32_t*)(base + o_perm);
    pv.mask = (const uint32_t*)(base + o_mask);
    pv.inst = (const InstDesc*)(base + o_inst);
    pv.mw = hp.mw;
    pv.kb_b = (T)hp.kb_b;
    return pv;
}

static int upload(flt_plan* p)
{
    const HostPlan& hp = p->hp;
    const bool f32 = hp.dtype == FLT_C64;
    Packer pk;
    const size_t o_bands = pk.add(hp.bands.data(), hp.bands.size() * sizeof(BandDesc));
    const size_t o_coef = f32 ? pk.add_cast<float>(hp.coef) : pk.add_cast<double>(hp.coef);
    const size_t o_deconv = f32 ? pk.add_cast<float>(hp.deconv) : pk.add_cast<double>(hp.deconv);
    const size_t o_ycheb = pk.add(hp.ycheb.data(), hp.ycheb.size() * sizeof(double));
    const size_t o_tws = f32 ? pk.add_cast<float>(hp.tw_stage) : pk.add_cast<double>(hp.tw_stage);
    const size_t o_twl = f32 ? pk.add_cast<float>(hp.tw_lo) : pk.add_cast<double>(hp.tw_lo);
    const size_t o_twh = f32 ? pk.add_cast<float>(hp.tw_hi) : pk.add_cast<double>(hp.tw_hi);
    const size_t o_nx = pk.add(hp.nx.data(), hp.nx.size() * sizeof(double));
    const size_t o_ny = pk.add(hp.ny.data(), hp.ny.size() * sizeof(double));
    const size_t o_perm = pk.add(hp.perm.data(), hp.perm.size() * sizeof(int32_t));
    const size_t o_l0 = pk.add(hp.onepass_fwd.data(), hp.onepass_fwd.size() * sizeof(FftItem));
    const size_t o_lf0 = pk.add(hp.onepass_fused.data(), hp.onepass_fused.size() * sizeof(FftItem));
    const size_t o_l1 = pk.add(hp.passA_fwd.data(), hp.passA_fwd.size() * sizeof(FftItem));
    const size_t o_l2 = pk.add(hp.passB.data(), hp.passB.size() * sizeof(FftItem));
    const size_t o_l3 = pk.add(hp.onepass_adj.data(), hp.onepass_adj.size() * sizeof(FftItem));
    const size_t o_l4 = pk.add(hp.passA_adj.data(), hp.passA_adj.size() * sizeof(FftItem));
    const size_t o_lf2 = pk.add(hp.passB_fused.data(), hp.passB_fused.size() * sizeof(FftItem));
    const size_t o_l5 = pk.add(hp.gather_st.data(), hp.gather_st.size() * sizeof(NodeItem));
    const size_t o_l5b = pk.add(hp.gather_ln.data(), hp.gather_ln.size() * sizeof(NodeItem));
    const size_t o_l6 = pk.add(hp.cells.data(), hp.cells.size() * sizeof(CellItem));
    const size_t o_l7 = pk.add(hp.nfft_nodes.data(), hp.nfft_nodes.size() * sizeof(NodeItem));
    const size_t o_l8 = pk.add(hp.direct_fwd.data(), hp.direct_fwd.size() * sizeof(DirectItem));
    const size_t o_l8s = pk.add(hp.direct_short.data(), hp.direct_short.size() * sizeof(DirectItem));
    const size_t o_l9 = pk.add(hp.direct_adj.data(), hp.direct_adj.size() * sizeof(DirectItem));
    const size_t o_dl = pk.add(hp.dlist.data(), hp.dlist.size() * sizeof(int32_t));
    const size_t o_cs = pk.add(hp.cstart.data(), hp.cstart.size() * sizeof(int32_t));
    const size_t o_cl = pk.add(hp.clist.data(), hp.clist.size() * sizeof(int32_t));
    const size_t o_mask = pk.add(hp.mask.data(), hp.mask.size() * sizeof(uint32_t));
    const size_t o_inst = pk.add(hp.inst.data(), hp.inst.size() * sizeof(InstDesc));
    const size_t o_sum = pk.add(hp.sum_items.data(), hp.sum_items.size() * sizeof(SumItem));

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) return hip_fail(e);
    e = hipMalloc(&p->dev, pk.buf.size());
    if (e != hipSuccess) return hip_fail(e);
    e = hipMemcpy(p->dev, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    char* base = (char*)p->dev;
    p->pv32 = make_view<float>(hp, base, o_bands, o_coef, o_deconv, o_ycheb, o_tws, o_twl, o_twh, o_nx, o_ny, o_perm, o_mask, o_inst);
    p->pv64 = make_view<double>(hp, base, o_bands, o_coef, o_deconv, o_ycheb, o_tws, o_twl, o_twh, o_nx, o_ny, o_perm, o_mask, o_inst);
    DevLists& L = p->lists;
    L.onepass_fwd = (const FftItem*)(base + o_l0);
    L.onepass_fused = (const FftItem*)(base + o_lf0);
    L.n_onepass_fwd = (int)hp.onepass_fwd.size();
    L.n_onepass_fused = (int)hp.onepass_fused.size();
    L.passA_fwd = (const FftItem*)(base + o_l1);
    L.passB = (const FftItem*)(base + o_l2);
    L.onepass_adj = (const FftItem*)(base + o_l3);
    L.passA_adj = (const FftItem*)(base + o_l4);
    L.passB_fused = (const FftItem*)(base + o_lf2);
    L.n_passB_fused = (int)hp.passB_fused.size();
    L.gather_st = (const NodeItem*)(base + o_l5);
    L.gather_ln = (const NodeItem*)(base + o_l5b);
    L.cells = (const CellItem*)(base + o_l6);
    L.nfft_nodes = (const NodeItem*)(base + o_l7);
    L.direct_fwd = (const DirectItem*)(base + o_l8);
    L.direct_short = (const DirectItem*)(base + o_l8s);
    L.n_direct_short = (int)hp.direct_short.size();
    L.direct_adj = (const DirectItem*)(base + o_l9);
    L.dlist = (const int32_t*)(base + o_dl);
    L.cstart = (const int32_t*)(base + o_cs);
    L.clist = (const int32_t*)(base + o_cl);
    L.sum_items = (const SumItem*)(base + o_sum);
    L.n_sum = (int)hp.sum_items.size();
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0) {
        L.persist_blocks = 2 * cus;
    }
    L.n_passA_fwd = (int)hp.passA_fwd.size();
    L.n_passB = (int)hp.passB.size();
    L.n_onepass_adj = (int)hp.onepass_adj.size();
    L.n_passA_adj = (int)hp.passA_adj.size();
    L.n_gather_st = (int)hp.gather_st.size();
    L.n_gather_ln = (int)hp.gather_ln.size();
    L.n_cells = (int)hp.cells.size();
    L.n_nfft_nodes = (int)hp.nfft_nodes.size();
    L.n_direct_fwd = (int)hp.direct_fwd.size();
    L.n_direct_adj = (int)hp.direct_adj.size();
    L.n_dlist = (int64_t)hp.dlist.size();
    L.g_onepass_fwd = hp.g_onepass_fwd;
    L.g_passA_fwd = hp.g_passA_fwd;
    L.g_passB = hp.g_passB;
    L.g_onepass_adj = hp.g_onepass_adj;
    L.g_passA_adj = hp.g_passA_adj;
    return FLT_OK;
}

static const uint32_t KNOWN_FLAGS =
    FLT_FLAG_HOST_ONLY | FLT_FLAG_NFFT_ONLY | FLT_FLAG_GRAPH | FLT_FLAG_AUTOTUNE | FLT_FLAG_TUNE_FORWARD;

static void release(flt_plan* p);
static hipError_t enqueue(flt_plan* p, int op, const void* in, void* out, void* out2, hipStream_t st);

// FLT_FLAG_AUTOTUNE: a plan's shape chosen by timing forward + adjoint
// (FLT_FLAG_TUNE_FORWARD: the forward alone) of candidates on the device, one
// dimension after the other:
//   1. the band policy's direct-sum rate factor (TUNE_SCALES, distinct band
//      choices only, one plan each);
//   2. workgroups per compute unit of the persistent pass B (TUNE_BLOCKS;
//      launch shapes of one plan).
// Every candidate of a step is timed twice, the first pass a warm-up; in the
// listed order each replaces the current choice only when at least 5% faster,
// so candidates within timing noise keep the first.  The result is cached per
// (objective, dtype, eps, instances, size class of sum N and sum M) for the
// life of the process.
namespace {
const double TUNE_SCALES[] = {0.0, 0.5, 1.0, 2.0, 4.0, 8.0};
const int TUNE_BLOCKS[] = {2, 1, 3, 4};
struct Tuned {
    PlanShape shape;
    int passB_per_cu = 2;
};
using TuneKey = std::tuple<int, int, double, int64_t, int, int>;
std::map<TuneKey, Tuned> g_tuned;
std::mutex g_tune_mu;

int size_class(int64_t v)
{
    int r = 0;
    while (((int64_t)1 << r) < v) ++r;
    return r;
}

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 256;
    return cus;
}

// Mean time (ms) of forward + adjoint (fwd_only: the forward) of an uploaded
// candidate, on buffers and a workspace of its own; FLT_OK or an error code.
int time_candidate(flt_plan* p, bool fwd_only, double* ms)
{
    const HostPlan& hp = p->hp;
    const size_t S = hp.elem_bytes();
    void *ws = nullptr, *c = nullptr, *f = nullptr, *g = nullptr, *h = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&ws, hp.ws_bytes);
    if (e == hipSuccess) e = hipMalloc(&c, (size_t)hp.N * S);
    if (e == hipSuccess) e = hipMalloc(&h, (size_t)hp.N * S);
    if (e == hipSuccess) e = hipMalloc(&f, (size_t)hp.M * S);
    if (e == hipSuccess) e = hipMalloc(&g, (size_t)hp.M * S);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemsetAsync(c, 0, (size_t)hp.N * S, st);
    if (e == hipSuccess) e = hipMemsetAsync(g, 0, (size_t)hp.M * S, st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        p->ws = (char*)ws;
        p->ws_bytes = hp.ws_bytes;
        const int reps = 5;
        e = enqueue(p, 0, c, f, nullptr, st);                       // warm-up
        if (e == hipSuccess && !fwd_only) e = enqueue(p, 2, g, h, nullptr, st);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            e = enqueue(p, 0, c, f, nullptr, st);
            if (e == hipSuccess && !fwd_only) e = enqueue(p, 2, g, h, nullptr, st);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        *ms = t / reps;
        p->ws = nullptr;
        p->ws_bytes = 0;
    }
    if (st) (void)hipStreamSynchronize(st);
    for (void* q : {ws, c, f, g, h})
        if (q) (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    return e == hipSuccess ? FLT_OK : hip_fail(e);
}

// Index of the first candidate that no later one beats by 2% (the timing noise
// of five calls, timed twice, is about 1%).
size_t pick(const std::vector<double>& ms)
{
    double best = 1e300;
    size_t at = 0;
    for (size_t i = 0; i < ms.size(); ++i)
        if (ms[i] < 0.98 * best) {
            best = ms[i];
            at = i;
        }
    return at;
}
}  // namespace

// Times the uploaded candidates twice (the first pass a warm-up) and returns
// the pick, or a negative error code.
static int time_and_pick(std::vector<flt_plan*>& cands, bool fwd_only, size_t* at)
{
    std::vector<double> ms(cands.size(), 0.0);
    int rc = FLT_OK;
    for (int pass = 0; pass < 2 && rc == FLT_OK; ++pass)
        for (size_t i = 0; i < cands.size() && rc == FLT_OK; ++i) rc = time_candidate(cands[i], fwd_only, &ms[i]);
    if (rc == FLT_OK) *at = pick(ms);
    return rc;
}

template <class Build> static int tuned_shape(uint32_t flags, Build&& build, Tuned* out)
{
    HostPlan probe;
    int rc = build(probe, PlanShape());
    if (rc != FLT_OK) return rc;
    const bool fwd_only = (flags & FLT_FLAG_TUNE_FORWARD) != 0;
    const TuneKey key{fwd_only ? 1 : 0, probe.dtype, probe.eps, (int64_t)probe.inst.size(), size_class(probe.N),
                      size_class(probe.M)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            *out = it->second;
            return FLT_OK;
        }
    }
    const int cus = device_cus();
    std::vector<flt_plan*> cands;
    auto release_all = [&]() {
        for (flt_plan* c : cands) release(c);
        cands.clear();
    };
    // a candidate plan of the given shape (or of a host plan already built for
    // it), uploaded (nullptr and rc set on failure)
    auto make = [&](const PlanShape& sh, HostPlan* built = nullptr) -> flt_plan* {
        flt_plan* cand = new (std::nothrow) flt_plan();
        if (!cand) {
            rc = FLT_ENOMEM;
            return nullptr;
        }
        if (built) cand->hp = std::move(*built);
        else rc = build(cand->hp, sh);
        if (rc == FLT_OK) {
            cand->host_only = false;
            rc = upload(cand);
        }
        if (rc != FLT_OK) {
            release(cand);
            return nullptr;
        }
        cand->lists.persist_blocks = 2 * cus;
        return cand;
    };
    Tuned best;
    size_t at = 0;
    // 1. the band policy: distinct sets of direct bands only
    {
        std::vector<std::vector<int>> seen;
        std::vector<double> scales;
        // the host plans of every factor, built on host threads at once for a
        // single instance (each is independent of the others; no exception may
        // leave a thread); a batch's planner already runs its members on threads
        constexpr int NS = (int)(sizeof(TUNE_SCALES) / sizeof(TUNE_SCALES[0]));
        std::vector<HostPlan> hps(NS);
        std::vector<int> rcs(NS, FLT_OK);
        auto build_one_scale = [&](int i) {
            try {
                PlanShape sh;
                sh.direct_scale = TUNE_SCALES[i];
                rcs[i] = build(hps[i], sh);
            } catch (const std::exception&) {
                rcs[i] = FLT_ENOMEM;
            }
        };
        {
            std::vector<std::thread> pool;
            int i = 0;
            if (probe.inst.size() == 1) {
                try {
                    for (; i < NS; ++i) pool.emplace_back(build_one_scale, i);
                } catch (const std::system_error&) {   // fewer threads: the rest here
                }
            }
            for (; i < NS; ++i) build_one_scale(i);
            for (std::thread& t : pool) t.join();
        }
        for (int si = 0; si < NS; ++si) {
            const double sc = TUNE_SCALES[si];
            HostPlan& hp = hps[si];
            PlanShape sh;
            sh.direct_scale = sc;
            rc = rcs[si];
            if (rc != FLT_OK) break;
            std::vector<int> sig;
            for (const BandDesc& B : hp.bands) sig.push_back(B.direct);
            bool dup = false;
            for (const auto& v : seen) dup = dup || v == sig;
            if (dup) continue;
            seen.push_back(sig);
            flt_plan* cand = make(sh, &hp);
            if (!cand) break;
            cands.push_back(cand);
            scales.push_back(sc);
        }
        if (rc == FLT_OK) rc = time_and_pick(cands, fwd_only, &at);
        release_all();
        if (rc != FLT_OK) return rc;
        best.shape.direct_scale = scales[at];
    }
    // 2. workgroups per compute unit of the persistent pass B
    {
        flt_plan* cand = make(best.shape);
        if (!cand) return rc;
        std::vector<double> ms;
        for (int b : TUNE_BLOCKS) {
            cand->lists.persist_blocks = b * cus;
            double t = 0;
            for (int pass = 0; pass < 2 && rc == FLT_OK; ++pass) rc = time_candidate(cand, fwd_only, &t);
            if (rc != FLT_OK) break;
            ms.push_back(t);
        }
        release(cand);
        if (rc != FLT_OK) return rc;
        best.passB_per_cu = TUNE_BLOCKS[pick(ms)];
    }
    *out = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
    return FLT_OK;
}

template <class Build> static int create(flt_plan** out, uint32_t flags, Build&& build)
{
    if (!out) return FLT_EINVAL;
    *out = nullptr;
    if (flags & ~KNOWN_FLAGS) return FLT_EINVAL;
    Tuned tuned;
    const bool tune = (flags & FLT_FLAG_AUTOTUNE) && !(flags & (FLT_FLAG_HOST_ONLY | FLT_FLAG_NFFT_ONLY));
    if (tune) {
        int rc;
        try {
            rc = tuned_shape(flags, build, &tuned);
        } catch (const std::bad_alloc&) {
            rc = FLT_ENOMEM;
        }
        if (rc != FLT_OK) return rc;
    }
    flt_plan* p = new (std::nothrow) flt_plan();
    if (!p) return FLT_ENOMEM;
    int rc;
    try {
        rc = build(p->hp, tuned.shape);
    } catch (const std::bad_alloc&) {
        rc = FLT_ENOMEM;
    }
    if (rc == FLT_OK && !(flags & FLT_FLAG_HOST_ONLY)) {
        p->host_only = false;
        rc = upload(p);
        if (rc == FLT_OK) {
            const int cus = device_cus();
            p->lists.persist_blocks = tuned.passB_per_cu * cus;
        }
        if (rc == FLT_OK && (flags & FLT_FLAG_GRAPH)) {
            const hipError_t e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
            if (e != hipSuccess) rc = hip_fail(e);
        }
    }
    if (rc != FLT_OK) {
        release(p);
        return rc;
    }
    *out = p;
    return FLT_OK;
}

static void release(flt_plan* p)
{
    if (!p) return;
    for (GraphSlot& g : p->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (p->capture) (void)hipStreamDestroy(p->capture);
    if (p->dev) (void)hipFree(p->dev);
    delete p;
}

// The real-exponent plan's inner batched integer plan: as
// flt_plan_create_batch, with eps allowed below the dtype's floor.
static int create_inner_batch(flt_plan** out, int32_t count, const int64_t* N, const int64_t* M, const double* z,
                              double eps, int dtype)
{
    return create(out, 0, [&](HostPlan& hp, const PlanShape& shape) {
        return build_batch_plan(hp, count, N, M, z, eps, dtype, PLAN_FLAG_NO_FLOOR, shape);
    });
}

extern "C" {

int flt_plan_create(flt_plan** out, int64_t N, int64_t M, const double* z, double eps, int dtype, uint32_t flags)
{
    return create(out, flags, [&](HostPlan& hp, const PlanShape& shape) {
        return build_host_plan(hp, N, M, z, eps, dtype, flags, shape);
    });
}

int flt_plan_create_policy(flt_plan** out, int64_t N, int64_t M, const double* z, double eps, int dtype,
                           uint32_t flags, double direct_scale)
{
    if (out) *out = nullptr;
    if ((flags & FLT_FLAG_AUTOTUNE) || !(direct_scale >= 0.0 && direct_scale <= 1.0e300)) return FLT_EINVAL;   // NaN and inf fail too
    return create(out, flags, [&](HostPlan& hp, const PlanShape& shape) {
        PlanShape sh = shape;   // the default shape (no tuning), with the given factor
        sh.direct_scale = direct_scale;
        return build_host_plan(hp, N, M, z, eps, dtype, flags, sh);
    });
}

int flt_plan_create_batch(flt_plan** out, int32_t count, const int64_t* N, const int64_t* M, const double* z,
                          double eps, int dtype, uint32_t flags)
{
    return create(out, flags, [&](HostPlan& hp, const PlanShape& shape) {
        return build_batch_plan(hp, count, N, M, z, eps, dtype, flags, shape);
    });
}

void flt_plan_destroy(flt_plan* p) { release(p); }

int flt_plan_info(const flt_plan* p, flt_info* o)
{
    if (!p || !o) return FLT_EINVAL;
    const HostPlan& hp = p->hp;
    memset(o, 0, sizeof(*o));
    o->N = hp.N;
    o->M = hp.M;
    o->dtype = hp.dtype;
    o->q = hp.q;
    o->D = hp.D;
    o->n_xi = hp.n_xi;
    o->mw = hp.mw;
    int nb = 0;
    for (const BandDesc& B : hp.bands) nb += B.q > 0;
    o->num_bands = nb;
    o->eps = hp.eps;
    o->eps_K = hp.eps_K;
    o->eps_A = hp.eps_A;
    o->y1 = hp.y1;
    o->nodes_z0 = hp.nodes_z0;
    o->workspace_bytes = hp.ws_bytes;
    o->bytes_forward = hp.bytes_forward;
    o->flops_forward = hp.flops_forward;
    o->direct_scale = hp.direct_scale;
    o->forward_scratch_bytes = hp.fwd_ws_bytes;
    o->passB_blocks = p->lists.persist_blocks;
    return FLT_OK;
}

int flt_plan_band(const flt_plan* p, int32_t i, flt_band_info* o)
{
    if (!p || !o) return FLT_EINVAL;
    int seen = 0;
    for (size_t b = 0; b < p->hp.bands.size(); ++b) {
        const BandDesc& B = p->hp.bands[b];
        if (B.q == 0) continue;
        if (seen++ != i) continue;
        memset(o, 0, sizeof(*o));
        o->m = p->hp.band_m[b];
        o->q = B.q;
        o->ell_lo = B.ell_lo;
        o->ell_hi = B.ell_hi;
        o->K = B.k0 * 2 > 0 ? B.k0 * 2 : 1;
        o->n = (int64_t)1 << B.log2n;
        o->k0 = B.k0;
        o->nodes = B.node_count;
        o->passes = B.direct ? 0 : (B.log2n2 > 0 ? 2 : 1);
        o->direct = B.direct;
        o->cells = B.direct ? 0 : B.cells;
        return FLT_OK;
    }
    return FLT_EINVAL;
}

int flt_plan_node_bands(const flt_plan* p, int32_t* out)
{
    if (!p || !out) return FLT_EINVAL;
    memcpy(out, p->hp.node_band.data(), p->hp.node_band.size() * sizeof(int32_t));
    return FLT_OK;
}

int flt_plan_workspace_size(const flt_plan* p, size_t* bytes)
{
    if (!p || !bytes) return FLT_EINVAL;
    *bytes = p->hp.ws_bytes;
    return FLT_OK;
}

int flt_plan_set_workspace(flt_plan* p, void* dev, size_t bytes)
{
    if (!p || !dev) return FLT_EINVAL;
    if (p->host_only) return FLT_ESTATE;
    if (bytes < p->hp.ws_bytes || ((uintptr_t)dev & 255)) return FLT_ENOWORKSPACE;
    p->ws = (char*)dev;
    p->ws_bytes = bytes;
    return FLT_OK;
}

static WsLayout layout(const flt_plan* p)
{
    const HostPlan& hp = p->hp;
    WsLayout W;
    W.ws = p->ws;
    W.off_grid = hp.off_grid;
    W.off_scratch = hp.off_scratch;
    W.off_acc = hp.off_acc;
    W.off_U = hp.off_U;
    W.off_phi = hp.off_phi;
    W.off_l0 = hp.off_l0;
    W.off_dacc = hp.off_dacc;
    W.off_base = hp.off_base;
    W.qs = hp.qs;
    W.N = hp.N;
    W.M = hp.M;
    W.grid_elems = hp.grid_elems;
    return W;
}

static int check_call(const flt_plan* p, const void* a, const void* b)
{
    if (!p || !a || !b) return FLT_EINVAL;
    if (p->host_only) return FLT_ESTATE;
    if (!p->ws) return FLT_ENOWORKSPACE;
    return FLT_OK;
}

// op 0: forward, 1: derivative, 2: adjoint, 3: forward (out) and derivative
// (out2) in one pass; enqueues the launch sequence on st.
static hipError_t enqueue(flt_plan* p, int op, const void* in, void* out, void* out2, hipStream_t st)
{
    const WsLayout W = layout(p);
    if (op == 2)
        return p->hp.dtype == FLT_C64 ? launch_adjoint<float>(p->lists, p->pv32, W, in, out, st)
                                      : launch_adjoint<double>(p->lists, p->pv64, W, in, out, st);
    void* f2 = op == 3 ? out2 : nullptr;
    const int deriv = op == 1;
    return p->hp.dtype == FLT_C64 ? launch_forward<float>(p->lists, p->pv32, W, in, out, f2, deriv, st)
                                  : launch_forward<double>(p->lists, p->pv64, W, in, out, f2, deriv, st);
}

// FLT_FLAG_GRAPH: replay the captured sequence when the buffers match the last
// capture of this operation, else capture anew on the plan's own stream (the
// kernels do not run during capture) and launch the graph on the caller's.
static hipError_t run_graph(flt_plan* p, int op, const void* in, void* out, void* out2, hipStream_t st)
{
    GraphSlot& g = p->graphs[op];
    if (!g.exec || g.in != in || g.out != out || g.out2 != out2 || g.ws != p->ws) {
        if (g.exec) {
            (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
        hipError_t e = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        const hipError_t le = enqueue(p, op, in, out, out2, p->capture);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(p->capture, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return le != hipSuccess ? le : e;
        }
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.exec = nullptr;
            return e;
        }
        g.in = in;
        g.out = out;
        g.out2 = out2;
        g.ws = p->ws;
    }
    return hipGraphLaunch(g.exec, st);
}

static int run(flt_plan* p, int op, const void* in, void* out, void* stream, void* out2 = nullptr)
{
    const int rc = check_call(p, in, out);
    if (rc != FLT_OK) return rc;
    if (op == 3 && (!out2 || out2 == out)) return FLT_EINVAL;
    const hipError_t e = p->capture ? run_graph(p, op, in, out, out2, (hipStream_t)stream)
                                    : enqueue(p, op, in, out, out2, (hipStream_t)stream);
    return e == hipSuccess ? FLT_OK : hip_fail(e);
}

int flt_forward(flt_plan* p, const void* c, void* f, void* stream) { return run(p, 0, c, f, stream); }

int flt_derivative(flt_plan* p, const void* c, void* fp, void* stream) { return run(p, 1, c, fp, stream); }

int flt_forward_noalloc(flt_plan* p, const void* c, void* f, void* stream)
{
    if (!p || !c || !f) return FLT_EINVAL;
    if (p->host_only) return FLT_ESTATE;
    const HostPlan& hp = p->hp;
    if (hp.fwd_ws_bytes > FLT_NOALLOC_MAX_BYTES) return FLT_ERANGE;
    char* base = nullptr;
    hipError_t e = noalloc_scratch_address(p->device, &base);
    if (e != hipSuccess) return hip_fail(e);
    // the forward's sections packed (one column set per band)
    WsLayout W;
    W.ws = base;
    W.off_grid = 0;
    W.off_scratch = hp.fwd_off_scratch;
    W.off_dacc = hp.fwd_off_dacc;
    W.off_base = hp.fwd_off_base;
    W.qs = hp.qs;
    W.N = hp.N;
    W.M = hp.M;
    W.grid_elems = hp.grid_elems;
    const hipStream_t st = (hipStream_t)stream;
    e = hp.dtype == FLT_C64 ? launch_forward<float>(p->lists, p->pv32, W, c, f, nullptr, 0, st)
                            : launch_forward<double>(p->lists, p->pv64, W, c, f, nullptr, 0, st);
    return e == hipSuccess ? FLT_OK : hip_fail(e);
}

int flt_adjoint(flt_plan* p, const void* g, void* c_out, void* stream) { return run(p, 2, g, c_out, stream); }

int flt_forward_derivative(flt_plan* p, const void* c, void* f, void* fp, void* stream)
{
    return run(p, 3, c, f, stream, fp);
}

// One measured call: ne HIP events recorded between the stages of the
// operation's launch sequence on the caller's stream, waited for, and the
// ne - 1 stage durations written to stage_ms.
static int profile(flt_plan* p, int op, const void* in, void* out, void* stream, double* stage_ms, int ne)
{
    int rc = check_call(p, in, out);
    if (rc != FLT_OK) return rc;
    if (!stage_ms) return FLT_EINVAL;
    const HostPlan& hp = p->hp;
    hipEvent_t ev[9] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i < ne && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    const WsLayout W = layout(p);
    const hipStream_t st = (hipStream_t)stream;
    if (e == hipSuccess) {
        if (op == 2)
            e = hp.dtype == FLT_C64 ? launch_adjoint<float>(p->lists, p->pv32, W, in, out, st, ev)
                                    : launch_adjoint<double>(p->lists, p->pv64, W, in, out, st, ev);
        else
            e = hp.dtype == FLT_C64 ? launch_forward<float>(p->lists, p->pv32, W, in, out, nullptr, 0, st, ev)
                                    : launch_forward<double>(p->lists, p->pv64, W, in, out, nullptr, 0, st, ev);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[ne - 1]);
    for (int i = 0; i + 1 < ne && e == hipSuccess; ++i) {
        float ms = 0;
        e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        stage_ms[i] = ms;
    }
    for (int i = 0; i < ne; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    return e == hipSuccess ? FLT_OK : hip_fail(e);
}

int flt_profile_forward(flt_plan* p, const void* c, void* f, void* stream, double* stage_ms)
{
    return profile(p, 0, c, f, stream, stage_ms, 6);
}

int flt_profile_adjoint(flt_plan* p, const void* g, void* c_out, void* stream, double* stage_ms)
{
    return profile(p, 2, g, c_out, stream, stage_ms, 9);
}

const char* flt_strerror(int code)
{
    switch (code) {
        case FLT_OK: return "ok";
        case FLT_EINVAL: return "invalid argument";
        case FLT_EDOMAIN: return "argument outside the method's domain (eps not in (0,1), Im z < 0, NaN or inf)";
        case FLT_EPRECISION: return "accuracy below what the dtype can deliver";
        case FLT_ENOWORKSPACE: return "workspace missing or too small";
        case FLT_EHIP: return "HIP runtime error";
        case FLT_ESTATE: return "plan has no device state (host-only plan)";
        case FLT_ENOMEM: return "host allocation failed";
        case FLT_ERANGE: return "size beyond the supported range";
        default: return "unknown error";
    }
}

int flt_last_hip_error(void) { return g_last_hip; }

}  // extern "C"

// ---------------------------------------------------------------------------
// The discrete Laplace transform (Sect. 3, Algorithm 1)
// ---------------------------------------------------------------------------
struct flt_laplace_plan {
    LapHost hp;
    bool host_only = true;
    void* dev = nullptr;      // tables, work items and the accumulator, one allocation
    LapView V{};
    const LapItem* items = nullptr;
};

extern "C" {

int flt_laplace_plan_create(flt_laplace_plan** out, int64_t N, const double* xi, int64_t M, const double* y,
                            double eps, int dtype, uint32_t flags)
{
    return flt_laplace_plan_create_kernel(out, FLT_KERNEL_EXP, N, xi, M, y, eps, dtype, flags);
}

int flt_laplace_plan_create_kernel(flt_laplace_plan** out, int32_t kernel, int64_t N, const double* xi, int64_t M,
                                   const double* y, double eps, int dtype, uint32_t flags)
{
    if (!out) return FLT_EINVAL;
    *out = nullptr;
    if (kernel != FLT_KERNEL_EXP && kernel != FLT_KERNEL_BESSEL_K_HALF) return FLT_EINVAL;
    if (flags & ~FLT_FLAG_HOST_ONLY) return FLT_EINVAL;
    flt_laplace_plan* p = new (std::nothrow) flt_laplace_plan();
    if (!p) return FLT_ENOMEM;
    int rc;
    try {
        rc = build_laplace_plan(p->hp, N, xi, M, y, eps, dtype, kernel);
    } catch (const std::bad_alloc&) {
        rc = FLT_ENOMEM;
    }
    if (rc != FLT_OK) {
        delete p;
        return rc;
    }
    if (!(flags & FLT_FLAG_HOST_ONLY)) {
        const LapHost& hp = p->hp;
        Packer pk;
        const size_t o_xs = pk.add(hp.xs.data(), hp.xs.size() * sizeof(double));
        const size_t o_kp = pk.add(hp.kperm.data(), hp.kperm.size() * sizeof(int32_t));
        const size_t o_bc = pk.add(hp.bcw.data(), hp.bcw.size() * sizeof(double));
        const size_t o_yc = pk.add(hp.ycw.data(), hp.ycw.size() * sizeof(double));
        const size_t o_lm = pk.add(hp.lm.data(), hp.lm.size() * sizeof(int32_t));
        const size_t o_Lm = pk.add(hp.Lm.data(), hp.Lm.size() * sizeof(int32_t));
        const size_t o_ko = pk.add(hp.koff.data(), hp.koff.size() * sizeof(int64_t));
        const size_t o_K = pk.add(hp.K.data(), hp.K.size() * sizeof(double));
        const size_t o_y = pk.add(hp.y.data(), hp.y.size() * sizeof(double));
        const size_t o_bd = pk.add(hp.band.data(), hp.band.size() * sizeof(int32_t));
        const size_t o_it = pk.add(hp.items.data(), hp.items.size() * sizeof(LapItem));
        const size_t o_bi = pk.add(hp.bitem.data(), hp.bitem.size() * sizeof(int32_t));
        std::vector<double> zeros((size_t)lap_acc_doubles(hp.L, hp.q) + hp.items.size() * 2 * hp.q, 0.0);
        const size_t o_acc = pk.add(zeros.data(), zeros.size() * sizeof(double));
        hipError_t e = hipMalloc(&p->dev, pk.buf.size());
        if (e == hipSuccess) e = hipMemcpy(p->dev, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (p->dev) (void)hipFree(p->dev);
            delete p;
            return hip_fail(e);
        }
        char* b = (char*)p->dev;
        LapView& V = p->V;
        V.q = hp.q;
        V.L = hp.L;
        V.kernel = hp.kernel;
        V.near0 = hp.near0;
        V.nnear = hp.nnear;
        V.N = hp.N;
        V.xs = (const double*)(b + o_xs);
        V.kperm = (const int32_t*)(b + o_kp);
        V.bcw = (const double*)(b + o_bc);
        V.ycw = (const double*)(b + o_yc);
        V.lm = (const int32_t*)(b + o_lm);
        V.Lm = (const int32_t*)(b + o_Lm);
        V.koff = (const int64_t*)(b + o_ko);
        V.K = (const double*)(b + o_K);
        V.y = (const double*)(b + o_y);
        V.band = (const int32_t*)(b + o_bd);
        V.bitem = (const int32_t*)(b + o_bi);
        V.nitems = (int32_t)hp.items.size();
        V.acc = (double*)(b + o_acc);
        V.part = V.acc + lap_acc_doubles(hp.L, hp.q);
        p->items = (const LapItem*)(b + o_it);
        p->host_only = false;
    }
    *out = p;
    return FLT_OK;
}

int flt_laplace_plan_info(const flt_laplace_plan* p, flt_laplace_info* o)
{
    if (!p || !o) return FLT_EINVAL;
    memset(o, 0, sizeof(*o));
    o->N = p->hp.N;
    o->M = p->hp.M;
    o->dtype = p->hp.dtype;
    o->q = p->hp.q;
    o->levels = p->hp.L;
    o->kernel = p->hp.kernel;
    o->eps = p->hp.eps;
    o->y1 = p->hp.y1;
    o->xi1 = p->hp.xi1;
    return FLT_OK;
}

int flt_laplace_forward(flt_laplace_plan* p, const void* fhat, void* f, void* stream)
{
    if (!p || !fhat || !f) return FLT_EINVAL;
    if (p->host_only) return FLT_ESTATE;
    const hipStream_t st = (hipStream_t)stream;
    const int ni = (int)p->hp.items.size();
    const hipError_t e = p->hp.dtype == FLT_C64 ? launch_laplace<float>(p->V, p->items, ni, p->hp.M, fhat, f, st)
                                                : launch_laplace<double>(p->V, p->items, ni, p->hp.M, fhat, f, st);
    return e == hipSuccess ? FLT_OK : hip_fail(e);
}

void flt_laplace_plan_destroy(flt_laplace_plan* p)
{
    if (!p) return;
    if (p->dev) (void)hipFree(p->dev);
    delete p;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Real exponents (eq. 4.1 with real xi_k; the transposed g(xi) of Sect. 4)
// ---------------------------------------------------------------------------
struct flt_xi_plan {
    XiHost hp;
    bool host_only = true;
    void* dev = nullptr;      // tables and work items
    void* buf = nullptr;      // inner coefficients, inner node values, FP64 accumulator
    void* ws = nullptr;       // the inner plan's workspace
    flt_plan* inner = nullptr;
    XiView<float> v32{};
    XiView<double> v64{};
    const XiItem* spread = nullptr;
    const XiItem* gather = nullptr;
    const NodeItem* nodes = nullptr;
    char* cin = nullptr;
    char* hout = nullptr;
    double* hacc = nullptr;
    int qmax = 1;
};

static void xi_release(flt_xi_plan* p)
{
    if (!p) return;
    if (p->inner) release(p->inner);
    if (p->ws) (void)hipFree(p->ws);
    if (p->buf) (void)hipFree(p->buf);
    if (p->dev) (void)hipFree(p->dev);
    delete p;
}

template <typename T>
static XiView<T> xi_view(const XiHost& hp, char* b, size_t o_bands, size_t o_coef, size_t o_yc, size_t o_xi,
                         size_t o_xp, size_t o_xpos, size_t o_ny, size_t o_perm)
{
    XiView<T> v;
    v.bands = (const XiBand*)(b + o_bands);
    v.coef = (const T*)(b + o_coef);
    v.ycheb = (const double*)(b + o_yc);
    v.xi = (const double*)(b + o_xi);
    v.xi_perm = (const int32_t*)(b + o_xp);
    v.xp = (const double*)(b + o_xpos);
    v.ny = (const double*)(b + o_ny);
    v.perm = (const int32_t*)(b + o_perm);
    v.mw1 = hp.mw1;
    return v;
}

static int xi_upload(flt_xi_plan* p)
{
    XiHost& hp = p->hp;
    const HostPlan& op = hp.outer;
    const bool f32 = hp.dtype == FLT_C64;
    int rc = create_inner_batch(&p->inner, (int32_t)hp.in_N.size(), hp.in_N.data(), hp.in_M.data(), hp.in_z.data(),
                                hp.eps_in, hp.dtype);
    if (rc != FLT_OK) return rc;
    std::vector<double>().swap(hp.in_z);   // the inner plan holds its copy
    size_t wsb = 0;
    rc = flt_plan_workspace_size(p->inner, &wsb);
    if (rc != FLT_OK) return rc;
    hipError_t e = hipMalloc(&p->ws, wsb ? wsb : 256);
    if (e != hipSuccess) return hip_fail(e);
    rc = flt_plan_set_workspace(p->inner, p->ws, wsb);
    if (rc != FLT_OK) return rc;

    Packer pk;
    const size_t o_bands = pk.add(hp.bands.data(), hp.bands.size() * sizeof(XiBand));
    const size_t o_sp = pk.add(hp.spread.data(), hp.spread.size() * sizeof(XiItem));
    const size_t o_ga = pk.add(hp.gather.data(), hp.gather.size() * sizeof(XiItem));
    const size_t o_nd = pk.add(hp.nodes.data(), hp.nodes.size() * sizeof(NodeItem));
    const size_t o_coef = f32 ? pk.add_cast<float>(op.coef) : pk.add_cast<double>(op.coef);
    const size_t o_yc = pk.add(op.ycheb.data(), op.ycheb.size() * sizeof(double));
    const size_t o_xi = pk.add(hp.xi.data(), hp.xi.size() * sizeof(double));
    const size_t o_xp = pk.add(hp.xi_perm.data(), hp.xi_perm.size() * sizeof(int32_t));
    const size_t o_xpos = pk.add(hp.xp.data(), hp.xp.size() * sizeof(double));
    const size_t o_ny = pk.add(op.ny.data(), op.ny.size() * sizeof(double));
    const size_t o_perm = pk.add(op.perm.data(), op.perm.size() * sizeof(int32_t));
    e = hipMalloc(&p->dev, pk.buf.size());
    if (e == hipSuccess) e = hipMemcpy(p->dev, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    char* b = (char*)p->dev;
    p->v32 = xi_view<float>(hp, b, o_bands, o_coef, o_yc, o_xi, o_xp, o_xpos, o_ny, o_perm);
    p->v64 = xi_view<double>(hp, b, o_bands, o_coef, o_yc, o_xi, o_xp, o_xpos, o_ny, o_perm);
    p->spread = (const XiItem*)(b + o_sp);
    p->gather = (const XiItem*)(b + o_ga);
    p->nodes = (const NodeItem*)(b + o_nd);
    for (const XiBand& X : hp.bands) p->qmax = std::max(p->qmax, (int)X.q);

    const size_t S = f32 ? 8 : 16;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t b_cin = al(std::max<int64_t>(hp.cin_elems, 1) * S);
    const size_t b_hout = al(std::max<int64_t>(hp.hout_elems, 1) * S);
    e = hipMalloc(&p->buf, b_cin + b_hout + (size_t)hp.N * 16);
    if (e != hipSuccess) return hip_fail(e);
    p->cin = (char*)p->buf;
    p->hout = p->cin + b_cin;
    p->hacc = (double*)(p->hout + b_hout);
    return FLT_OK;
}

extern "C" {

int flt_xi_plan_create(flt_xi_plan** out, int64_t N, const double* xi, int64_t M, const double* z, double eps,
                       int dtype, uint32_t flags)
{
    if (!out) return FLT_EINVAL;
    *out = nullptr;
    if (flags & ~FLT_FLAG_HOST_ONLY) return FLT_EINVAL;
    flt_xi_plan* p = new (std::nothrow) flt_xi_plan();
    if (!p) return FLT_ENOMEM;
    int rc;
    try {
        rc = build_xi_plan(p->hp, N, xi, M, z, eps, dtype);
        if (rc == FLT_OK && !(flags & FLT_FLAG_HOST_ONLY)) {
            rc = xi_upload(p);
            if (rc == FLT_OK) p->host_only = false;
        }
    } catch (const std::bad_alloc&) {
        rc = FLT_ENOMEM;
    }
    if (rc != FLT_OK) {
        xi_release(p);
        return rc;
    }
    *out = p;
    return FLT_OK;
}

int flt_xi_plan_info(const flt_xi_plan* p, flt_xi_info* o)
{
    if (!p || !o) return FLT_EINVAL;
    const XiHost& hp = p->hp;
    memset(o, 0, sizeof(*o));
    o->N = hp.N;
    o->M = hp.M;
    o->dtype = hp.dtype;
    o->q = hp.outer.q;
    o->mw1 = hp.mw1;
    int nb = 0;
    for (const XiBand& X : hp.bands) nb += X.q > 0;
    o->num_bands = nb;
    o->inner_instances = (int32_t)hp.in_N.size();
    o->eps = hp.eps;
    o->eps_w = hp.eps_w;
    o->eps_in = hp.eps_in;
    o->sigma_min = hp.sig_min;
    o->amp = hp.amp;
    o->inner_coefficients = hp.cin_elems;
    o->inner_nodes = hp.hout_elems;
    if (p->inner) {
        o->inner_mw = p->inner->hp.mw;
        o->inner_workspace_bytes = p->inner->hp.ws_bytes;
    }
    return FLT_OK;
}

static int xi_run(flt_xi_plan* p, int op, const void* in, void* out, void* stream)
{
    if (!p || !in || !out) return FLT_EINVAL;
    if (p->host_only) return FLT_ESTATE;
    const hipStream_t st = (hipStream_t)stream;
    const XiHost& hp = p->hp;
    const bool f32 = hp.dtype == FLT_C64;
    hipError_t e;
    int rc;
    if (op == 0) {
        e = f32 ? launch_xi_spread<float>(p->v32, p->qmax, p->spread, (int)hp.spread.size(), in, p->cin, st)
                : launch_xi_spread<double>(p->v64, p->qmax, p->spread, (int)hp.spread.size(), in, p->cin, st);
        if (e != hipSuccess) return hip_fail(e);
        rc = flt_forward(p->inner, p->cin, p->hout, stream);
        if (rc != FLT_OK) return rc;
        e = f32 ? launch_xi_combine<float>(p->v32, p->nodes, (int)hp.nodes.size(), p->hout, out, st)
                : launch_xi_combine<double>(p->v64, p->nodes, (int)hp.nodes.size(), p->hout, out, st);
        return e == hipSuccess ? FLT_OK : hip_fail(e);
    }
    const int conj = op == 2;
    e = f32 ? launch_xi_prep<float>(p->v32, p->nodes, (int)hp.nodes.size(), in, conj, p->hout, st)
            : launch_xi_prep<double>(p->v64, p->nodes, (int)hp.nodes.size(), in, conj, p->hout, st);
    if (e != hipSuccess) return hip_fail(e);
    rc = flt_adjoint(p->inner, p->hout, p->cin, stream);
    if (rc != FLT_OK) return rc;
    e = f32 ? launch_xi_gather<float>(p->v32, p->qmax, p->gather, (int)hp.gather.size(), p->cin, p->hacc, hp.N, conj,
                                      out, st)
            : launch_xi_gather<double>(p->v64, p->qmax, p->gather, (int)hp.gather.size(), p->cin, p->hacc, hp.N,
                                       conj, out, st);
    return e == hipSuccess ? FLT_OK : hip_fail(e);
}

int flt_xi_forward(flt_xi_plan* p, const void* c, void* f, void* stream) { return xi_run(p, 0, c, f, stream); }
int flt_xi_transposed(flt_xi_plan* p, const void* g, void* h, void* stream) { return xi_run(p, 1, g, h, stream); }
int flt_xi_adjoint(flt_xi_plan* p, const void* g, void* h, void* stream) { return xi_run(p, 2, g, h, stream); }
void flt_xi_plan_destroy(flt_xi_plan* p) { xi_release(p); }

}  // extern "C"
