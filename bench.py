#!/usr/bin/env python3
"""Benchmark of the fast Fourier-Laplace transform on one MI355X.

Workload: N = M = 2^20, c_k complex64 with Re/Im ~ N(0,1); the first M/2 nodes
uniform by area in the annulus 1-1e-3 < |w| <= 1, the rest uniform by area in
the unit disk (seed 3, see paper_1606_03255_amd/inputs.py).

value      node evaluations per second of the FP32 form (eps = 1e-6): M times
           the number of timed forward calls over their wall time, inputs
           resident in HBM, plan built beforehand (plan time reported apart).
fwd_bwd    forward and derivative (f and f' for dL/dz, one fused call) plus the
           adjoint (dL/dc) per step, for the FP32 form and for the plain FP64
           path (eps = 1e-11) on the same inputs; speedup = t(FP64) / t(FP32).
           ms_separate_fp32 times the three calls made one by one.  The same
           step at N = M = 2^18 (nodes in the disk) is fwd_bwd_grad.  Every
           output of a timed step carries its error E against the oracle.
roofline   the dominant kernel's algorithmic bytes per launch over its launch
           duration (HIP events recorded between the launches on the stream
           the kernels run on), against the 8 TB/s HBM peak; for the direct
           sums (ALU-bound) their flops against the FP32 vector peak.  The
           adjoint's dominant stage (roofline_adjoint) and the FP64 path's
           forward (roofline_fp64) are reported the same way; hbm_copy_GBs is
           a measured device-to-device copy rate beside the datasheet peak.
laplace    the discrete Laplace transform (Algorithm 1) at N = M = 2^20: time
           per call, node evals/s, algorithmic bytes against the HBM peak, and
           its error on sampled nodes against the oracle's direct sums; k12:
           the same for Thm 3.3's example kernel K_{1/2}(y xi), its error as a
           fraction of the block-relative bar.
xi         real exponents xi_k uniform in [1, N] (eq. 4.1; the transposed
           g(xi) of Sect. 4) at N = M = 2^20 (--xi-log2n): time per forward
           and transposed call, evals/s, error on sampled nodes / exponents.
direct_scale  the band-policy factor of the forward-tuned plan (the step's own
           plan reports its factor in fwd_bwd).
cpu_baseline  the FP64 direct-sum oracle on a random sample of the nodes, on
           the host cores; the same sample (plus every node of sparsely filled
           bands) gives the error E of both GPU forms against it.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node evals/s at N=M=2^20, err<=1e-6 vs FP64 direct; fwd+bwd speedup vs plain FP64"
HBM_PEAK_GBS = 8000.0
# MI355X FP32 vector peak without packed FP32 instructions (the build turns
# them off): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 78.6
STAGES = ("onepass_fft", "passA_fft", "passB_fft", "gather", "direct")
KERNEL_NAMES = {"onepass_fft": "k_onepass_fwd", "passA_fft": "k_passA_fwd", "passB_fft": "k_passB",
                "gather": "k_gather", "direct": "k_direct_fwd"}
ADJ_STAGES = ("clear_sum_g", "node_prep", "cell_spread", "passB_fft", "passA_fft", "onepass_fft", "direct",
              "finalize")
ADJ_KERNEL_NAMES = {"clear_sum_g": "k_sum_g", "node_prep": "k_adj_prep", "cell_spread": "k_adj_cells",
                    "passB_fft": "k_passB", "passA_fft": "k_passA_adj", "onepass_fft": "k_onepass_adj",
                    "direct": "k_direct_adj", "finalize": "k_finalize_adj"}
DIRECT_NG = 8      # nodes per direct-sum workgroup (c is read once per group)
DIRECT_ANG = 256   # nodes per direct-adjoint workgroup (each adds into every accumulator)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels_impl.h", "kernels.hip", "flt_types.h"):
        with open(os.path.join(ROOT, "paper_1606_03255_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stage_bytes(plan, S):
    """Algorithmic HBM bytes per launch of each forward stage.
    c is read once per band by the stage that generates its columns.  One-pass
    FFT: the band's q grids written once.  Pass A: its output written once.
    Pass B: that output read once and the grid written at the cells some
    node's window reads ("cells" per column).  Gather: those cells (at most
    2 mw per node and column), node records (x, y: 16 B, index 4 B) and the
    result.  Direct bands: c read once per group of DIRECT_NG nodes, node
    records and results."""
    info = plan.info()
    mw = info["mw"]
    b = {k: 0.0 for k in STAGES}
    for band in plan.bands():
        q, n, nodes, cells = band["q"], band["n"], band["nodes"], band["cells"]
        kmax = min(band["K"], plan.N - 1)
        if band["direct"]:
            b["direct"] += -(-nodes // DIRECT_NG) * plan.N * S + nodes * (16 + 4 + S)
            continue
        if band["passes"] == 1:
            b["onepass_fft"] += q * n * S + kmax * S
        else:
            b["passA_fft"] += q * n * S + kmax * S
            b["passB_fft"] += q * n * S + q * cells * S
        b["gather"] += q * min(cells, nodes * 2 * mw) * S
    b["gather"] += plan.M * (16 + 4 + S)
    return b


def stage_fracs(stage_ms, stage_b):
    """Each stage's algorithmic bytes per second as a fraction of the HBM peak
    (stages whose bound is not HBM traffic, such as the direct sums, included
    for reference)."""
    return {k: round(stage_b[k] / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            for k in stage_ms if stage_b.get(k) and stage_ms[k] > 0}


def adjoint_stage_bytes(plan, S):
    """Algorithmic HBM bytes per launch of each adjoint stage.  Clearing: the
    FP64 accumulator (16 N) written, g read once for the k = 0 sum.  Node
    side: per node of an NFFT band its record (x, y, index: 20 B) and g in,
    its q weighted values, 2 mw window values and cell index out.  Cell
    spread: those read once per node, the grid written (every cell of a
    one-pass band, the cells some window touches of a two-pass band).  Pass B:
    those cells read, the pass-A input written in full.  Pass A and the
    one-pass bands: the band's grid read once, and one read-modify-write of
    the FP64 accumulator (32 B) per coefficient of the band's support.  Direct
    bands: the accumulator read and written once per group of DIRECT_ANG
    nodes, plus the node records.  Finalize: the accumulator read, c_out
    written."""
    info = plan.info()
    mw = info["mw"]
    N, M = plan.N, plan.M
    b = {k: 0.0 for k in ADJ_STAGES}
    b["clear_sum_g"] = 16.0 * N + M * S
    b["finalize"] = 16.0 * N + N * S
    for band in plan.bands():
        q, n, nodes, cells = band["q"], band["n"], band["nodes"], band["cells"]
        kmax = min(band["K"], N - 1)
        if band["direct"]:
            b["direct"] += -(-nodes // DIRECT_ANG) * 32.0 * N + nodes * (20 + S)
            continue
        per_node = q * S + 2 * mw * S / 2 + 4
        b["node_prep"] += nodes * (20 + S + per_node)
        b["cell_spread"] += nodes * per_node + q * (n if band["passes"] == 1 else cells) * S
        if band["passes"] == 1:
            b["onepass_fft"] += q * n * S + 32.0 * kmax
        else:
            b["passB_fft"] += q * cells * S + q * n * S
            b["passA_fft"] += q * n * S + 32.0 * kmax
    return b


def roofline_of(stage_ms, sb, names, bound_note=None):
    """The dominant stage's algorithmic bytes over its duration, against HBM."""
    dom = max(stage_ms, key=lambda k: stage_ms[k])
    achieved = sb[dom] / (stage_ms[dom] * 1e-3) / 1e9
    rec = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": names[dom], "bytes_per_launch": sb[dom],
           "ms_per_launch": round(stage_ms[dom], 4)}
    if bound_note:
        rec["note"] = bound_note
    return rec


def time_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return t0.elapsed_time(t1) / steps, wall


def traffic_for(kernel, algorithmic_bytes):
    """HBM traffic per launch from the committed rocprofv3 counter summary, or
    None if it was taken on different kernel sources or on a plan whose
    stage moves different algorithmic bytes (the band policy is tuned at run
    time, so two runs can pick different plans)."""
    path = os.path.join(ROOT, "profiles", "traffic_large_fp32.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    # the default band policy's plan, then any other plan the counters were taken on
    for plan in [rec] + rec.get("plans", []):
        v = plan.get("kernels", {}).get(KERNEL_NAMES[kernel])
        if v is not None and v.get("algorithmic_bytes_per_launch") == algorithmic_bytes:
            return v.get("bytes_per_launch")
    return None


def copy_bandwidth(torch, dev, mib=2048, reps=5):
    """A measured device-to-device copy rate (bytes read + written per second)."""
    src = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    ms, _ = time_steps(torch, lambda: dst.copy_(src), reps, 2)
    del src, dst
    return round(2.0 * (mib << 20) / (ms * 1e-3) / 1e9, 1)


def profile_stages(plan, fn_name, x, reps, names):
    acc = [0.0] * len(names)
    for _ in range(reps):
        _, ms = getattr(plan, fn_name)(x)
        acc = [a + b for a, b in zip(acc, ms)]
    return {k: v / reps for k, v in zip(names, acc)}


def step_leg(torch, dev, w, eps32, eps64, args, tune, log, label, profile):
    """The training step (fused forward + derivative, then the adjoint) in the
    FP32 form and on the plain FP64 path, on plans tuned for that step.
    Returns the record and the outputs (host) for the error check."""
    import numpy as np

    from paper_1606_03255_amd import Plan, inputs
    N, M = w["N"], w["M"]
    c32 = torch.from_numpy(np.ascontiguousarray(w["c"], np.complex64)).to(dev)
    g32 = torch.from_numpy(inputs.adjoint_input(M)).to(dev)
    steps = max(3, args.steps // 2)
    out = {}
    rec = {"N": N, "M": M, "eps_fp32": eps32, "eps_fp64": eps64}
    for form, eps, tdt in (("fp32", eps32, torch.complex64), ("fp64", eps64, torch.complex128)):
        t = time.perf_counter()
        p = Plan(N, w["z"], eps, tdt, device=dev, autotune=tune)     # tuned on forward + adjoint
        rec["plan_ms_" + form] = round((time.perf_counter() - t) * 1e3, 1)
        c = c32.to(tdt)
        g = g32.to(tdt)
        f = torch.empty(M, dtype=tdt, device=dev)
        fp = torch.empty_like(f)
        h = torch.empty(N, dtype=tdt, device=dev)

        def step():
            p.forward_derivative(c, out=f, out_prime=fp)
            p.adjoint(g, out=h)
        ms, _ = time_steps(torch, step, steps, 1)
        rec["ms_" + form] = round(ms, 4)
        rec["direct_scale_" + form] = p.info()["direct_scale"]
        out[form] = {"f": f.cpu().numpy(), "fp": fp.cpu().numpy(), "h": h.cpu().numpy(),
                     "bands": p.node_bands()}
        if form == "fp32":
            def step_sep():
                p.forward(c, out=f)
                p.adjoint(g, out=h)
                p.derivative(c, out=fp)
            rec["ms_separate_fp32"] = round(time_steps(torch, step_sep, steps, 1)[0], 4)
        if profile:
            reps = max(3, min(args.steps, 10))
            sa = profile_stages(p, "profile_adjoint", g, reps, ADJ_STAGES)
            rec["adjoint_stages_ms_" + form] = {k: round(v, 4) for k, v in sa.items()}
            S = 8 if form == "fp32" else 16
            sab = adjoint_stage_bytes(p, S)
            rec["adjoint_stage_bytes_" + form] = sab
            rec["adjoint_stage_frac_hbm_" + form] = stage_fracs(sa, sab)
            rec["roofline_adjoint_" + form] = roofline_of(sa, sab, ADJ_KERNEL_NAMES)
            if form == "fp64":
                rec["ms_fp64_forward"] = round(time_steps(torch, lambda: p.forward(c, out=f), steps, 1)[0], 4)
                sf = profile_stages(p, "profile_forward", c, reps, STAGES)
                rec["forward_stages_ms_fp64"] = {k: round(v, 4) for k, v in sf.items()}
                rec["roofline_fp64_forward"] = roofline_of(sf, stage_bytes(p, 16), KERNEL_NAMES)
        p.close()
        del c, g, f, fp, h
    rec["speedup"] = round(rec["ms_fp64"] / rec["ms_fp32"], 3)
    log("%s fwd+bwd FP32 %.3f ms, FP64 %.3f ms, speedup %.2f" % (label, rec["ms_fp32"], rec["ms_fp64"],
                                                                 rec["speedup"]))
    return rec, out


def _sample_with_sparse_bands(rng, M, bands, k):
    import numpy as np
    idx = set(rng.choice(M, size=min(k, M), replace=False).tolist())
    for b in np.unique(bands):
        sel = np.nonzero(bands == b)[0]
        if len(sel) < 64:
            idx.update(sel.tolist())
    return np.array(sorted(idx))


def step_errors(w, out, rec, seed):
    """E of every output of a timed step against the oracle: f and f' on 2000
    random nodes plus every node of bands holding < 64 nodes (relative to
    sum |c_k| and sum |2 pi k c_k|), the adjoint on 66 blocks of 32
    consecutive coefficients (the first, the last and 64 random ones;
    relative to sum |g_j|)."""
    import numpy as np

    import oracle
    from paper_1606_03255_amd import inputs
    N, M = w["N"], w["M"]
    c = np.asarray(w["c"], np.complex64).astype(np.complex128)
    g = inputs.adjoint_input(M).astype(np.complex128)
    rng = np.random.default_rng(seed)
    sel = _sample_with_sparse_bands(rng, M, out["fp32"]["bands"], 2000)
    zs = w["z"][sel]
    fr = oracle.forward(c, zs)
    fpr = oracle.derivative(c, zs)
    B = oracle.direct.block_size()
    nblk = -(-N // B)
    blocks = np.unique(np.concatenate([[0, nblk - 1], rng.choice(nblk, size=64, replace=False)]))
    k, hr = oracle.adjoint_blocks(g, w["z"], N, blocks)
    n1, n1d, n1g = np.abs(c).sum(), np.abs(2 * np.pi * np.arange(N) * c).sum(), np.abs(g).sum()
    for form in ("fp32", "fp64"):
        o = out[form]
        rec["E_f_" + form] = float(np.abs(o["f"][sel] - fr).max() / n1)
        rec["E_fprime_" + form] = float(np.abs(o["fp"][sel] - fpr).max() / n1d)
        rec["E_adjoint_" + form] = float(np.abs(o["h"][k] - hr).max() / n1g)
    rec["error_sample"] = "%d nodes, %d coefficients" % (len(sel), len(k))


def cpu_baseline(w, f32, f64, plan_bands, target_s=12.0):
    import numpy as np

    import oracle
    rng = np.random.default_rng(12345)
    c = w["c"].astype(np.complex128)
    z = w["z"]
    M = len(z)
    oracle.load()
    cal = rng.choice(M, size=256, replace=False)
    t = time.perf_counter()
    oracle.forward(c, z[cal])
    tc = time.perf_counter() - t
    S = int(min(M, max(256, 256 * target_s / max(tc, 1e-3))))
    sel = rng.choice(M, size=S, replace=False)
    t = time.perf_counter()
    ref = oracle.forward(c, z[sel])
    dt = time.perf_counter() - t
    # the independent cross-check algorithm (compensated Horner), timed on a
    # smaller sample of the same nodes
    hs = sel[:max(64, S // 16)]
    t = time.perf_counter()
    oracle.horner(c, z[hs])
    dth = time.perf_counter() - t
    # error check: the timed sample plus every node of bands holding < 64 nodes
    extra = []
    for bnd in np.unique(plan_bands):
        idx = np.nonzero(plan_bands == bnd)[0]
        if len(idx) < 64:
            extra.extend(idx.tolist())
    extra = np.setdiff1d(np.array(extra, dtype=np.int64), sel)
    ref_x = oracle.forward(c, z[extra]) if len(extra) else np.zeros(0, np.complex128)
    allsel = np.concatenate([sel, extra])
    allref = np.concatenate([ref, ref_x])
    n1 = np.abs(c).sum()
    E32 = float(np.abs(f32[allsel] - allref).max() / n1)
    E64 = float(np.abs(f64[allsel] - allref).max() / n1) if f64 is not None else None
    omp = os.environ.get("OMP_NUM_THREADS")
    return {"value": S / dt, "unit": "node evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "host_cpu_count": os.cpu_count(), "omp_num_threads": int(omp) if omp and omp.isdigit() else None,
            "horner_value": len(hs) / dth,
            "sample": "%d of the %d nodes drawn uniformly at random (seed 12345), all N=%d coefficients; "
                      "FP64 direct sum, %.1f s (compensated Horner: the first %d of them, %.1f s)"
                      % (S, M, len(c), dt, len(hs), dth)}, E32, E64, int(len(allsel))


def batched_leg(torch, dev, args, tune, log):
    """512 independent instances (N_i, M_i log-uniform in [2^8, 2^16], FP32 form,
    eps 1e-6) in one batched plan: forward per step, eager and graph-replayed.
    Returns the record and what the error check needs."""
    import numpy as np

    from paper_1606_03255_amd import Plan, inputs
    w = inputs.workload("batched")
    zs = [z for _, z in w["instances"]]
    c = torch.from_numpy(np.concatenate([ci for ci, _ in w["instances"]])).to(dev)
    t = time.perf_counter()
    pe = Plan.batch(w["N"], zs, 1e-6, torch.complex64, device=dev, autotune=tune)
    plan_ms = (time.perf_counter() - t) * 1e3
    pg = Plan.batch(w["N"], zs, 1e-6, torch.complex64, device=dev, graph=True, autotune=tune)
    f = torch.empty(pe.M, dtype=torch.complex64, device=dev)
    steps = max(5, args.steps)
    ms_e, _ = time_steps(torch, lambda: pe.forward(c, out=f), steps, args.warmup)
    fe = f.cpu().numpy()
    ms_g, _ = time_steps(torch, lambda: pg.forward(c, out=f), steps, args.warmup)
    fg = f.cpu().numpy()
    M = pe.M
    rec = {"instances": int(w["count"]), "sum_N": int(pe.N), "sum_M": int(M), "eps": 1e-6,
           "ms_forward_eager": round(ms_e, 4), "ms_forward_graph": round(ms_g, 4),
           "node_evals_per_s_graph": M / (ms_g * 1e-3), "plan_ms": round(plan_ms, 1),
           "direct_scale": pe.info()["direct_scale"], "graph_equals_eager": bool(np.array_equal(fe, fg))}
    log("batched: %d instances, forward eager %.3f ms, graph %.3f ms" % (rec["instances"], ms_e, ms_g))
    sample = {"w": w, "f": fg, "f_off": pe.f_offsets}
    pe.close()
    pg.close()
    return rec, sample


def batched_error(sample, rec):
    """E of the graph-replayed batched forward: 48 random nodes of each of 64
    random instances against the oracle, each relative to that instance's
    sum |c_k|; the worst instance is reported."""
    import numpy as np

    import oracle
    w, f, fo = sample["w"], sample["f"], sample["f_off"]
    rng = np.random.default_rng(4321)
    worst = 0.0
    insts = rng.choice(w["count"], size=64, replace=False)
    for i in insts:
        ci, zi = w["instances"][i]
        ci = ci.astype(np.complex128)
        sel = np.sort(rng.choice(len(zi), size=min(48, len(zi)), replace=False))
        E = np.abs(f[fo[i] + sel] - oracle.forward(ci, zi[sel])).max() / np.abs(ci).sum()
        worst = max(worst, float(E))
    rec["E"] = worst
    rec["error_sample"] = "48 nodes of each of 64 random instances"


def laplace_error(sample):
    """Part of the CPU-baseline leg: the Laplace leg's sampled nodes against
    the oracle's direct sums, relative to ||fhat||_1 (Thm A.3's E); for the
    K_{1/2} kernel, the largest error over the block-relative bar
    eps sum_k |fhat_k| max(1, K_{1/2}(y xi / 4)) (<= 1 required)."""
    import numpy as np

    import oracle.laplace as OL
    ref = OL.direct(sample["fhat"], sample["xi"], sample["y"])
    E = float(np.abs(sample["f"] - ref).max() / np.abs(sample["fhat"]).sum())
    Ek = None
    if "f_k12" in sample:
        refk = OL.direct_kernel(sample["fhat"], sample["xi"], sample["y_k12"], "bessel_k_half")
        w = np.maximum(1.0, OL.bessel_k_half(np.outer(sample["y_k12"], sample["xi"]) / 4.0))
        Ek = float((np.abs(sample["f_k12"] - refk) / (1e-6 * (w @ np.abs(sample["fhat"])))).max())
    return E, Ek


def laplace_leg(torch, dev, args, log):
    """The discrete Laplace transform (Algorithm 1) at N = M = 2^20: xi_k
    uniform in (0, N], y_j uniform in [0, 20/N] (exp(-y xi) spans 1 .. e^-20),
    complex64 coefficients, eps 1e-6.  Roofline: the algorithmic bytes of one
    call (per frequency: sorted value 8 B, index 4 B, fhat 8 B; per node: y
    8 B, band 4 B, f 8 B) over its time, against the HBM peak."""
    import numpy as np

    from paper_1606_03255_amd import LaplacePlan
    N = M = 1 << 20
    rng = np.random.default_rng(21)
    xi = rng.random(N) * N + 1e-3
    y = rng.random(M) * (20.0 / N)
    fhat = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    t = time.perf_counter()
    plan = LaplacePlan(xi, y, 1e-6, torch.complex64, device=dev)
    plan_ms = (time.perf_counter() - t) * 1e3
    fh = torch.from_numpy(fhat).to(dev)
    f = torch.empty(M, dtype=torch.complex64, device=dev)
    ms, _ = time_steps(torch, lambda: plan.forward(fh, out=f), max(5, args.steps), args.warmup)
    sel = np.sort(rng.choice(M, 64, replace=False))
    sample = {"fhat": fhat.astype(np.complex128), "xi": xi, "y": y[sel], "f": f.cpu().numpy()[sel]}
    nbytes = N * (8 + 4 + 8) + M * (8 + 4 + 8)
    info = plan.info()
    plan.close()
    rec = {"N": N, "M": M, "eps": 1e-6, "dtype": "c64 in/out, f64 arithmetic", "q": info["q"],
           "levels": info["levels"], "ms": round(ms, 4), "node_evals_per_s": M / (ms * 1e-3),
           "bytes_per_call": nbytes, "achieved_GBs": round(nbytes / (ms * 1e-3) / 1e9, 1),
           "frac_hbm": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "E": None, "plan_ms": round(plan_ms, 1)}
    log("laplace: %.4f ms, %.3e node evals/s" % (ms, rec["node_evals_per_s"]))
    # Thm 3.3's example kernel K_{1/2}(y xi) on the same frequencies, nodes moved off 0
    yk = y + 1e-9
    t = time.perf_counter()
    pk = LaplacePlan(xi, yk, 1e-6, torch.complex64, device=dev, kernel="bessel_k_half")
    plan_k = (time.perf_counter() - t) * 1e3
    ms_k, _ = time_steps(torch, lambda: pk.forward(fh, out=f), max(5, args.steps), args.warmup)
    ik = pk.info()
    pk.close()
    sample["y_k12"] = yk[sel]
    sample["f_k12"] = f.cpu().numpy()[sel]
    rec["k12"] = {"kernel": "K_1/2(y xi)", "y": "uniform in [1e-9, 20/N + 1e-9]", "q": ik["q"],
                  "levels": ik["levels"], "ms": round(ms_k, 4), "node_evals_per_s": M / (ms_k * 1e-3),
                  "E_over_bar": None, "plan_ms": round(plan_k, 1)}
    log("laplace K_1/2: %.4f ms, q %d, levels %d" % (ms_k, ik["q"], ik["levels"]))
    return rec, sample


def xi_error(sample):
    """Part of the CPU-baseline leg: the real-exponent leg's sampled nodes and
    exponents against the oracle's term-by-term sums, relative to the 1-norm
    of the input."""
    import numpy as np

    import oracle
    Ef = np.abs(sample["f"] - oracle.forward_xi(sample["c"], sample["xi"], sample["zs"])).max() / np.abs(sample["c"]).sum()
    Eh = np.abs(sample["h"] - oracle.transposed_xi(sample["g"], sample["z"], sample["xis"])).max() / np.abs(sample["g"]).sum()
    return float(Ef), float(Eh)


def xi_leg(torch, dev, args, log):
    """Real exponents (eq. 4.1 with real xi_k; the transposed g(xi) of Sect. 4)
    at N = M = 2^args.xi_log2n: exponents uniform in [1, N], nodes as the
    main workload (half annulus, half disk), complex64, eps 1e-6 (FP32 form):
    time per forward and per transposed call, node evals/s, and the error of
    both on sampled nodes / exponents."""
    import numpy as np

    from paper_1606_03255_amd import XiPlan, inputs
    w = inputs.workload("xi", log2n=args.xi_log2n)
    N, M = w["N"], w["M"]
    t = time.perf_counter()
    plan = XiPlan(w["xi"], w["z"], 1e-6, torch.complex64, device=dev)
    plan_ms = (time.perf_counter() - t) * 1e3
    c = torch.from_numpy(w["c"]).to(dev)
    g_h = inputs.adjoint_input(M)
    g = torch.from_numpy(g_h).to(dev)
    f = torch.empty(M, dtype=torch.complex64, device=dev)
    h = torch.empty(N, dtype=torch.complex64, device=dev)
    ms_f, _ = time_steps(torch, lambda: plan.forward(c, out=f), max(5, args.steps), args.warmup)
    ms_h, _ = time_steps(torch, lambda: plan.transposed(g, out=h), max(5, args.steps), args.warmup)
    info = plan.info()
    plan.close()
    rng = np.random.default_rng(23)
    sj = np.sort(rng.choice(M, 256, replace=False))
    sk = np.sort(rng.choice(N, 128, replace=False))
    sample = {"c": w["c"].astype(np.complex128), "xi": w["xi"], "zs": w["z"][sj], "f": f.cpu().numpy()[sj],
              "g": g_h.astype(np.complex128), "z": w["z"], "xis": w["xi"][sk], "h": h.cpu().numpy()[sk]}
    rec = {"N": N, "M": M, "eps": 1e-6, "dtype": "c64 (FP32 form)", "exponents": "uniform in [1, N]",
           "ms_forward": round(ms_f, 4), "ms_transposed": round(ms_h, 4),
           "node_evals_per_s": M / (ms_f * 1e-3), "exponent_evals_per_s": N / (ms_h * 1e-3),
           "mw1": info["mw1"], "inner_mw": info["inner_mw"], "inner_instances": info["inner_instances"],
           "inner_nodes": info["inner_nodes"], "inner_coefficients": info["inner_coefficients"],
           "sigma_min": round(info["sigma_min"], 4), "eps_inner": info["eps_in"],
           "E_forward": None, "E_transposed": None, "plan_ms": round(plan_ms, 1)}
    log("xi: forward %.4f ms (%.3e node evals/s), transposed %.4f ms" % (ms_f, rec["node_evals_per_s"], ms_h))
    return rec, sample


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forward-only", action="store_true", help="skip the fwd+bwd and FP64 legs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="plans with the default band policy instead of the timed choice")
    ap.add_argument("--direct-scale", type=float, default=None,
                    help="the main FP32 plan's band-policy factor, fixed instead of timed (for counter "
                         "runs that reproduce a tuned plan)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-instance batched leg")
    ap.add_argument("--no-laplace", action="store_true", help="skip the Laplace-transform (Algorithm 1) leg")
    ap.add_argument("--no-grad", action="store_true", help="skip the fwd+bwd step at N = M = 2^18")
    ap.add_argument("--no-xi", action="store_true", help="skip the real-exponent leg")
    ap.add_argument("--xi-log2n", type=int, default=20, help="log2 N = log2 M of the real-exponent leg")
    ap.add_argument("--only", choices=["batched", "xi", "laplace"],
                    help="run this side leg alone and print its record instead of the benchmark line "
                         "(for profiling one workload's kernels)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a known-size reference "
                         "for HBM counter readings)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this transform runs on one GPU; --gpus %d is not supported (use --gpus 1)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1606_03255_amd import Plan, inputs

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe_mb:
        src = torch.empty(args.copy_probe_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only:
        tune = not args.no_autotune
        leg = {"batched": lambda: batched_leg(torch, dev, args, tune, log),
               "xi": lambda: xi_leg(torch, dev, args, log),
               "laplace": lambda: laplace_leg(torch, dev, args, log)}[args.only]
        rec, _ = leg()
        print(json.dumps({"only": args.only, args.only: rec}, default=float), flush=True)
        return
    copy_gbs = copy_bandwidth(torch, dev)
    log("device-to-device copy %.1f GB/s" % copy_gbs)
    w = inputs.workload("large")
    N, M = w["N"], w["M"]
    t = time.perf_counter()
    tune = not args.no_autotune
    # the value is a forward throughput: its plan's band policy is tuned on the
    # forward alone; the fwd+bwd step uses plans tuned on forward + adjoint
    if args.direct_scale is not None:
        p32 = Plan(N, w["z"], 1e-6, torch.complex64, device=dev, direct_scale=args.direct_scale)
    else:
        p32 = Plan(N, w["z"], 1e-6, torch.complex64, device=dev, autotune="forward" if tune else False)
    plan32_ms = (time.perf_counter() - t) * 1e3
    log("FP32 plan built in %.0f ms" % plan32_ms)
    c32 = torch.from_numpy(w["c"]).to(dev)
    f32_out = torch.empty(M, dtype=torch.complex64, device=dev)

    ms_fwd, wall = time_steps(torch, lambda: p32.forward(c32, out=f32_out), args.steps, args.warmup)
    value = M / (ms_fwd * 1e-3)
    log("FP32 forward %.3f ms/step -> %.3e node evals/s" % (ms_fwd, value))
    f32 = f32_out.cpu().numpy().astype(np.complex128)

    # per-kernel durations (HIP events between the launches on the current stream)
    reps = max(3, min(args.steps, 10))
    stage_ms = profile_stages(p32, "profile_forward", c32, reps, STAGES)
    sb = stage_bytes(p32, 8)
    dom = max(STAGES, key=lambda k: stage_ms[k])
    if dom == "direct":
        # direct sums: c comes from L2 and the Infinity Cache; the bound is the
        # FP32 ALU: 4 FMAs (8 flops) per term and node (Horner's scheme)
        nd = sum(b["nodes"] for b in p32.bands() if b["direct"])
        flops = 8.0 * nd * N
        achieved = flops / (stage_ms[dom] * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": traffic_for(dom, sb[dom]),
                    "kernel": KERNEL_NAMES[dom], "flops_per_launch": flops, "ms_per_launch": round(stage_ms[dom], 4)}
    else:
        achieved = sb[dom] / (stage_ms[dom] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom, sb[dom]),
                    "kernel": KERNEL_NAMES[dom], "bytes_per_launch": sb[dom], "ms_per_launch": round(stage_ms[dom], 4),
                    "frac_of_measured_copy": round(achieved / copy_gbs, 4)}
    log("stages ms", {k: round(v, 4) for k, v in stage_ms.items()})

    fwd_bwd = fwd_bwd_grad = None
    step_out = grad_out = None
    f64 = None
    E64 = None
    if not args.forward_only:
        fwd_bwd, step_out = step_leg(torch, dev, w, 1e-6, 1e-11, args, tune, log, "N=M=2^20", True)
        f64 = step_out["fp64"]["f"].astype(np.complex128)
        if not args.no_grad:
            wg = inputs.workload("grad")
            fwd_bwd_grad, grad_out = step_leg(torch, dev, wg, 1e-6, 1e-11, args, tune, log, "N=M=2^18", False)

    batched = bsample = None
    if not args.no_batched:
        batched, bsample = batched_leg(torch, dev, args, tune, log)
    laplace = lap_sample = None
    if not args.no_laplace and not args.forward_only:
        laplace, lap_sample = laplace_leg(torch, dev, args, log)

    xi = xi_sample = None
    if not args.no_xi and not args.forward_only:
        xi, xi_sample = xi_leg(torch, dev, args, log)

    cpu = None
    E32 = None
    n_checked = 0
    if not args.no_cpu_baseline:
        cpu, E32, E64, n_checked = cpu_baseline(w, f32, f64, p32.node_bands())
        log("cpu baseline", cpu, "E32", E32, "E64", E64)
        if fwd_bwd is not None:
            step_errors(w, step_out, fwd_bwd, 11)
        if fwd_bwd_grad is not None:
            step_errors(inputs.workload("grad"), grad_out, fwd_bwd_grad, 12)
        if batched is not None:
            batched_error(bsample, batched)
        if laplace is not None:
            laplace["E"], laplace["k12"]["E_over_bar"] = laplace_error(lap_sample)
            log("laplace E", laplace["E"], "K_1/2 error / bar", laplace["k12"]["E_over_bar"])
        if xi is not None:
            xi["E_forward"], xi["E_transposed"] = xi_error(xi_sample)
            log("xi E", xi["E_forward"], xi["E_transposed"])

    info = p32.info()
    rec = {
        "metric": METRIC, "value": value, "unit": "node evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_fwd, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "N=M=2^20, half annulus 1-1e-3<|w|<=1, half disk, complex64, eps=1e-6, FP32 form",
                   "N": N, "M": M, "eps": 1e-6, "q": info["q"], "D": info["D"], "mw": info["mw"],
                   "bands": info["num_bands"], "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error": {"E_fp32_form": E32, "E_fp64_path": E64, "nodes_checked": n_checked},
        "fwd_bwd": fwd_bwd,
        "fwd_bwd_grad": fwd_bwd_grad,
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_bytes": sb,
        "stage_frac_hbm": stage_fracs(stage_ms, sb),
        "hbm_copy_GBs": copy_gbs,
        "plan_ms": round(plan32_ms, 1),
        "direct_scale": info["direct_scale"],
        "batched": batched,
        "laplace": laplace,
        "xi": xi,
        "bytes_forward_model": info["bytes_forward"],
        "wall_s_timed": round(wall, 3),
    }
    p32.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
