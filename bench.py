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
           ms_separate_fp32 times the three calls made one by one.
roofline   the dominant kernel's algorithmic bytes per launch over its launch
           duration (HIP events recorded between the launches on the stream
           the kernels run on), against the 8 TB/s HBM peak; for the direct
           sums (ALU-bound) their flops against the FP32 vector peak.
laplace    the discrete Laplace transform (Algorithm 1) at N = M = 2^20: time
           per call, node evals/s, algorithmic bytes against the HBM peak, and
           its error on sampled nodes against the oracle's direct sums.
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
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32, published
STAGES = ("onepass_fft", "passA_fft", "passB_fft", "gather", "direct")
KERNEL_NAMES = {"onepass_fft": "k_onepass_fwd", "passA_fft": "k_passA_fwd", "passB_fft": "k_passB",
                "gather": "k_gather", "direct": "k_direct_fwd"}
DIRECT_NG = 8   # nodes per direct-sum workgroup (c is read once per group)


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
    v = rec.get("kernels", {}).get(KERNEL_NAMES[kernel])
    if v is None or v.get("algorithmic_bytes_per_launch") != algorithmic_bytes:
        return None
    return v.get("bytes_per_launch")


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
    E64 = float(np.abs(f64[allsel] - allref).max() / n1)
    return {"value": S / dt, "unit": "node evals/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d of the %d nodes drawn uniformly at random (seed 12345), all N=%d coefficients; "
                      "FP64 direct sum, %.1f s" % (S, M, len(c), dt)}, E32, E64, int(len(allsel))


def batched_leg(torch, dev, args, tune, log):
    """512 independent instances (N_i, M_i log-uniform in [2^8, 2^16], FP32 form,
    eps 1e-6) in one batched plan: forward per step, eager and graph-replayed."""
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
    ms_g, _ = time_steps(torch, lambda: pg.forward(c, out=f), steps, args.warmup)
    M = pe.M
    rec = {"instances": int(w["count"]), "sum_N": int(pe.N), "sum_M": int(M), "eps": 1e-6,
           "ms_forward_eager": round(ms_e, 4), "ms_forward_graph": round(ms_g, 4),
           "node_evals_per_s_graph": M / (ms_g * 1e-3), "plan_ms": round(plan_ms, 1),
           "direct_scale": pe.info()["direct_scale"]}
    log("batched: %d instances, forward eager %.3f ms, graph %.3f ms" % (rec["instances"], ms_e, ms_g))
    pe.close()
    pg.close()
    return rec


def laplace_error(sample):
    """Part of the CPU-baseline leg: the Laplace leg's sampled nodes against
    the oracle's direct sums, relative to ||fhat||_1 (Thm A.3's E)."""
    import numpy as np

    import oracle.laplace as OL
    ref = OL.direct(sample["fhat"], sample["xi"], sample["y"])
    return float(np.abs(sample["f"] - ref).max() / np.abs(sample["fhat"]).sum())


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
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-instance batched leg")
    ap.add_argument("--no-laplace", action="store_true", help="skip the Laplace-transform (Algorithm 1) leg")
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
    w = inputs.workload("large")
    N, M = w["N"], w["M"]
    t = time.perf_counter()
    tune = not args.no_autotune
    # the value is a forward throughput: its plan's band policy is tuned on the
    # forward alone; the fwd+bwd step uses plans tuned on forward + adjoint
    p32 = Plan(N, w["z"], 1e-6, torch.complex64, device=dev, autotune="forward" if tune else False)
    plan32_ms = (time.perf_counter() - t) * 1e3
    log("FP32 plan built in %.0f ms" % plan32_ms)
    c32 = torch.from_numpy(w["c"]).to(dev)
    rng = np.random.default_rng(7)
    g = (rng.standard_normal(M) + 1j * rng.standard_normal(M)) * np.sqrt(0.5)
    g32 = torch.from_numpy(g.astype(np.complex64)).to(dev)
    f32_out = torch.empty(M, dtype=torch.complex64, device=dev)

    ms_fwd, wall = time_steps(torch, lambda: p32.forward(c32, out=f32_out), args.steps, args.warmup)
    value = M / (ms_fwd * 1e-3)
    log("FP32 forward %.3f ms/step -> %.3e node evals/s" % (ms_fwd, value))
    f32 = f32_out.cpu().numpy().astype(np.complex128)

    # per-kernel durations (HIP events between the launches on the current stream)
    reps = max(3, min(args.steps, 10))
    acc = [0.0] * 5
    for _ in range(reps):
        _, ms = p32.profile_forward(c32)
        acc = [a + b for a, b in zip(acc, ms)]
    stage_ms = {k: v / reps for k, v in zip(STAGES, acc)}
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
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom, sb[dom]), "kernel": KERNEL_NAMES[dom],
                    "bytes_per_launch": sb[dom], "ms_per_launch": round(stage_ms[dom], 4)}
    log("stages ms", {k: round(v, 4) for k, v in stage_ms.items()})

    fwd_bwd = None
    f64 = None
    E64 = None
    if not args.forward_only:
        fp32_out = torch.empty_like(f32_out)
        ps = Plan(N, w["z"], 1e-6, torch.complex64, device=dev, autotune=tune)   # tuned on forward + adjoint
        step_scale = ps.info()["direct_scale"]

        def step32():
            ps.forward_derivative(c32, out=f32_out, out_prime=fp32_out)
            ps.adjoint(g32)
        ms32, _ = time_steps(torch, step32, max(3, args.steps // 2), 1)

        def step32_separate():
            ps.forward(c32, out=f32_out)
            ps.adjoint(g32)
            ps.derivative(c32)
        ms32_sep, _ = time_steps(torch, step32_separate, max(3, args.steps // 2), 1)
        ps.close()
        p64 = Plan(N, w["z"], 1e-11, torch.complex128, device=dev, autotune=tune)
        c64 = c32.to(torch.complex128)
        g64 = g32.to(torch.complex128)
        f64_out = torch.empty(M, dtype=torch.complex128, device=dev)
        fp64_out = torch.empty_like(f64_out)

        def step64():
            p64.forward_derivative(c64, out=f64_out, out_prime=fp64_out)
            p64.adjoint(g64)
        ms64, _ = time_steps(torch, step64, max(3, args.steps // 2), 1)
        ms64_fwd, _ = time_steps(torch, lambda: p64.forward(c64, out=f64_out), max(3, args.steps // 2), 1)
        f64 = f64_out.cpu().numpy()
        p64.close()
        fwd_bwd = {"ms_fp32_form": round(ms32, 4), "ms_fp64_path": round(ms64, 4),
                   "speedup": round(ms64 / ms32, 3), "ms_fp64_forward": round(ms64_fwd, 4),
                   "ms_separate_fp32": round(ms32_sep, 4), "direct_scale_fp32": step_scale}
        log("fwd+bwd FP32 %.3f ms, FP64 %.3f ms, speedup %.2f" % (ms32, ms64, ms64 / ms32))

    batched = None
    if not args.no_batched:
        batched = batched_leg(torch, dev, args, tune, log)
    laplace = lap_sample = None
    if not args.no_laplace and not args.forward_only:
        laplace, lap_sample = laplace_leg(torch, dev, args, log)

    cpu = None
    E32 = None
    n_checked = 0
    if not args.no_cpu_baseline:
        cpu, E32, E64c, n_checked = cpu_baseline(w, f32, f64 if f64 is not None else f32, p32.node_bands())
        E64 = E64c if f64 is not None else None
        log("cpu baseline", cpu, "E32", E32, "E64", E64)
        if laplace is not None:
            laplace["E"] = laplace_error(lap_sample)
            log("laplace E", laplace["E"])

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
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_bytes": sb,
        "plan_ms": round(plan32_ms, 1),
        "direct_scale": info["direct_scale"],
        "batched": batched,
        "laplace": laplace,
        "bytes_forward_model": info["bytes_forward"],
        "wall_s_timed": round(wall, 3),
    }
    p32.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
