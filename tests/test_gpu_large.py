"""GPU parity at the benchmark's own size, N = M = 2^20 (half annulus
1 - 1e-3 < |w| <= 1, half disk), in the launch configurations the benchmark
times: the forward on a plan tuned for the forward alone, and the training
step (fused forward + derivative, then the adjoint) on plans tuned for that
step, for the FP32 form (eps 1e-6) and the plain FP64 path (eps 1e-11).

The oracle cannot afford all 2^40 terms here, so every result is compared on
a sample the oracle computes one by one:
* f and f' on every node of each band holding < 64 nodes plus 1500 random
  nodes (FP64 direct sums at those nodes, all N coefficients);
* the adjoint C^H g on 66 whole blocks of 32 consecutive coefficients (the
  first, the last, which is ragged, and 64 random ones), each an FP64 sum over
  all M nodes.
Bars (Thm 4.3, relative to the 1-norm of the transform's input): forward
E <= eps; derivative E <= eps against sum |2 pi k c_k|; adjoint E <= eps
against sum |g_j|.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1606_03255_amd import inputs

pytestmark = pytest.mark.gpu

STEP_CASES = [("c64", 1e-6), ("c128", 1e-11)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def large():
    return inputs.workload("large")


def _sample_nodes(plan_bands, M, rng, k=1500):
    """Every node of each band with < 64 nodes plus k random nodes."""
    idx = set(rng.choice(M, size=min(k, M), replace=False).tolist())
    for b in np.unique(plan_bands):
        sel = np.nonzero(plan_bands == b)[0]
        if len(sel) < 64:
            idx.update(sel.tolist())
    return np.array(sorted(idx))


def _sample_blocks(N, rng, k=64):
    B = oracle.direct.block_size()
    nblk = -(-N // B)
    return np.unique(np.concatenate([[0, nblk - 1], rng.choice(nblk, size=k, replace=False)]))


def _tdt(torch, dtype):
    return torch.complex64 if dtype == "c64" else torch.complex128


@pytest.mark.parametrize("dtype,eps,tune", [("c64", 1e-6, "forward"), ("c128", 1e-11, "forward"),
                                            ("c64", 1e-6, "nfft_only")])
def test_large_forward_sampled(torch, large, dtype, eps, tune):
    """The forward on the plan the benchmark's value is timed on (tuned on the
    forward alone), and with every band on the NFFT path."""
    from paper_1606_03255_amd import Plan
    w = large
    _say("large forward", dtype, eps, tune)
    c = w["c"].astype(np.complex128)
    tdt = _tdt(torch, dtype)
    plan = Plan(w["N"], w["z"], eps, tdt, nfft_only=tune == "nfft_only",
                autotune="forward" if tune == "forward" else False)
    f = plan.forward(torch.from_numpy(c).to("cuda", tdt)).cpu().numpy().astype(np.complex128)
    sel = _sample_nodes(plan.node_bands(), w["M"], np.random.default_rng(0))
    _say("   direct_scale", plan.info()["direct_scale"])
    plan.close()
    E = np.abs(f[sel] - oracle.forward(c, w["z"][sel])).max() / np.abs(c).sum()
    _say("   sampled nodes", len(sel), "E =", E)
    assert E <= eps


@pytest.mark.parametrize("dtype,eps", STEP_CASES)
def test_large_training_step_sampled(torch, large, dtype, eps):
    """The benchmark's fwd+bwd step on its step-tuned plan: the fused
    forward + derivative call, the adjoint of the benchmark's g, and the
    derivative by its own call."""
    from paper_1606_03255_amd import Plan
    w = large
    N, M = w["N"], w["M"]
    tdt = _tdt(torch, dtype)
    c = w["c"].astype(np.complex128)            # complex64 values (the FP64 path gets them promoted)
    g = inputs.adjoint_input(M).astype(np.complex128)
    plan = Plan(N, w["z"], eps, tdt, autotune=True)
    _say("large step", dtype, eps, "direct_scale", plan.info()["direct_scale"])
    ct = torch.from_numpy(c).to("cuda", tdt)
    gt = torch.from_numpy(g).to("cuda", tdt)
    f, fp = plan.forward_derivative(ct)
    h = plan.adjoint(gt)
    fp_sep = plan.derivative(ct)
    torch.cuda.synchronize()
    f, fp, h, fp_sep = (t.cpu().numpy().astype(np.complex128) for t in (f, fp, h, fp_sep))
    rng = np.random.default_rng(1)
    sel = _sample_nodes(plan.node_bands(), M, rng)
    plan.close()

    n1, n1d, n1g = np.abs(c).sum(), np.abs(2 * np.pi * np.arange(N) * c).sum(), np.abs(g).sum()
    zs = w["z"][sel]
    E = np.abs(f[sel] - oracle.forward(c, zs)).max() / n1
    fpr = oracle.derivative(c, zs)
    Ed = np.abs(fp[sel] - fpr).max() / n1d
    Eds = np.abs(fp_sep[sel] - fpr).max() / n1d
    k, href = oracle.adjoint_blocks(g, w["z"], N, _sample_blocks(N, rng))
    Eh = np.abs(h[k] - href).max() / n1g
    _say("   nodes", len(sel), "coefficients", len(k), "E f =", E, " E f' (fused) =", Ed,
         " E f' (own call) =", Eds, " E C^H g =", Eh)
    assert E <= eps and Ed <= eps and Eds <= eps and Eh <= eps
