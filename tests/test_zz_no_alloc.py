"""flt_forward_noalloc, the forward without a workspace (its scratch is the
library's static device array), called through the C ABI and checked against
flt_forward on the same plans, to the same bar as every forward: the two
agree to rounding, and each meets E <= eps against the FP64 direct sums.

Two calls in a row on one stream, the second with a smaller plan (the array
then still holds the first call's larger contents), and a plan whose forward
needs more scratch than the array holds, which is refused before any device
work."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1606_03255_amd import _lib as L
from paper_1606_03255_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _noalloc(torch, plan, c, f):
    lib = L.load()
    stream = torch.cuda.current_stream().cuda_stream
    return lib.flt_forward_noalloc(plan._ptr, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                   ctypes.c_void_p(stream))


def _nodes(rng, M):
    return np.concatenate([inputs.nodes_annulus(rng, M // 2), inputs.nodes_disk(rng, M - M // 2)])


def test_noalloc_forward_two_calls_against_workspace_forward(torch):
    from paper_1606_03255_amd import Plan
    rng = np.random.default_rng(2024)
    # (N, M, eps, dtype): the larger first (two-pass FFT bands, several tiles,
    # direct-sum bands), then a smaller one-pass plan in the other dtype
    cases = [(1 << 14, 1 << 14, 1e-6, torch.complex64), (700, 300, 1e-10, torch.complex128)]
    runs = []
    for N, M, eps, tdt in cases:
        z = _nodes(rng, M)
        c = inputs.coefficients(rng, N)
        if tdt == torch.complex64:
            c = c.astype(np.complex64).astype(np.complex128)
        plan = Plan(N, z, eps, tdt)
        info = plan.info()
        assert 0 < info["forward_scratch_bytes"] <= L.FLT_NOALLOC_MAX_BYTES
        ct = torch.from_numpy(c).to("cuda", tdt)
        runs.append((N, M, eps, tdt, z, c, plan, ct, torch.empty(M, dtype=tdt, device="cuda")))
    for N, M, eps, tdt, z, c, plan, ct, fna in runs:          # the two calls, back to back
        _say("noalloc forward", N, M, eps, tdt)
        assert _noalloc(torch, plan, ct, fna) == 0
    torch.cuda.synchronize()
    for N, M, eps, tdt, z, c, plan, ct, fna in runs:
        fws = plan.forward(ct).cpu().numpy().astype(np.complex128)
        f = fna.cpu().numpy().astype(np.complex128)
        n1 = np.abs(c).sum()
        E = np.abs(f - oracle.forward(c, z)).max() / n1
        D = np.abs(f - fws).max() / n1
        # same kernels and plan: rounding differences only (the direct-sum
        # bands' FP64 partial sums may be added in another order)
        tol = 1e-7 if tdt == torch.complex64 else 1e-15
        _say("   E =", E, " |noalloc - workspace| / ||c||_1 =", D)
        assert E <= eps and D <= tol
        plan.close()


def test_noalloc_forward_refuses_plans_beyond_the_array(torch):
    from paper_1606_03255_amd import Plan
    rng = np.random.default_rng(5)
    N = M = 1 << 16
    plan = Plan(N, _nodes(rng, M), 1e-6, torch.complex64)
    assert plan.info()["forward_scratch_bytes"] > L.FLT_NOALLOC_MAX_BYTES
    c = torch.zeros(N, dtype=torch.complex64, device="cuda")
    f = torch.full((M,), 7.0, dtype=torch.complex64, device="cuda")
    assert _noalloc(torch, plan, c, f) == -8          # FLT_ERANGE
    torch.cuda.synchronize()
    assert bool((f == 7.0).all())                     # nothing was launched
    plan.close()
