"""Host-side checks of the C ABI (no GPU): the library loads and exports every
symbol the header declares; host-only plans report the parameters of
Def. 3.2 / Lemma 4.1 and the partition the oracle computes; invalid input is
rejected with the documented codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1606_03255_amd as flt
from paper_1606_03255_amd import _lib as L
from paper_1606_03255_amd import inputs
from oracle import method as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    lib = L.load()
    hdr = open(os.path.join(ROOT, "include", "flt.h")).read()
    declared = set(re.findall(r"\b(flt_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("N,eps,dt", [(256, 1e-10, "complex128"), (1 << 14, 1e-6, "complex64"),
                                      (1 << 20, 1e-11, "complex128"), (3, 1e-4, "complex64"), (1, 1e-6, "complex64")])
def test_host_plan_parameters_and_partition(N, eps, dt):
    rng = np.random.default_rng(N)
    z = np.concatenate([inputs.nodes_disk(rng, 500), inputs.nodes_annulus(rng, 500)])
    z[0] = complex(0.1, np.inf)
    z[1] = 0.5 + 0j
    p = flt.Plan(N, z, eps, dt, host_only=True)
    info = p.info()
    P = O.Params(N, eps)
    assert (info["q"], info["D"], info["n_xi"], info["mw"]) == (P.q, P.D, P.n, P.mw)
    assert info["eps_K"] == pytest.approx(eps / 3) and info["eps_A"] == pytest.approx(eps / 3)
    x, y = O.polar(z)
    assert np.array_equal(p.node_bands(), O.node_band(P, y))
    bands = p.bands()
    assert sum(b["nodes"] for b in bands) + info["nodes_z0"] == len(z) or N == 1
    for b in bands:
        m = b["m"]
        if m < P.D:
            assert (b["ell_lo"], b["ell_hi"]) == (P.ell(m), P.L(m))
            assert b["q"] == P.q
            assert (b["n"], b["k0"]) == P.grid(m)
        else:
            assert b["q"] == 1 and (b["n"], b["k0"]) == P.grid(P.D)
    p.close()


def _create(N, M, z, eps, dtype, flags=L.FLT_FLAG_HOST_ONLY):
    lib = L.load()
    ptr = ctypes.c_void_p()
    zz = np.ascontiguousarray(z, np.complex128)
    rc = lib.flt_plan_create(ctypes.byref(ptr), N, M, zz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             eps, dtype, flags)
    if rc == 0:
        lib.flt_plan_destroy(ptr)
    return rc


def test_error_codes():
    z = np.array([0.1 + 0.1j, 0.2 + 0.0j])
    assert _create(10, 2, z, 1e-6, 1) == 0
    assert _create(0, 2, z, 1e-6, 1) == -1                               # N < 1: EINVAL
    assert _create(10, 0, z, 1e-6, 1) == -1                               # M < 1
    assert _create(10, 2, z, 1e-6, 3) == -1                               # dtype
    assert _create(10, 2, z, 1e-6, 1, flags=1 << 7) == -1                 # flags
    assert _create(10, 2, z, 1e-6, 1, flags=L.FLT_FLAG_HOST_ONLY | L.FLT_FLAG_AUTOTUNE | L.FLT_FLAG_TUNE_FORWARD) == 0
    assert _create(10, 2, z, 1.5, 1) == -2                                # eps not in (0,1)
    assert _create(10, 2, z, 0.0, 1) == -2
    assert _create(10, 2, np.array([0.1 - 1e-9j, 0.2]), 1e-6, 1) == -2    # Im z < 0
    assert _create(10, 2, np.array([complex(np.nan, 0.1), 0.2]), 1e-6, 1) == -2
    assert _create(10, 2, np.array([complex(np.inf, 0.1), 0.2]), 1e-6, 1) == -2
    assert _create(10, 2, np.array([complex(0.1, np.nan), 0.2]), 1e-6, 1) == -2
    assert _create(10, 2, np.array([complex(0.1, np.inf), 0.2]), 1e-6, 1) == 0   # w = 0 is fine
    assert _create(10, 2, z, 1e-7, 1) == -3                               # below the FP32 floor
    assert _create(10, 2, z, 1e-15, 2) == -3                              # below the FP64 floor
    assert _create((1 << 21) + 2, 2, z, 1e-6, 1) == -8                    # beyond the largest grid


def test_host_only_plan_refuses_device_work():
    lib = L.load()
    ptr = ctypes.c_void_p()
    z = np.ascontiguousarray(np.array([0.1 + 0.1j, 0.2 + 0.0j]))
    assert lib.flt_plan_create(ctypes.byref(ptr), 10, 2, z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               1e-6, 1, L.FLT_FLAG_HOST_ONLY) == 0
    dummy = ctypes.c_void_p(16)
    assert lib.flt_forward(ptr, dummy, dummy, None) == -6
    assert lib.flt_adjoint(ptr, dummy, dummy, None) == -6
    assert lib.flt_plan_set_workspace(ptr, dummy, 1 << 30) == -6
    assert lib.flt_forward_derivative(ptr, dummy, dummy, ctypes.c_void_p(32), None) == -6
    assert lib.flt_forward(None, dummy, dummy, None) == -1
    assert lib.flt_forward_derivative(None, dummy, dummy, ctypes.c_void_p(32), None) == -1
    assert lib.flt_forward_derivative(ptr, None, dummy, ctypes.c_void_p(32), None) == -1
    size = ctypes.c_size_t()
    assert lib.flt_plan_workspace_size(ptr, ctypes.byref(size)) == 0 and size.value > 0
    assert lib.flt_strerror(-4) == b"workspace missing or too small"
    lib.flt_plan_destroy(ptr)
    lib.flt_plan_destroy(None)


def test_byte_model_large_workload():
    w = inputs.workload("large")
    p = flt.Plan(w["N"], w["z"], 1e-6, "complex64", host_only=True)
    info = p.info()
    bands = p.bands()
    S = 8
    expect = w["M"] * (16 + 4 + S)
    for b in bands:
        if b["direct"]:    # c read once per group of 8 nodes of a direct-sum band
            expect += w["N"] * S * -(-b["nodes"] // 8)
        else:              # c once; grids: one-pass written once, two-pass pass-A output
            #                written and read once plus the masked cells; gather reads
            cells = b["cells"]
            expect += min(b["K"], w["N"] - 1) * S + b["q"] * min(cells, b["nodes"] * 2 * info["mw"]) * S
            expect += (2 * b["q"] * b["n"] + b["q"] * cells if b["passes"] == 2 else b["q"] * b["n"]) * S
    assert info["bytes_forward"] == pytest.approx(expect, rel=1e-12)
    assert (info["q"], info["D"]) == (12, 47)
    # the policy sends exactly the sparsely filled full-size bands to the direct sum
    assert all(b["nodes"] < 300 for b in bands if b["direct"])
    assert all(b["n"] == 1 << 21 for b in bands if b["direct"])
    p2 = flt.Plan(w["N"], w["z"], 1e-6, "complex64", host_only=True, nfft_only=True)
    assert not any(b["direct"] for b in p2.bands())


def test_cell_counts_cover_every_window():
    """cells = size of the union of the nodes' windows [l0 - mw + 1, l0 + mw]
    (mod n), l0 = floor(n x): the cells pass B stores and the gather reads."""
    rng = np.random.default_rng(11)
    N, M = 70000, 3000
    z = np.concatenate([inputs.nodes_annulus(rng, M // 2), inputs.nodes_disk(rng, M - M // 2)])
    p = flt.Plan(N, z, 1e-6, "complex64", host_only=True)
    mw = p.info()["mw"]
    nb = p.node_bands()
    x = z.real - np.floor(z.real)
    for b in p.bands():
        if b["direct"]:
            assert b["cells"] == 0
            continue
        n = b["n"]
        l0 = np.floor(np.ldexp(x[nb == b["m"]], int(np.log2(n)))).astype(np.int64)
        hit = np.zeros(n, bool)
        for t in range(2 * mw):
            hit[(l0 - mw + 1 + t) % n] = True
        assert b["cells"] == hit.sum(), b


def test_batched_host_plan_concatenates_members():
    """A batched host plan holds every member's bands and nodes: counts, band
    lists and per-node bands equal those of the members' own plans."""
    rng = np.random.default_rng(3)
    Ns = [300, 1, 5000, 70000]
    zs = [inputs.nodes_disk(rng, m) for m in (100, 7, 1000, 2000)]
    bp = flt.Plan.batch(Ns, zs, 1e-6, "complex64", host_only=True)
    singles = [flt.Plan(n, z, 1e-6, "complex64", host_only=True) for n, z in zip(Ns, zs)]
    info = bp.info()
    assert info["N"] == sum(Ns) and info["M"] == sum(len(z) for z in zs)
    assert info["num_bands"] == sum(s.info()["num_bands"] for s in singles)
    assert info["bytes_forward"] == pytest.approx(sum(s.info()["bytes_forward"] for s in singles), rel=1e-12)
    assert [b for s in singles for b in s.bands()] == bp.bands()
    assert np.array_equal(bp.node_bands(), np.concatenate([s.node_bands() for s in singles]))
    assert list(bp.c_offsets) == [0, 300, 301, 5301] and list(bp.f_offsets) == [0, 100, 107, 1107]


def test_batched_errors():
    lib = L.load()
    ptr = ctypes.c_void_p()
    N = np.array([10, 20], np.int64)
    M = np.array([2, 2], np.int64)
    z = np.zeros(4, np.complex128)
    I64 = ctypes.POINTER(ctypes.c_int64)
    zp = z.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    host = L.FLT_FLAG_HOST_ONLY
    assert lib.flt_plan_create_batch(ctypes.byref(ptr), 0, N.ctypes.data_as(I64), M.ctypes.data_as(I64), zp,
                                     1e-6, 1, host) == -1
    assert lib.flt_plan_create_batch(ctypes.byref(ptr), 2, None, M.ctypes.data_as(I64), zp, 1e-6, 1, host) == -1
    z[3] = -1j                                   # Im z < 0 in the second member
    assert lib.flt_plan_create_batch(ctypes.byref(ptr), 2, N.ctypes.data_as(I64), M.ctypes.data_as(I64), zp,
                                     1e-6, 1, host) == -2
    assert lib.flt_plan_create_batch(ctypes.byref(ptr), 2, N.ctypes.data_as(I64), M.ctypes.data_as(I64), zp,
                                     1e-6, 1, 1 << 7) == -1


def test_autotune_flag_on_host_only_plans_keeps_the_default_policy():
    rng = np.random.default_rng(4)
    z = inputs.nodes_disk(rng, 500)
    p = flt.Plan(3000, z, 1e-6, "complex64", host_only=True, autotune=True)
    q = flt.Plan(3000, z, 1e-6, "complex64", host_only=True)
    assert p.info()["direct_scale"] == 1.0
    assert p.bands() == q.bands()


def test_fixed_band_policy():
    """flt_plan_create_policy rebuilds a plan with the given band-policy
    factor: the factor is reported, a larger factor never makes fewer bands
    direct (the direct-sum cost is divided by it), factor 1 equals the default
    plan, and invalid factors or the tuning flag are refused."""
    rng = np.random.default_rng(5)
    z = np.concatenate([inputs.nodes_disk(rng, 3000), inputs.nodes_annulus(rng, 300)])
    base = flt.Plan(70000, z, 1e-6, "complex64", host_only=True)
    prev = None
    for sc in (0.0, 0.5, 1.0, 2.0, 8.0):
        p = flt.Plan(70000, z, 1e-6, "complex64", host_only=True, direct_scale=sc)
        assert p.info()["direct_scale"] == sc
        direct = [b["direct"] for b in p.bands()]
        if prev is not None:
            assert all(d >= e for d, e in zip(direct, prev))
        prev = direct
        if sc == 1.0:
            assert p.bands() == base.bands()
        p.close()
    lib = L.load()
    ptr = ctypes.c_void_p()
    zz = np.ascontiguousarray(z.astype(np.complex128))
    zp = zz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for sc, flags in ((-1.0, L.FLT_FLAG_HOST_ONLY), (float("nan"), L.FLT_FLAG_HOST_ONLY),
                      (float("inf"), L.FLT_FLAG_HOST_ONLY), (1.0, L.FLT_FLAG_HOST_ONLY | L.FLT_FLAG_AUTOTUNE)):
        assert lib.flt_plan_create_policy(ctypes.byref(ptr), 70000, len(z), zp, 1e-6, 1, flags, sc) == -1   # FLT_EINVAL
        assert not ptr.value
    with pytest.raises(ValueError):
        flt.Plan(70000, z, 1e-6, "complex64", host_only=True, autotune=True, direct_scale=2.0)


def test_binding_checks_outputs():
    """The binding rejects an output tensor that does not match the plan
    (type, size, device) or is not contiguous, before anything reaches the
    kernels (which write through the output's data pointer)."""
    import torch

    from paper_1606_03255_amd import plan as P
    dev = torch.device("cpu")
    ok = torch.zeros(6, dtype=torch.complex64)
    assert P._check_out(ok, 6, "out", torch.complex64, dev) is ok
    with pytest.raises(TypeError):
        P._check_out(ok, 6, "out", torch.complex128, dev)
    with pytest.raises(ValueError):
        P._check_out(ok, 5, "out", torch.complex64, dev)
    with pytest.raises(ValueError):
        P._check_out(torch.zeros(12, dtype=torch.complex64)[::2], 6, "out", torch.complex64, dev)
    with pytest.raises(ValueError):
        P._check_out(ok, 6, "out", torch.complex64, torch.device("cuda", 0))
    with pytest.raises(TypeError):
        P._check_out(np.zeros(6, np.complex64), 6, "out", torch.complex64, dev)
    # inputs may be strided (a contiguous copy is passed on)
    assert P._check_tensor(torch.zeros(12, dtype=torch.complex64)[::2], 6, "c", torch.complex64, dev).numel() == 6
