"""The Laplace transform (Sect. 3, Algorithm 1) without a GPU: the planner's
parameters against the oracle's reading of Def. 3.2, the kernel bodies built
for the CPU against the oracle (Algorithm 1 step by step: the same
approximation up to rounding; the direct sums: Thm A.3's bound), and the
C ABI's argument checks."""
import ctypes
import os

import numpy as np
import pytest

from oracle import laplace as LP
from paper_1606_03255_amd import LaplacePlan
from paper_1606_03255_amd import _lib as L

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.environ.get("FLT_EMU_LIB", os.path.join(os.path.dirname(HERE), "paper_1606_03255_amd", "libflt_emu.so"))


@pytest.fixture(scope="module")
def emu():
    if not os.path.exists(EMU):
        from paper_1606_03255_amd import build
        build.build_emu()
    lib = ctypes.CDLL(EMU)
    lib.flt_emu_laplace.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def run(lib, fhat, xi, y, eps, dt):
    ct = np.complex64 if dt == 1 else np.complex128
    xi = np.ascontiguousarray(xi, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    inp = np.ascontiguousarray(fhat, ct)
    out = np.zeros(len(y), ct)
    rc = lib.flt_emu_laplace(len(xi), xi.ctypes.data, len(y), y.ctypes.data, eps, dt, inp.ctypes.data,
                             out.ctypes.data)
    assert rc == 0
    return out.astype(np.complex128)


def _case(seed, N, M, kind):
    rng = np.random.default_rng(seed)
    if kind == "integer":
        xi = np.arange(1, N + 1, dtype=np.float64)
    elif kind == "clustered":   # most frequencies in one block: several chunks per block
        xi = np.concatenate([900.0 + 100.0 * rng.random(N - 10), rng.random(10) * 1e-3 + 1e-6])
    else:
        xi = rng.random(N) * 3000.0 + 1e-4
    y = np.concatenate([rng.random(max(M - 4, 0)) * 0.02, [0.0, 0.02, 1e-12, 0.01]])[:M]
    fhat = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return fhat, xi, y


@pytest.mark.parametrize("N,M,eps", [(1000, 300, 1e-8), (4097, 777, 1e-12), (1, 5, 1e-6), (300, 1, 1e-10)])
def test_plan_parameters_match_definition_3_2(N, M, eps):
    fhat, xi, y = _case(N + M, N, M, "random")
    info = LaplacePlan(xi, y, eps, "complex128", host_only=True).info()
    P = LP.params(xi, y, eps)
    assert (info["q"], info["levels"]) == (P["q"], P["M"])
    assert info["y1"] == P["y1"] and info["xi1"] == P["xi1"]


@pytest.mark.parametrize("kind", ["integer", "random", "clustered"])
@pytest.mark.parametrize("eps,dt", [(1e-12, 2), (1e-8, 2), (1e-6, 1)])
def test_cpu_build_vs_oracle(emu, kind, eps, dt):
    fhat, xi, y = _case(7 + (kind == "random"), 5000, 900, kind)
    if dt == 1:
        fhat = fhat.astype(np.complex64).astype(np.complex128)
    got = run(emu, fhat, xi, y, eps, dt)
    n1 = np.abs(fhat).sum()
    assert np.abs(got - LP.direct(fhat, xi, y)).max() <= eps * n1
    if dt == 2:   # the same approximant as Algorithm 1 step by step, up to rounding
        assert np.abs(got - LP.alg1(fhat, xi, y, eps)).max() <= 1e-13 * n1


def test_cpu_build_edge_cases(emu):
    rng = np.random.default_rng(11)
    eps = 1e-10
    # all nodes at 0: exactly the coefficient sum
    fhat = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    xi = rng.random(50) * 10 + 0.5
    got = run(emu, fhat, xi, np.zeros(9), eps, 2)
    assert np.abs(got - fhat.sum()).max() <= 1e-14 * np.abs(fhat).sum()
    # nodes and frequencies exactly on Chebyshev nodes (the Lagrange form's removable singularities)
    N, M = 400, 60
    fhat = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    xi = rng.random(N) * 100 + 1.0
    y = rng.random(M) * 0.05
    tr = {}
    LP.alg1(fhat, xi, y, eps, trace=tr)
    P = tr["P"]
    from oracle.method import interval_nodes
    xi[:3] = interval_nodes(P["xi1"] * 2.0 ** -2, P["xi1"] * 2.0 ** -1, P["q"])[:3]
    y[:2] = interval_nodes(P["y1"] * 2.0 ** -3, P["y1"] * 2.0 ** -2, P["q"])[:2]
    got = run(emu, fhat, xi, y, eps, 2)
    n1 = np.abs(fhat).sum()
    assert np.abs(got - LP.direct(fhat, xi, y)).max() <= eps * n1
    assert np.abs(got - LP.alg1(fhat, xi, y, eps)).max() <= 1e-13 * n1
    # one frequency, one node
    got = run(emu, np.array([2 - 1j]), np.array([3.0]), np.array([0.25]), eps, 2)
    assert abs(got[0] - (2 - 1j) * np.exp(-0.75)) <= eps * abs(2 - 1j)


def _wide(seed, N, M):
    # frequencies and nodes over many decades (most products y xi far past
    # exp underflow): q = 24 and L > 160 at eps = 1e-14, so the node kernel
    # reads its band data from global memory (too large to stage in LDS)
    rng = np.random.default_rng(seed)
    xi = 10.0 ** rng.uniform(-3, 19, N)
    y = np.concatenate([[0.0], 10.0 ** rng.uniform(-20, 17, M - 1)])
    fhat = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return fhat, xi, y


def test_cpu_build_wide_range(emu):
    fhat, xi, y = _wide(3, 2000, 700)
    eps = 1e-14
    info = LaplacePlan(xi, y, eps, "complex128", host_only=True).info()
    assert 2 * info["levels"] * info["q"] + 2 * info["levels"] > 8192
    got = run(emu, fhat, xi, y, eps, 2)
    n1 = np.abs(fhat).sum()
    assert np.abs(got - LP.direct(fhat, xi, y)).max() <= eps * n1
    assert np.abs(got - LP.alg1(fhat, xi, y, eps)).max() <= 1e-13 * n1


def test_abi_argument_checks():
    lib = L.load()
    ptr = ctypes.c_void_p()
    D = ctypes.POINTER(ctypes.c_double)

    def create(xi, y, eps=1e-8, dt=2, flags=L.FLT_FLAG_HOST_ONLY):
        xi = np.ascontiguousarray(xi, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        rc = lib.flt_laplace_plan_create(ctypes.byref(ptr), len(xi), xi.ctypes.data_as(D), len(y),
                                         y.ctypes.data_as(D), eps, dt, flags)
        if rc == 0:
            lib.flt_laplace_plan_destroy(ptr)
        return rc

    ok_x, ok_y = np.array([1.0, 2.0]), np.array([0.0, 0.5])
    assert create(ok_x, ok_y) == 0
    assert create(np.array([1.0, 0.0]), ok_y) == -2          # xi <= 0
    assert create(np.array([1.0, np.inf]), ok_y) == -2
    assert create(ok_x, np.array([-1e-9, 0.5])) == -2        # y < 0
    assert create(ok_x, np.array([np.nan, 0.5])) == -2
    assert create(ok_x, ok_y, eps=1.5) == -2
    assert create(ok_x, ok_y, eps=1e-9, dt=1) == -3          # below the complex64 floor
    assert create(ok_x, ok_y, dt=3) == -1
    assert create(ok_x, ok_y, flags=L.FLT_FLAG_GRAPH) == -1  # only HOST_ONLY is a Laplace flag
    assert lib.flt_laplace_plan_create(None, 2, ok_x.ctypes.data_as(D), 2, ok_y.ctypes.data_as(D), 1e-8, 2, 1) == -1
    xi = np.ascontiguousarray(ok_x)
    y = np.ascontiguousarray(ok_y)
    assert lib.flt_laplace_plan_create(ctypes.byref(ptr), 2, xi.ctypes.data_as(D), 2, y.ctypes.data_as(D), 1e-8,
                                       2, L.FLT_FLAG_HOST_ONLY) == 0
    dummy = ctypes.c_void_p(16)
    assert lib.flt_laplace_forward(ptr, dummy, dummy, None) == -6   # host-only plan
    assert lib.flt_laplace_forward(ptr, None, dummy, None) == -1
    lib.flt_laplace_plan_destroy(ptr)
    lib.flt_laplace_plan_destroy(None)
