"""The asymptotically smooth kernel of Thm 3.3's example, K_{1/2}(y xi), on
the CPU build of the Laplace kernel bodies against the oracle's direct sums.
Bar: |f_j - f~_j| <= eps sum_k |fhat_k| max(1, K_{1/2}(y_j xi_k / 4)) (the
block-relative reading of the theorem's per-block condition; the planner's
target is half of it)."""
import ctypes
import os

import numpy as np
import pytest

from oracle import laplace as LP
from paper_1606_03255_amd import LaplacePlan

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.environ.get("FLT_EMU_LIB", os.path.join(os.path.dirname(HERE), "paper_1606_03255_amd", "libflt_emu.so"))


@pytest.fixture(scope="module")
def emu():
    if not os.path.exists(EMU):
        from paper_1606_03255_amd import build
        build.build_emu()
    lib = ctypes.CDLL(EMU)
    lib.flt_emu_laplace_kernel.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_void_p]
    return lib


def run(lib, fhat, xi, y, eps, dt):
    ct = np.complex64 if dt == 1 else np.complex128
    xi = np.ascontiguousarray(xi, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    inp = np.ascontiguousarray(fhat, ct)
    out = np.zeros(len(y), ct)
    rc = lib.flt_emu_laplace_kernel(1, len(xi), xi.ctypes.data, len(y), y.ctypes.data, eps, dt, inp.ctypes.data,
                                    out.ctypes.data)
    assert rc == 0, rc
    return out.astype(np.complex128)


def bar(fhat, xi, y, eps):
    """eps sum_k |fhat_k| max(1, K_{1/2}(y_j xi_k / 4)), per node."""
    w = np.maximum(1.0, LP.bessel_k_half(np.outer(y, xi) / 4.0))
    return eps * (w @ np.abs(fhat))


def case(seed, N, M, near=True):
    rng = np.random.default_rng(seed)
    xi = rng.random(N) * N + 1e-3
    y = rng.random(M) * (20.0 / N) + 1e-9
    if near and N > 4 and M > 4:
        xi[:3] = [1e-12, 3e-11, 1e-9]          # the near field Omega_M
        y[:3] = [1e-18, 4e-17, 2e-15]          # nodes of Y_M (summed directly)
        y[3] = 20.0 / N                        # y_1 itself
    fhat = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    return fhat, xi, y


@pytest.mark.parametrize("N,M,eps,dt", [(1000, 700, 1e-6, 1), (1000, 700, 1e-10, 2), (3000, 2000, 1e-12, 2),
                                        (5000, 300, 1e-6, 1), (1, 5, 1e-8, 2), (300, 1, 1e-9, 2)])
def test_k12_cpu_build_vs_direct(emu, N, M, eps, dt):
    fhat, xi, y = case(N + M, N, M)
    if dt == 1:
        fhat = fhat.astype(np.complex64).astype(np.complex128)
    f = run(emu, fhat, xi, y, eps, dt)
    ref = LP.direct_kernel(fhat, xi, y, "bessel_k_half")
    err = np.abs(f - ref)
    assert np.all(err <= bar(fhat, xi, y, eps)), (err / bar(fhat, xi, y, eps)).max()


def test_k12_plan_parameters():
    fhat, xi, y = case(5, 4096, 100, near=False)
    info = LaplacePlan(xi, y, 1e-8, "complex128", host_only=True, kernel="bessel_k_half").info()
    y1, xi1 = y.max(), xi.max()
    assert info["kernel"] == 1
    assert info["levels"] == int(np.ceil(np.log2(y1 * xi1 * 4096 / 1e-8))) + 1   # Thm 3.3's M
    assert 2 <= info["q"] <= 32


def test_k12_rejects_a_node_at_zero():
    from paper_1606_03255_amd._lib import FltError
    with pytest.raises(FltError):
        LaplacePlan(np.array([1.0, 2.0]), np.array([0.0, 0.1]), 1e-6, "complex128", host_only=True,
                    kernel="bessel_k_half")
    with pytest.raises(ValueError):
        LaplacePlan(np.array([1.0]), np.array([0.1]), 1e-6, "complex128", host_only=True, kernel="nope")
