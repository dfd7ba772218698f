"""Real exponents on the CPU build of the kernel bodies (the same work lists,
tables and inner batched plan as the GPU launches) against the real-exponent
oracle: forward, transposed g(xi) and adjoint, bars eps * ||input||_1."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_1606_03255_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EMU = os.environ.get("FLT_EMU_LIB", os.path.join(ROOT, "paper_1606_03255_amd", "libflt_emu.so"))


@pytest.fixture(scope="module")
def emu():
    if not os.path.exists(EMU):
        from paper_1606_03255_amd import build
        build.build_emu()
    os.environ.setdefault("OMP_WAIT_POLICY", "passive")
    lib = ctypes.CDLL(EMU)
    lib.flt_emu_xi.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double,
                               ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def run(lib, xi, z, eps, dt, op, x):
    xi = np.ascontiguousarray(xi, np.float64)
    z = np.ascontiguousarray(z, np.complex128)
    ct = np.complex64 if dt == 1 else np.complex128
    inp = np.ascontiguousarray(x, ct)
    out = np.zeros(len(z) if op == 0 else len(xi), ct)
    rc = lib.flt_emu_xi(len(xi), xi.ctypes.data, len(z), z.ctypes.data, eps, dt, op, inp.ctypes.data,
                        out.ctypes.data)
    assert rc == 0, rc
    return out.astype(np.complex128)


def _case(rng, N, M, hi=None):
    xi = inputs.exponents(rng, N, 1.0, hi)
    xi[0] = 1.0                       # the smallest exponent allowed
    xi[1] = xi[2] = 0.5 * (1 + xi[3])  # repeated exponents
    xi[4] = float(int(xi[4]))         # an integer one
    z = np.concatenate([inputs.nodes_disk(rng, M // 2), inputs.nodes_annulus(rng, M - M // 2)])
    z[0] = complex(0.3, np.inf)       # w = 0
    z[1] = 0.999999999 + 0j           # on the circle, just left of the cut's side
    z[2] = 0.5 + 0.001j               # Re z = 1/2: x_p = +1/2
    z[3] = -0.25 + 0j                 # Re z outside [0, 1)
    return xi, z


# N exponents in [1, N] (or [1, hi]), M nodes, eps, dtype (1 = c64, 2 = c128)
CASES = [(200, 300, 1e-6, 1, None), (200, 300, 1e-10, 2, None), (3000, 500, 1e-9, 2, None),
         (5000, 2000, 1e-6, 1, None), (1, 40, 1e-8, 2, None), (600, 400, 1e-6, 1, 20000.0),
         (2500, 6000, 1e-11, 2, None)]


@pytest.mark.parametrize("N,M,eps,dt,hi", CASES)
def test_cpu_xi_vs_oracle(emu, N, M, eps, dt, hi):
    rng = np.random.default_rng(N + 7 * M)
    xi, z = _case(rng, N, M, hi) if N > 4 else (np.array([2.75]), inputs.nodes_disk(rng, M))
    c = inputs.coefficients(rng, N)
    g = inputs.coefficients(rng, M)
    if dt == 1:
        c = c.astype(np.complex64).astype(np.complex128)
        g = g.astype(np.complex64).astype(np.complex128)
    f = run(emu, xi, z, eps, dt, 0, c)
    assert np.abs(f - oracle.forward_xi(c, xi, z)).max() <= eps * np.abs(c).sum()
    h = run(emu, xi, z, eps, dt, 1, g)
    assert np.abs(h - oracle.transposed_xi(g, z, xi)).max() <= eps * np.abs(g).sum()
    ha = run(emu, xi, z, eps, dt, 2, g)
    ref = np.conj(oracle.transposed_xi(np.conj(g), z, xi))
    assert np.abs(ha - ref).max() <= eps * np.abs(g).sum()
