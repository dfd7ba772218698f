"""The kernel bodies built for the CPU (OpenMP teams with real barriers, the
same work lists and tables as the GPU launches) against the oracle: index
arithmetic, synchronisation and both band policies are checked here, before
and apart from any GPU run.  Bars as in the GPU parity tests."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from oracle import method as O
from paper_1606_03255_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# FLT_EMU_LIB selects another build of the bodies (the sanitizer run below)
EMU = os.environ.get("FLT_EMU_LIB", os.path.join(ROOT, "paper_1606_03255_amd", "libflt_emu.so"))


@pytest.fixture(scope="module")
def emu():
    if not os.path.exists(EMU):
        from paper_1606_03255_amd import build
        build.build_emu()
    os.environ.setdefault("OMP_WAIT_POLICY", "passive")
    lib = ctypes.CDLL(EMU)
    lib.flt_emu_run.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.flt_emu_run_batch.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p]
    return lib


def run(lib, x, z, eps, dt, op, N, flags):
    z = np.ascontiguousarray(z, np.complex128)
    ct = np.complex64 if dt == 1 else np.complex128
    inp = np.ascontiguousarray(x, ct)
    out = np.zeros(N if op == 2 else (2 if op == 3 else 1) * len(z), ct)   # op 3: f, then f'
    rc = lib.flt_emu_run(N, len(z), z.ctypes.data, eps, dt, flags, op, inp.ctypes.data, out.ctypes.data)
    assert rc == 0
    return out.astype(np.complex128)


# N, M, eps, dtype (1 = c64, 2 = c128): one-pass only, two-pass FFT bands, ragged N
CASES = [(300, 120, 1e-6, 1), (256, 100, 1e-10, 2), (2100, 60, 1e-9, 2), (4200, 40, 1e-6, 1), (2, 9, 1e-8, 2),
         (300, 3000, 1e-6, 1), (200, 2500, 1e-11, 2),   # these two fill low bands densely (LDS tiles)
         (70000, 40, 1e-6, 1),   # grids up to 2^18 points: pass A's output twiddles from the LDS power table
         (300, 16000, 1e-6, 1)]   # dense bands: the gather's staged runs of cells


@pytest.mark.parametrize("N,M,eps,dt", CASES)
@pytest.mark.parametrize("flags", [0, 2])
def test_cpu_build_vs_oracle(emu, N, M, eps, dt, flags):
    rng = np.random.default_rng(N + M + flags)
    c = inputs.coefficients(rng, N)
    g = inputs.coefficients(rng, M)
    if dt == 1:
        c = c.astype(np.complex64).astype(np.complex128)
        g = g.astype(np.complex64).astype(np.complex128)
    z = np.concatenate([inputs.nodes_disk(rng, M // 2), inputs.nodes_annulus(rng, M - M // 2)])
    z[0] = complex(0.3, np.inf)
    z[1] = 0.999999999 + 0j
    f = run(emu, c, z, eps, dt, 0, N, flags)
    assert np.abs(f - oracle.forward(c, z)).max() <= eps * np.abs(c).sum()
    fp = run(emu, c, z, eps, dt, 1, N, flags)
    assert np.abs(fp - oracle.derivative(c, z)).max() <= eps * np.abs(2 * np.pi * np.arange(N) * c).sum()
    h = run(emu, g, z, eps, dt, 2, N, flags)
    assert np.abs(h - oracle.adjoint(g, z, N)).max() <= eps * np.abs(g).sum()
    # forward and derivative in one pass (2q columns per band): the bars, and the
    # separate calls' values up to rounding
    ffp = run(emu, c, z, eps, dt, 3, N, flags)
    f3, fp3 = ffp[:M], ffp[M:]
    n1, n1d = np.abs(c).sum(), np.abs(2 * np.pi * np.arange(N) * c).sum()
    assert np.abs(f3 - oracle.forward(c, z)).max() <= eps * n1
    assert np.abs(fp3 - oracle.derivative(c, z)).max() <= eps * n1d
    tol = 1e-6 if dt == 1 else 1e-14
    assert np.abs(f3 - f).max() <= tol * n1
    assert np.abs(fp3 - fp).max() <= tol * n1d
    if dt == 2 and flags == 2:
        n1 = np.abs(c).sum()
        assert np.abs(f - O.alg2_forward(c, z, eps, "nfft")).max() <= 1e-13 * n1
        assert np.abs(h - O.alg2_adjoint(g, z, N, eps, "nfft")).max() <= 1e-13 * np.abs(g).sum()


def test_cpu_build_batched_equals_single_instances(emu):
    """A batched plan computes, for every member, what that member's own plan
    computes (same bands, tables and work items, offset into packed arrays);
    each member also meets the oracle bar."""
    rng = np.random.default_rng(77)
    Ns = np.array([300, 2, 4200, 1, 777, 2100], np.int64)
    Ms = np.array([120, 9, 40, 5, 300, 61], np.int64)
    eps, dt = 1e-6, 1
    zs = []
    for M in Ms:
        z = np.concatenate([inputs.nodes_disk(rng, M // 2), inputs.nodes_annulus(rng, M - M // 2)])
        z[0] = complex(0.3, np.inf)
        zs.append(z)
    cs = [inputs.coefficients(rng, N).astype(np.complex64).astype(np.complex128) for N in Ns]
    gs = [inputs.coefficients(rng, M).astype(np.complex64).astype(np.complex128) for M in Ms]
    zp = np.ascontiguousarray(np.concatenate(zs))
    co = np.concatenate([[0], np.cumsum(Ns)])
    fo = np.concatenate([[0], np.cumsum(Ms)])
    runs = [(0, op) for op in (0, 1, 2, 3)] + [(2, 0)]    # NFFT-only: forward (its sparse bands are slow here)
    for flags, op in runs:
        x, nout = (gs, Ns) if op == 2 else (cs, Ms)
        inp = np.ascontiguousarray(np.concatenate(x), np.complex64)
        out = np.zeros(int(nout.sum()) * (2 if op == 3 else 1), np.complex64)   # op 3: all f, then all f'
        rc = emu.flt_emu_run_batch(len(Ns), Ns.ctypes.data, Ms.ctypes.data, zp.ctypes.data, eps, dt, flags, op,
                                   inp.ctypes.data, out.ctypes.data)
        assert rc == 0
        oo = co if op == 2 else fo
        for part, kind in ((0, op),) if op != 3 else ((0, 0), (int(Ms.sum()), 1)):
            for i in range(len(Ns)):
                got = out[part + oo[i]:part + oo[i + 1]].astype(np.complex128)
                scale = np.abs(x[i]).sum() * (1.0 if kind != 1 else 2 * np.pi * Ns[i])
                if flags == 0:
                    single = run(emu, x[i], zs[i], eps, dt, kind, int(Ns[i]), flags)
                    assert np.abs(got - single).max() <= 1e-9 * scale, (op, kind, i)
                if kind == 0:
                    ref = oracle.forward(x[i], zs[i])
                elif kind == 1:
                    ref = oracle.derivative(x[i], zs[i])
                else:
                    ref = oracle.adjoint(x[i], zs[i], int(Ns[i]))
                assert np.abs(got - ref).max() <= eps * scale, (op, kind, i)


@pytest.mark.skipif(os.environ.get("FLT_EMU_LIB") is not None, reason="already the sanitizer run")
@pytest.mark.skipif(os.environ.get("FLT_ASAN") != "1",
                    reason="about 8 minutes (2 of them the sanitizer build); run with FLT_ASAN=1")
def test_cpu_build_under_address_sanitizer():
    """A one-pass case (complex64, band policy on), a two-pass case
    (complex128, NFFT only) and a dense case (the gather's staged runs of
    cells) of the test above, forward, derivative, adjoint and the fused call
    each, a real-exponent case and the general-kernel Laplace tests, on the
    bodies built with AddressSanitizer and UndefinedBehaviorSanitizer (every
    buffer exactly sized): any out-of-bounds access or undefined operation
    aborts the child run."""
    from paper_1606_03255_amd import build
    lib = build.build_emu(sanitize=True)
    asan = subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, FLT_EMU_LIB=lib, LD_PRELOAD=asan, OMP_WAIT_POLICY="passive",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_cpu_build.py"), os.path.join(HERE, "test_cpu_xi.py"),
                        os.path.join(HERE, "test_laplace_kernel_cpu.py"), "-k",
                        "0-300-120-1e-06-1 or 2-2100-60-1e-09-2 or 0-300-3000-1e-06-1 or 200-300-1e-06-1 or k12"],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "12 passed" in r.stdout, r.stdout[-2000:]
