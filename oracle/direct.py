"""ORACLE (test infrastructure only): ctypes binding of ``direct.c``.

The plain FP64 definition of the exponential sums (eq. 4.1 with xi_k = k and
the polar form eq. 4.2); see the header of ``direct.c`` for the method and its
error (<~ 1.5e-14 * ||c||_1).  The shared library is compiled from source on
first use (gcc, OpenMP) or by ``build()``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile ``direct.c`` into ``liboracle.so`` (FMA required for the
    error-free products; contraction of other expressions is disabled so the
    compensated sums stay error-free)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-mfma", "-mavx2",
           "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        for name in ("oracle_forward", "oracle_derivative", "oracle_adjoint", "oracle_horner_comp"):
            fn = getattr(lib, name)
            fn.argtypes = [i64, i64, dp, dp, dp]
            fn.restype = None
        lib.oracle_forward_xi.argtypes = [i64, dp, dp, i64, dp, dp]
        lib.oracle_forward_xi.restype = None
        lib.oracle_transposed_xi.argtypes = [i64, dp, dp, i64, dp, dp]
        lib.oracle_transposed_xi.restype = None
        lib.oracle_adjoint_blocks.argtypes = [i64, i64, dp, dp, i64, ctypes.POINTER(ctypes.c_int64), dp]
        lib.oracle_adjoint_blocks.restype = None
        lib.oracle_block_size.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _c128(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_z(z):
    z = _c128(z)
    if np.any(np.imag(z) < 0) or np.any(np.isnan(z)):
        raise ValueError("nodes must satisfy Im z >= 0 (|w| <= 1) and be free of NaN")
    return z


def forward(c, z):
    """f_j = sum_{k<N} c_k exp(2 pi i k z_j), FP64."""
    c = _c128(c)
    z = _check_z(z)
    f = np.empty(z.shape[0], np.complex128)
    load().oracle_forward(c.shape[0], z.shape[0], _ptr(c), _ptr(z), _ptr(f))
    return f


def derivative(c, z):
    """f'(z_j) = sum_{k<N} 2 pi i k c_k exp(2 pi i k z_j), FP64."""
    c = _c128(c)
    z = _check_z(z)
    f = np.empty(z.shape[0], np.complex128)
    load().oracle_derivative(c.shape[0], z.shape[0], _ptr(c), _ptr(z), _ptr(f))
    return f


def adjoint(g, z, N):
    """h_k = sum_j g_j conj(exp(2 pi i k z_j)), k < N, FP64."""
    g = _c128(g)
    z = _check_z(z)
    h = np.empty(int(N), np.complex128)
    load().oracle_adjoint(int(N), z.shape[0], _ptr(g), _ptr(z), _ptr(h))
    return h


def adjoint_blocks(g, z, N, blocks):
    """The adjoint h_k = sum_j g_j conj(exp(2 pi i k z_j)) on whole blocks of
    consecutive k only (block b: k = B b .. B b + B - 1, B = block_size(),
    k < N), for sizes where all N coefficients would take too long.  Returns
    (k, h_k) as two arrays, blocks in the order given."""
    g = _c128(g)
    z = _check_z(z)
    blocks = np.ascontiguousarray(np.asarray(blocks, dtype=np.int64).reshape(-1))
    B = block_size()
    if np.any(blocks < 0) or np.any(blocks * B >= int(N)):
        raise ValueError("block outside 0 .. ceil(N / %d) - 1" % B)
    h = np.empty(len(blocks) * B, np.complex128)
    load().oracle_adjoint_blocks(int(N), z.shape[0], _ptr(g), _ptr(z), len(blocks),
                                 blocks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(h))
    k = (blocks[:, None] * B + np.arange(B)[None, :]).reshape(-1)
    keep = k < int(N)
    return k[keep], h[keep]


def _xi(xi):
    xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float64).reshape(-1))
    if not np.all(np.isfinite(xi)):
        raise ValueError("exponents must be finite")
    return xi


def forward_xi(c, xi, z):
    """f_j = sum_k c_k w_j^{xi_k}, real exponents, principal power
    (Re z reduced to (-1/2, 1/2]), FP64 term by term."""
    c = _c128(c)
    xi = _xi(xi)
    z = _check_z(z)
    if c.shape[0] != xi.shape[0]:
        raise ValueError("c and xi differ in length")
    f = np.empty(z.shape[0], np.complex128)
    load().oracle_forward_xi(xi.shape[0], _ptr(xi), _ptr(c), z.shape[0], _ptr(z), _ptr(f))
    return f


def transposed_xi(g, z, xi):
    """h_k = sum_j g_j w_j^{xi_k} (the transposed evaluation g(xi) of Sect. 4),
    principal power, FP64 term by term."""
    g = _c128(g)
    z = _check_z(z)
    xi = _xi(xi)
    if g.shape[0] != z.shape[0]:
        raise ValueError("g and z differ in length")
    h = np.empty(xi.shape[0], np.complex128)
    load().oracle_transposed_xi(z.shape[0], _ptr(z), _ptr(g), xi.shape[0], _ptr(xi), _ptr(h))
    return h


def block_size():
    return int(load().oracle_block_size())


def horner(c, z):
    """Compensated Horner on the rounded w_j (cross-check; N <~ 1e3)."""
    c = _c128(c)
    z = _check_z(z)
    f = np.empty(z.shape[0], np.complex128)
    load().oracle_horner_comp(c.shape[0], z.shape[0], _ptr(c), _ptr(z), _ptr(f))
    return f


def num_threads():
    return int(load().oracle_num_threads())
