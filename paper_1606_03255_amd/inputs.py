"""Seeded synthetic workloads for the Fourier-Laplace transform.

This module only draws random numbers; it holds none of the transform's
arithmetic, so both the GPU path and the CPU oracle can be fed from it.

Recipe (numpy ``default_rng(seed)``, PCG64, fixed draw order):

* coefficients: one ``standard_normal((N, 2))`` draw, column 0 = Re, 1 = Im;
* nodes: ``x = random(M)`` then ``U = random(M)``;
  - disk, uniform by area: r = sqrt(1 - U) in (0, 1];
  - annulus 1 - 1e-3 < r <= 1, uniform by area: r^2 = 1 - U (1 - r0^2);
  - Im z = -ln(r) / (2 pi) = -log1p(r^2 - 1) / (4 pi), Re z = x;
  so w = exp(2 pi i z) = r e^{2 pi i x} lies in the closed unit disk.

Named workloads (N coefficients, M nodes):

  ``small``      N = M = 256, disk, complex128, eps 1e-10                     (seed 1)
  ``medium``     N = M = 2^14, disk, complex128 (FP32 form rounds to c64)    (seed 2)
  ``large``      N = M = 2^20, first M/2 annulus then M/2 disk, c64          (seed 3)
  ``batched``    512 instances, N_i, M_i = floor(2^{8 + 8U}), disk, c64      (seed 4)
  ``grad``       N = M = 2^18, disk, c64, targets t_j ~ CN(0, 1)             (seed 5)
  ``xi``         N = M = 2^16 (``log2n`` to change), real exponents uniform in
                 [1, N] (one ``random(N)`` draw, unsorted), then coefficients,
                 then nodes as ``large`` (half annulus, half disk), c64    (seed 6)
"""
import numpy as np

ANNULUS_R0 = 1.0 - 1e-3
_FOUR_PI = 4.0 * np.pi


def coefficients(rng, N, dtype=np.complex128):
    a = rng.standard_normal((N, 2))
    return (a[:, 0] + 1j * a[:, 1]).astype(dtype)


def _im_from_r2m1(r2m1):
    # Im z = -ln(r)/(2 pi) = -log1p(r^2 - 1)/(4 pi); r^2 - 1 is what was drawn
    return -np.log1p(r2m1) / _FOUR_PI


def nodes_disk(rng, M):
    x = rng.random(M)
    U = rng.random(M)
    return x + 1j * _im_from_r2m1(-U)


def nodes_annulus(rng, M, r0=ANNULUS_R0):
    x = rng.random(M)
    U = rng.random(M)
    return x + 1j * _im_from_r2m1(-U * (1.0 - r0 * r0))


def exponents(rng, N, lo=1.0, hi=None):
    """N real exponents uniform in [lo, hi] (hi = N by default), unsorted."""
    hi = float(N) if hi is None else float(hi)
    return lo + (hi - lo) * rng.random(N)


def workload(name, seed=None, log2n=16):
    """Return a dict with the named workload's arrays (numpy, host)."""
    if name == "small":
        rng = np.random.default_rng(1 if seed is None else seed)
        N = M = 256
        c = coefficients(rng, N)
        z = nodes_disk(rng, M)
        return dict(name=name, N=N, M=M, c=c, z=z, eps=1e-10)
    if name == "medium":
        rng = np.random.default_rng(2 if seed is None else seed)
        N = M = 1 << 14
        c = coefficients(rng, N)
        z = nodes_disk(rng, M)
        return dict(name=name, N=N, M=M, c=c, z=z, eps64=1e-11, eps32=1e-6)
    if name == "large":
        rng = np.random.default_rng(3 if seed is None else seed)
        N = M = 1 << 20
        c = coefficients(rng, N, np.complex64)
        h = M // 2
        xa = rng.random(h)
        Ua = rng.random(h)
        xd = rng.random(M - h)
        Ud = rng.random(M - h)
        z = np.concatenate([xa + 1j * _im_from_r2m1(-Ua * (1.0 - ANNULUS_R0 ** 2)),
                            xd + 1j * _im_from_r2m1(-Ud)])
        return dict(name=name, N=N, M=M, c=c, z=z, eps32=1e-6, eps64=1e-11)
    if name == "grad":
        rng = np.random.default_rng(5 if seed is None else seed)
        N = M = 1 << 18
        c = coefficients(rng, N, np.complex64)
        z = nodes_disk(rng, M)
        t = rng.standard_normal((M, 2)) * np.sqrt(0.5)
        t = (t[:, 0] + 1j * t[:, 1]).astype(np.complex64)
        return dict(name=name, N=N, M=M, c=c, z=z, t=t, eps32=1e-6)
    if name == "batched":
        return batched(512, seed=4 if seed is None else seed)
    if name == "xi":
        rng = np.random.default_rng(6 if seed is None else seed)
        N = M = 1 << int(log2n)
        xi = exponents(rng, N)
        c = coefficients(rng, N, np.complex64)
        z = np.concatenate([nodes_annulus(rng, M // 2), nodes_disk(rng, M - M // 2)])
        return dict(name=name, N=N, M=M, xi=xi, c=c, z=z, eps32=1e-6, eps64=1e-11)
    raise KeyError(name)


def adjoint_input(M, seed=7, dtype=np.complex64):
    """Input g of the adjoint at M nodes (the gradient a backward pass would
    receive): Re, Im ~ N(0, 1/2), i.e. g_j ~ CN(0, 1)."""
    rng = np.random.default_rng(seed)
    g = (rng.standard_normal(M) + 1j * rng.standard_normal(M)) * np.sqrt(0.5)
    return g.astype(dtype)


def batched(count=512, seed=4, lo=8, hi=16):
    """``count`` independent instances, sizes log-uniform in [2^lo, 2^hi]."""
    rng = np.random.default_rng(seed)
    Ns = np.floor(2.0 ** (lo + (hi - lo) * rng.random(count))).astype(np.int64)
    Ms = np.floor(2.0 ** (lo + (hi - lo) * rng.random(count))).astype(np.int64)
    inst = []
    for i in range(count):
        c = coefficients(rng, int(Ns[i]), np.complex64)
        z = nodes_disk(rng, int(Ms[i]))
        inst.append((c, z))
    return dict(name="batched", count=count, N=Ns, M=Ms, instances=inst, eps32=1e-6)
