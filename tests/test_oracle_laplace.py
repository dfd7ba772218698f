"""Pins of the Laplace-transform oracle (Sect. 3, Algorithm 1, Thm A.3)
against facts other than its own formulas: a closed-form geometric sum, the
hot path's pinned oracle at x = 0 (eq. 4.2 with Re z = 0), exact cases of the
approximant, and the error bound of Thm A.3 against the direct sums; the
K_{1/2} kernel of Thm 3.3's example against the library's kv, its integral
definition and mpmath."""
import numpy as np
import pytest

import oracle
from oracle import laplace as LP


def test_direct_geometric_closed_form():
    # sum_{k=1}^{N} exp(-k y) = e^{-y} (1 - e^{-N y}) / (1 - e^{-y})
    N = 500
    xi = np.arange(1, N + 1, dtype=np.float64)
    y = np.array([1e-4, 0.01, 0.3, 2.0, 7.5])
    got = LP.direct(np.ones(N), xi, y)
    ref = np.exp(-y) * -np.expm1(-N * y) / -np.expm1(-y)
    assert np.allclose(got.real, ref, rtol=1e-13, atol=0) and np.all(got.imag == 0)


def test_direct_is_the_polynomial_at_x_zero():
    # integer xi_k = k: sum_k c_k exp(-k y) = sum_k c_k w^k with w = exp(2 pi i z), z = i y / (2 pi)
    rng = np.random.default_rng(3)
    N, M = 300, 40
    c = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = rng.random(M) * 0.2
    z = 1j * y / (2 * np.pi)
    got = LP.direct(c, np.arange(N, dtype=np.float64), y)
    assert np.abs(got - oracle.forward(c, z)).max() <= 1e-12 * np.abs(c).sum()


def test_all_nodes_at_zero_give_the_coefficient_sum():
    rng = np.random.default_rng(4)
    fhat = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    xi = rng.random(50) * 100 + 0.1
    got = LP.alg1(fhat, xi, np.zeros(7), 1e-8)
    assert np.all(got == fhat.sum())


def test_levels_partition_the_intervals():
    # every value lands in the dyadic interval of Def. 3.2 that holds it
    v1, M = 10.0, 12
    for v in [10.0, 5.0, 5.0000001, 4.9999999, 1e-3, 10 * 2.0 ** -11, 10 * 2.0 ** -10, 0.0]:
        i = LP.level(v, v1, M)
        if i == M:
            assert v <= v1 * 2.0 ** (1 - M)
        else:
            assert v1 * 2.0 ** -i < v <= v1 * 2.0 ** (1 - i)


@pytest.mark.parametrize("eps", [1e-4, 1e-8, 1e-12])
@pytest.mark.parametrize("kind", ["integer", "random"])
def test_alg1_meets_theorem_a3(eps, kind):
    rng = np.random.default_rng(int(-np.log10(eps)) + (kind == "random"))
    N, M = 1200, 700
    if kind == "integer":
        xi = np.arange(1, N + 1, dtype=np.float64)
    else:
        xi = rng.random(N) * 5000.0 + 1e-3
    fhat = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = np.concatenate([rng.random(M - 6) * 0.05, [0.0, 0.05, 0.025, 0.0125, 1e-9, 0.05 * 2.0 ** -20]])
    E = np.abs(LP.alg1(fhat, xi, y, eps) - LP.direct(fhat, xi, y)).max() / np.abs(fhat).sum()
    assert E <= eps


def test_alg1_dropping_a_part_fails():
    # the approximant needs each of its three parts: without the "kernel = 1"
    # blocks (g_{L_m+1}) the bound breaks on inputs whose low frequencies dominate
    rng = np.random.default_rng(8)
    N, M, eps = 800, 300, 1e-8
    xi = np.concatenate([rng.random(N - 50) * 2000 + 1.0, rng.random(50) * 1e-6])
    fhat = np.ones(N, np.complex128)
    y = rng.random(M) * 0.5
    tr = {}
    f = LP.alg1(fhat, xi, y, eps, trace=tr)
    ref = LP.direct(fhat, xi, y)
    assert np.abs(f - ref).max() <= eps * N
    P, g, band = tr["P"], tr["g"], tr["band"]
    broken = f.copy()
    for j in range(M):
        m = band[j]
        if m < P["M"]:
            broken[j] -= g[P["Lm"][m] + 1]
    assert np.abs(broken - ref).max() > 1e3 * eps * N


# ---- the asymptotically smooth kernel of Thm 3.3's example
def test_bessel_k_half_closed_form_is_the_library_kv():
    scipy_special = pytest.importorskip("scipy.special")
    x = np.geomspace(1e-8, 40.0, 200)
    ref = scipy_special.kv(0.5, x)
    assert np.allclose(LP.bessel_k_half(x), ref, rtol=1e-13, atol=0)


def test_bessel_k_half_closed_form_is_the_integral_definition():
    # K_eta(x) = int_0^inf exp(-x cosh t) cosh(eta t) dt, eta = 1/2 (the paper's definition)
    integrate = pytest.importorskip("scipy.integrate")
    for x in (0.01, 0.3, 1.0, 2.5, 7.0):
        top = np.arccosh(750.0 / x)   # beyond it the integrand is below e^-750
        val, err = integrate.quad(lambda t: np.exp(-x * np.cosh(t)) * np.cosh(0.5 * t), 0, top, limit=400)
        assert abs(val - LP.bessel_k_half(x)) <= 1e-10 * val


def test_direct_kernel_mpmath_tiny():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    rng = np.random.default_rng(41)
    xi = rng.random(9) * 20 + 1e-3
    y = rng.random(7) * 0.5 + 1e-4
    fh = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    got = LP.direct_kernel(fh, xi, y, "bessel_k_half")
    for j in range(len(y)):
        ref = sum(mpmath.mpc(complex(fh[k])) * mpmath.besselk(0.5, mpmath.mpf(float(y[j])) * mpmath.mpf(float(xi[k])))
                  for k in range(len(xi)))
        assert abs(complex(ref) - got[j]) <= 1e-14 * np.abs(fh).sum() * float(LP.bessel_k_half(y[j] * xi.min()))


def test_direct_kernel_exp_is_direct():
    rng = np.random.default_rng(42)
    xi = rng.random(50) * 50
    y = rng.random(30)
    fh = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    assert np.array_equal(LP.direct_kernel(fh, xi, y, "exp"), LP.direct(fh, xi, y))
