"""Pins of the real-exponent oracle (eq. 4.1 with real xi_k; the transposed
evaluation g(xi) of Sect. 4) against what mathematics fixes: the integer
oracle at integer exponents, mpmath's principal power formed term by term, the
closed form of a geometric sum with real exponents in arithmetic progression,
the bilinear identity between forward and transposed, the side of the branch
cut, and |f| <= ||c||_1 on the disk."""
import numpy as np
import pytest

import oracle
from paper_1606_03255_amd import inputs

mpmath = pytest.importorskip("mpmath")


def _nodes(rng, M):
    z = inputs.nodes_disk(rng, M)
    z[0] = 0.21 + 0.0j            # on the unit circle
    z[1] = 0.4999 + 0.01j         # just above the branch cut's side x_p = 1/2
    z[2] = 0.5001 + 0.02j         # just below it (x_p = -0.4999)
    z[3] = -0.3 + 0.05j           # Re z outside [0, 1)
    return z


def test_integer_exponents_equal_the_integer_oracle():
    rng = np.random.default_rng(31)
    N, M = 300, 120
    c = inputs.coefficients(rng, N)
    z = _nodes(rng, M)
    k = np.arange(N, dtype=np.float64)
    ref = oracle.forward(c, z)
    assert np.abs(oracle.forward_xi(c, k, z) - ref).max() <= 1e-14 * np.abs(c).sum()
    g = inputs.coefficients(rng, M)
    # sum_j g_j w_j^k = conj(sum_j conj(g_j) conj(w_j)^k), the conjugated adjoint
    adj = np.conj(oracle.adjoint(np.conj(g), z, N))
    assert np.abs(oracle.transposed_xi(g, z, k) - adj).max() <= 1e-14 * np.abs(g).sum()


def test_mpmath_principal_power_tiny():
    rng = np.random.default_rng(32)
    mpmath.mp.dps = 40
    N, M = 23, 17
    xi = inputs.exponents(rng, N, 1.0, 40.0)
    c = inputs.coefficients(rng, N)
    z = _nodes(rng, M)
    got = oracle.forward_xi(c, xi, z)
    for j in range(M):
        w = mpmath.exp(2j * mpmath.pi * mpmath.mpc(float(z[j].real), float(z[j].imag)))
        ref = sum(mpmath.mpc(complex(c[k])) * mpmath.power(w, mpmath.mpf(float(xi[k]))) for k in range(N))
        assert abs(complex(ref) - got[j]) <= 2e-15 * np.abs(c).sum(), j
    g = inputs.coefficients(rng, M)
    h = oracle.transposed_xi(g, z, xi)
    for k in range(N):
        ref = sum(mpmath.mpc(complex(g[j])) * mpmath.power(
            mpmath.exp(2j * mpmath.pi * mpmath.mpc(float(z[j].real), float(z[j].imag))), mpmath.mpf(float(xi[k])))
            for j in range(M))
        assert abs(complex(ref) - h[k]) <= 2e-15 * np.abs(g).sum(), k


def test_geometric_closed_form_real_progression():
    # sum_{k<N} w^{a + k d} = w^a (1 - w^{N d}) / (1 - w^d) with principal
    # powers w^p = exp(p Log w), Log w from numpy's principal complex log
    rng = np.random.default_rng(33)
    N = 500
    a, d = 1.37, 0.731
    xi = a + d * np.arange(N)
    c = np.ones(N, np.complex128)
    z = _nodes(rng, 60)
    z = z[np.imag(z) > 1e-3]      # |1 - w^d| away from 0
    logw = np.log(np.exp(2j * np.pi * z))
    wa, wd, wnd = np.exp(a * logw), np.exp(d * logw), np.exp(N * d * logw)
    ref = wa * (1 - wnd) / (1 - wd)
    got = oracle.forward_xi(c, xi, z)
    assert np.abs(got - ref).max() <= 1e-12 * N


def test_branch_side():
    # Re z = 1/2 (and -1/2): x_p = +1/2, so w^xi = e^{-xi y} e^{i pi xi}
    xi = np.array([1.25, 2.5, 7.75])
    c = np.array([1.0, 0.0, 0.0], np.complex128)
    for re in (0.5, -0.5, 2.5):
        z = np.array([re + 0.03j])
        y = 2 * np.pi * 0.03
        for k in range(3):
            ck = np.zeros(3, np.complex128)
            ck[k] = 1
            got = oracle.forward_xi(ck, xi, z)[0]
            ref = np.exp(-xi[k] * y) * np.exp(1j * np.pi * xi[k])
            assert abs(got - ref) <= 1e-15, (re, k)


def test_bilinear_identity_and_bound():
    rng = np.random.default_rng(34)
    N, M = 400, 350
    xi = inputs.exponents(rng, N)
    c = inputs.coefficients(rng, N)
    g = inputs.coefficients(rng, M)
    z = _nodes(rng, M)
    f = oracle.forward_xi(c, xi, z)
    h = oracle.transposed_xi(g, z, xi)
    lhs, rhs = np.sum(g * f), np.sum(c * h)
    assert abs(lhs - rhs) <= 1e-12 * np.abs(c).sum() * np.abs(g).sum()
    assert np.all(np.abs(f) <= np.abs(c).sum() * (1 + 1e-14))


def test_far_nodes_vanish():
    # Im z = +inf: w = 0 and every term w^xi (xi >= 1) is 0
    xi = np.array([1.0, 2.5])
    c = np.array([1 + 1j, 2.0])
    z = np.array([complex(0.3, np.inf)])
    assert oracle.forward_xi(c, xi, z)[0] == 0
