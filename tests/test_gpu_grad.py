"""GPU parity of the differentiation form: the gradients of
L = sum_j |f(z_j) - t_j|^2 that the autograd Function returns,

    dL/dc   = C^H grad_f                 (the adjoint transform),
    dL/dz_j = grad_f_j conj(f'(z_j))     (the derivative transform),

with grad_f = 2 (f - t) and PyTorch's convention dL/dRe + i dL/dIm, checked
against the FP64 direct gradient and against central finite differences of
the FP64 loss.

Workload: N = M = 2^18, complex64 coefficients, nodes uniform by area in the
disk, targets t_j ~ CN(0, 1), eps = 1e-6 (the FP32 form), on the plan the
benchmark times the fwd+bwd step on (tuned on forward + adjoint); plus a tiny
FP64 case (N = 16) with h = 1e-3 in every real coordinate.

Bars, from Thm 4.3 carried through the loss (E of a transform <= eps times the
1-norm of its input):
* dL/dc against C^H applied to the grad_f the backward received:
  max|.| <= eps sum|grad_f|;
* dL/dc against the FP64 direct gradient C^H 2 (f_ex - t): that, plus
  sum |C^H (grad_f - 2 (f_ex - t))| <= 2 sum_j |f_j - f_ex_j| (|w|^k <= 1);
* dL/dz_j against 2 (f_ex - t) conj(f'_ex): |grad_f_j| eps sum|2 pi k c_k| +
  |f'_ex(z_j)| |grad_f_j - 2 (f_ex_j - t_j)|;
* a central difference of step h in a coordinate s of a function L(s) is off
  its derivative by (h^2 / 6) times L's third derivative at 0, plus O(h^4),
  plus the rounding of the two evaluations over 2 h.  For L in c the loss is
  quadratic and only rounding remains; in z the h^2 term is computed from
  f', f'', f''' at the node and the h^4 remainder is bounded with
  |d^n f / ds^n| <= A_n = sum_k (2 pi k)^n |c_k| |w|^k e^{2 pi k h} on the
  interval (|w| may grow by e^{2 pi k h} as Im z drops); see _fd_z_tolerance.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1606_03255_amd import inputs

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53
# relative error of one term c_k w^k in the oracle's direct sums: an exactly
# reduced anchor every 32 terms and at most 31 recurrence steps from it
ORACLE_TERM_ERR = 130 * U64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _autograd(torch, c, z, t, eps, tdt, autotune):
    """dL/dc, dL/dz and f through fourier_laplace (the HIP path)."""
    from paper_1606_03255_amd import Plan, fourier_laplace
    plan = Plan(len(c), z, eps, tdt, autotune=autotune)
    ct = torch.from_numpy(c).to("cuda", tdt).requires_grad_(True)
    zt = torch.from_numpy(z).to("cuda").requires_grad_(True)
    tt = torch.from_numpy(t).to("cuda", tdt)
    f = fourier_laplace(ct, zt, plan)
    loss = (f - tt).abs().pow(2).sum()
    loss.backward()
    torch.cuda.synchronize()
    out = (ct.grad.cpu().numpy().astype(np.complex128), zt.grad.cpu().numpy(),
           f.detach().cpu().numpy().astype(np.complex128), plan.info()["direct_scale"])
    plan.close()
    return out


def _loss(c, z, t):
    return float(np.sum(np.abs(oracle.forward(c, z) - t) ** 2))


def _fd_z_tolerance(c, z, t, h):
    """Per node, a bound on |FD - (dL/dRe + i dL/dIm)| for _fd_z.  Along a
    direction d (1 or i), L(s) = |F(s)|^2 with F(s) = f(z + s d) - t, and the
    central difference is L'(0) + (h^2 / 6) L3 + R with |R| <= (h^4 / 120)
    sup|L5|, L3 and L5 the third and fifth derivatives of L.  L3 at 0 is
    2 Re(F3 conj F) + 6 Re(F2 conj F1), Fn = d^n f^(n)(z) from the oracle;
    sup|L5| <= sum_a C(5, a) A_a A_(5-a) with A_n >= |f^(n)| on the interval
    (A_0 + |t| for F itself).  Plus the rounding of the two evaluations over
    2 h: the oracle's error at a node is at most ORACLE_TERM_ERR times the sum
    of its terms' moduli, sum_k |c_k| |w|^k <= A_0."""
    N = len(c)
    kk = np.arange(N, dtype=np.float64)
    fn = [oracle.forward(c * (2j * np.pi * kk) ** n, z) for n in range(4)]
    F = fn[0] - t
    ac = np.abs(c)
    tol = np.zeros(len(z))
    for j, zj in enumerate(z):
        wk = np.exp(-2 * np.pi * kk * (zj.imag - h))          # |w|^k e^{2 pi k h}
        A = [float(np.sum((2 * np.pi * kk) ** n * ac * wk)) for n in range(6)]
        delta = ORACLE_TERM_ERR * A[0]
        A[0] += abs(t[j])
        B5 = sum(float(math.comb(5, a)) * A[a] * A[5 - a] for a in range(6))
        for d in (1.0, 1j):
            F1, F2, F3 = d * fn[1][j], d ** 2 * fn[2][j], d ** 3 * fn[3][j]
            L3 = 2 * np.real(F3 * np.conj(F[j])) + 6 * np.real(F2 * np.conj(F1))
            Fa = abs(F[j]) + A[1] * h
            tol[j] += h * h / 6 * abs(L3) + h ** 4 / 120 * B5 + (2 * Fa * delta + 4 * U64 * (Fa + delta) ** 2) / h
    return tol


def _fd_z(c, z, t, h):
    """Central differences of L_j(z_j) = |f(z_j) - t_j|^2 along Re z and Im z (FP64,
    the oracle at the shifted nodes), as dL/dRe + i dL/dIm."""
    Lp = np.abs(oracle.forward(c, z + h) - t) ** 2
    Lm = np.abs(oracle.forward(c, z - h) - t) ** 2
    Ip = np.abs(oracle.forward(c, z + 1j * h) - t) ** 2
    Im = np.abs(oracle.forward(c, z - 1j * h) - t) ** 2
    return (Lp - Lm) / (2 * h) + 1j * (Ip - Im) / (2 * h)


def test_grad_workload_against_fp64_direct_gradient_and_fd(torch):
    w = inputs.workload("grad")
    N, M, eps = w["N"], w["M"], w["eps32"]
    c = w["c"].astype(np.complex128)            # the complex64 values
    z = w["z"]
    t = w["t"].astype(np.complex128)
    _say("grad workload N = M =", N)
    gc, gz, f, scale = _autograd(torch, w["c"], z, w["t"], eps, torch.complex64, True)
    _say("   plan direct_scale", scale)

    n1 = np.abs(c).sum()
    n1d = np.abs(2 * np.pi * np.arange(N) * c).sum()
    f_ex = oracle.forward(c, z)
    Ef = np.abs(f - f_ex).max() / n1
    gf = 2 * (f - t)                             # what the backward received
    gf_ex = 2 * (f_ex - t)
    # dL/dc, every coefficient
    gc_ref = oracle.adjoint(gf, z, N)
    Ec = np.abs(gc - gc_ref).max() / np.abs(gf).sum()
    gc_ex = oracle.adjoint(gf_ex, z, N)
    dc = np.abs(gc - gc_ex).max()
    bar_c = eps * np.abs(gf).sum() + np.abs(gf - gf_ex).sum()
    _say("   E f =", Ef, " E dL/dc (same grad_f) =", Ec, " max|dL/dc - direct| =", dc, "bar", bar_c)
    assert Ef <= eps and Ec <= eps and dc <= bar_c

    # dL/dz on sampled nodes (2^12 random, interior to the step interval)
    rng = np.random.default_rng(3)
    h = 1e-3 / (2 * np.pi * N)
    cand = np.nonzero(z.imag > 2 * h)[0]
    sel = np.sort(rng.choice(cand, size=4096, replace=False))
    fp_ex = oracle.derivative(c, z[sel])
    gz_ex = gf_ex[sel] * np.conj(fp_ex)
    dz = np.abs(gz[sel] - gz_ex)
    bar_z = np.abs(gf[sel]) * eps * n1d + np.abs(fp_ex) * np.abs(gf[sel] - gf_ex[sel])
    _say("   dL/dz: max|err| / bar =", (dz / bar_z).max(), " max relative =", (dz / np.abs(gz_ex)).max())
    assert np.all(dz <= bar_z)

    # central differences in z on 256 of those nodes, h = 1e-3 / (2 pi N)
    sz = sel[:256]
    fd = _fd_z(c, z[sz], t[sz], h)
    tol_fd = _fd_z_tolerance(c, z[sz], t[sz], h)
    e_fd_ex = np.abs(fd - gf_ex[sz] * np.conj(oracle.derivative(c, z[sz])))
    e_fd_gpu = np.abs(fd - gz[sz])
    _say("   FD z: max|FD - direct| / tol =", (e_fd_ex / tol_fd).max(), " max|FD - GPU| / tol =",
         (e_fd_gpu / (tol_fd + bar_z[:256])).max())
    assert np.all(e_fd_ex <= tol_fd)
    assert np.all(e_fd_gpu <= tol_fd + bar_z[:256])

    # central differences in c along two random directions, h = 1e-3 (L is
    # quadratic in c: only the rounding of the two evaluations remains)
    hc = 1e-3
    for d in range(2):
        v = inputs.coefficients(np.random.default_rng(100 + d), N)
        fpl = oracle.forward(c + hc * v, z)
        fmi = oracle.forward(c - hc * v, z)
        Lp = np.sum(np.abs(fpl - t) ** 2)
        Lm = np.sum(np.abs(fmi - t) ** 2)
        fd_c = (Lp - Lm) / (2 * hc)
        Fmax = np.abs(fpl - t) + np.abs(fmi - t)
        dlt = 1.5e-14 * (n1 + hc * np.abs(v).sum())
        r_c = (np.sum(Fmax * dlt) + 2 * 20 * U64 * (Lp + Lm)) / (2 * hc)
        dd_ex = np.real(np.vdot(gc_ex, v))
        dd_gpu = np.real(np.vdot(gc, v))
        _say("   FD c dir", d, ": FD", fd_c, " direct", dd_ex, " GPU", dd_gpu, " rounding bar", r_c)
        assert abs(fd_c - dd_ex) <= r_c
        assert abs(fd_c - dd_gpu) <= r_c + np.abs(v).sum() * dc


def test_tiny_fp64_finite_differences(torch):
    """N = 16, FP64 form at eps 1e-12: central differences with h = 1e-3 in
    every real coordinate of c and z against the GPU gradient."""
    rng = np.random.default_rng(16)
    N, M, eps, h = 16, 8, 1e-12, 1e-3
    c = inputs.coefficients(rng, N)
    z = inputs.nodes_disk(rng, 64)
    z = z[z.imag > 2 * h][:M]
    t = inputs.coefficients(rng, M) * np.sqrt(0.5)
    gc, gz, f, _ = _autograd(torch, c, z, t, eps, torch.complex128, False)
    f_ex = oracle.forward(c, z)
    gf, gf_ex = 2 * (f - t), 2 * (f_ex - t)
    n1 = np.abs(c).sum()
    delta = 1.5e-14 * (n1 + 2 * h)
    # c: every real and imaginary part
    fd = np.empty(N, np.complex128)
    for k in range(N):
        parts = []
        for e in (1.0, 1j):
            cp, cm = c.copy(), c.copy()
            cp[k] += e * h
            cm[k] -= e * h
            parts.append((_loss(cp, z, t) - _loss(cm, z, t)) / (2 * h))
        fd[k] = parts[0] + 1j * parts[1]
    Ltot = np.sum(np.abs(f_ex - t) ** 2)
    r_c = (np.sum(2 * (np.abs(f_ex - t) + 2 * h) * delta) + 4 * 20 * U64 * Ltot) / (2 * h)
    bar_c = eps * np.abs(gf).sum() + np.abs(gf - gf_ex).sum()
    e_c = np.abs(gc - fd)
    _say("tiny FD c: max|GPU - FD| =", e_c.max(), " bar", 2 * r_c + bar_c)
    assert np.all(e_c <= 2 * r_c + bar_c)
    # z: Re and Im of every node
    fdz = _fd_z(c, z, t, h)
    tol = _fd_z_tolerance(c, z, t, h)
    fp_ex = oracle.derivative(c, z)
    n1d = np.abs(2 * np.pi * np.arange(N) * c).sum()
    bar_z = np.abs(gf) * eps * n1d + np.abs(fp_ex) * np.abs(gf - gf_ex)
    e_z = np.abs(gz - fdz)
    _say("tiny FD z: max|GPU - FD| / bar =", (e_z / (tol + bar_z)).max(), " max relative",
         (e_z / np.abs(fdz)).max())
    assert np.all(np.abs(fdz - gf_ex * np.conj(fp_ex)) <= tol)
    assert np.all(e_z <= tol + bar_z)
