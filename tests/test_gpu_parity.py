"""GPU parity of the HIP path (through the C ABI) against the oracle.

Bars (all relative to the 1-norm of the input, the paper's E of eq. 5.1):
* against the FP64 direct sums: E <= eps (Thm 4.3) for the FP64 form, and
  E <= eps for the FP32 form with eps >= 1e-6;
* against Algorithm 2 step by step with the same Kaiser-Bessel box (FP64):
  <= 1e-13, i.e. the same approximation up to rounding.
The benchmark's own size (N = M = 2^20) is covered in test_gpu_large.py, the
gradient workload (N = M = 2^18) in test_gpu_grad.py.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import method as O
from paper_1606_03255_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _run(torch, c, z, eps, dtype, op="forward", N=None, nfft_only=False):
    from paper_1606_03255_amd import Plan
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    N = len(c) if N is None else N
    plan = Plan(N, z, eps, tdt, nfft_only=nfft_only)
    x = torch.from_numpy(np.ascontiguousarray(c)).to("cuda", tdt)
    out = getattr(plan, op)(x)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.complex128)
    plan.close()
    return res


def _nodes(rng, M, kind):
    if kind == "disk":
        return inputs.nodes_disk(rng, M)
    if kind == "annulus":
        return inputs.nodes_annulus(rng, M)
    return np.concatenate([inputs.nodes_annulus(rng, M // 2), inputs.nodes_disk(rng, M - M // 2)])


CASES = [
    # N, M, eps, dtype, nodes      (one-pass only / two-pass FFT bands / ragged sizes)
    (256, 256, 1e-10, "c128", "disk"),
    (256, 256, 1e-6, "c64", "mixed"),
    (1000, 777, 1e-8, "c128", "mixed"),
    (5000, 900, 1e-11, "c128", "mixed"),
    (9000, 1500, 1e-6, "c64", "mixed"),
    (1 << 14, 1 << 14, 1e-11, "c128", "disk"),
    (1 << 14, 1 << 14, 1e-6, "c64", "disk"),
    (70000, 3000, 1e-6, "c64", "annulus"),
    (70000, 3000, 1e-12, "c128", "annulus"),
]


@pytest.mark.parametrize("nfft_only", [True, False])
@pytest.mark.parametrize("N,M,eps,dtype,kind", CASES)
def test_forward_vs_direct(torch, N, M, eps, dtype, kind, nfft_only):
    _say("forward", N, M, eps, dtype, kind, "nfft_only" if nfft_only else "policy")
    rng = np.random.default_rng(N + M)
    c = inputs.coefficients(rng, N)
    if dtype == "c64":
        c = c.astype(np.complex64).astype(np.complex128)
    z = _nodes(rng, M, kind)
    f = _run(torch, c, z, eps, dtype, nfft_only=nfft_only)
    E = np.abs(f - oracle.forward(c, z)).max() / np.abs(c).sum()
    _say("   E =", E)
    assert E <= eps


@pytest.mark.parametrize("nfft_only", [True, False])
@pytest.mark.parametrize("N,M,eps,dtype,kind", CASES)
def test_adjoint_and_derivative_vs_direct(torch, N, M, eps, dtype, kind, nfft_only):
    _say("adjoint/derivative", N, M, eps, dtype, kind, "nfft_only" if nfft_only else "policy")
    rng = np.random.default_rng(N + 2 * M)
    z = _nodes(rng, M, kind)
    g = inputs.coefficients(rng, M)
    c = inputs.coefficients(rng, N)
    if dtype == "c64":
        g = g.astype(np.complex64).astype(np.complex128)
        c = c.astype(np.complex64).astype(np.complex128)
    h = _run(torch, g, z, eps, dtype, "adjoint", N=N, nfft_only=nfft_only)
    Eh = np.abs(h - oracle.adjoint(g, z, N)).max() / np.abs(g).sum()
    fp = _run(torch, c, z, eps, dtype, "derivative", nfft_only=nfft_only)
    Ed = np.abs(fp - oracle.derivative(c, z)).max() / np.abs(2 * np.pi * np.arange(N) * c).sum()
    _say("   E adjoint =", Eh, " E derivative =", Ed)
    assert Eh <= eps
    assert Ed <= eps


@pytest.mark.parametrize("N,M,eps", [(256, 256, 1e-10), (3000, 500, 1e-8), (300, 200, 1e-6)])
def test_fp64_matches_algorithm2_step_by_step(torch, N, M, eps):
    """Same readings, same Kaiser-Bessel box: agreement to rounding."""
    _say("alg2 parity", N, M, eps)
    rng = np.random.default_rng(7 * N + M)
    c = inputs.coefficients(rng, N)
    z = _nodes(rng, M, "mixed")
    n1 = np.abs(c).sum()
    f = _run(torch, c, z, eps, "c128", nfft_only=True)
    assert np.abs(f - O.alg2_forward(c, z, eps, "nfft")).max() <= 1e-13 * n1
    g = inputs.coefficients(rng, M)
    h = _run(torch, g, z, eps, "c128", "adjoint", N=N, nfft_only=True)
    assert np.abs(h - O.alg2_adjoint(g, z, N, eps, "nfft")).max() <= 1e-13 * np.abs(g).sum()


def test_edge_cases(torch):
    rng = np.random.default_rng(99)
    # N = 1: f = c_0 everywhere; N = 2: a single frequency
    for N in (1, 2, 3, 17):
        _say("edge N", N)
        c = inputs.coefficients(rng, N)
        z = _nodes(rng, 50, "mixed")
        z[0] = complex(0.25, np.inf)   # w = 0
        z[1] = 0.999999999999 + 0j     # on the circle, x -> 1
        z[2] = 3.5 + 0j                # Re z outside [0, 1)
        z[3] = -0.25 + 1e-9j
        for dt, eps in (("c128", 1e-12), ("c64", 1e-6)):
            cc = c.astype(np.complex64).astype(np.complex128) if dt == "c64" else c
            f = _run(torch, cc, z, eps, dt)
            assert np.abs(f - oracle.forward(cc, z)).max() <= eps * np.abs(cc).sum()
    # M = 1; nodes exactly on band boundaries y = y_1 2^-m
    N = 600
    c = inputs.coefficients(rng, N)
    P = O.Params(N, 1e-9)
    ys = np.array([P.y1 * 2.0 ** -m for m in range(1, 30)] + [P.y1, 0.0])
    z = rng.random(len(ys)) + 1j * ys / (2 * np.pi)
    for zz in (z[:1], z):
        _say("edge boundaries", len(zz))
        f = _run(torch, c, zz, 1e-9, "c128")
        assert np.abs(f - oracle.forward(c, zz)).max() <= 1e-9 * np.abs(c).sum()
    # adversarial coefficients: every phase aligned at one node
    z = _nodes(rng, 64, "annulus")
    w = np.exp(2j * np.pi * z[5])
    k = np.arange(3000)
    c = np.conj(w ** k) / np.maximum(np.abs(w ** k), 1e-300)
    f = _run(torch, c, z, 1e-10, "c128")
    assert np.abs(f - oracle.forward(c, z)).max() <= 1e-10 * np.abs(c).sum()


def test_dot_identity(torch):
    """<C c, g> = <c, C^H g> for the realised operator (to rounding)."""
    rng = np.random.default_rng(5)
    N, M = 5000, 2000
    z = _nodes(rng, M, "mixed")
    c = inputs.coefficients(rng, N)
    g = inputs.coefficients(rng, M)
    f = _run(torch, c, z, 1e-9, "c128")
    h = _run(torch, g, z, 1e-9, "c128", "adjoint", N=N)
    lhs = np.vdot(g, f)
    rhs = np.vdot(h, c)
    assert abs(lhs - rhs) <= 1e-12 * np.abs(c).sum() * np.abs(g).sum()


FUSED_CASES = [
    # N, M, eps, dtype, nfft_only     (one-pass only / two-pass FFT bands; both band policies)
    (1000, 777, 1e-8, "c128", False),
    (9000, 1500, 1e-6, "c64", False),
    (9000, 1500, 1e-6, "c64", True),
    (70000, 3000, 1e-6, "c64", False),
    (70000, 3000, 1e-12, "c128", True),
]


@pytest.mark.parametrize("N,M,eps,dtype,nfft_only", FUSED_CASES)
def test_forward_derivative_one_pass(torch, N, M, eps, dtype, nfft_only):
    """flt_forward_derivative: f and f' in one pass (2q columns per band) meet
    the bars against the direct sums and agree with the separate calls."""
    from paper_1606_03255_amd import Plan
    _say("forward+derivative", N, M, eps, dtype, "nfft_only" if nfft_only else "policy")
    rng = np.random.default_rng(N + M + 31)
    c = inputs.coefficients(rng, N)
    z = _nodes(rng, M, "mixed")
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    if dtype == "c64":
        c = c.astype(np.complex64).astype(np.complex128)
    plan = Plan(N, z, eps, tdt, nfft_only=nfft_only)
    x = torch.from_numpy(c).to("cuda", tdt)
    f, fp = plan.forward_derivative(x)
    f0, fp0 = plan.forward(x), plan.derivative(x)
    torch.cuda.synchronize()
    f, fp, f0, fp0 = (t.cpu().numpy().astype(np.complex128) for t in (f, fp, f0, fp0))
    plan.close()
    n1, n1d = np.abs(c).sum(), np.abs(2 * np.pi * np.arange(N) * c).sum()
    E = np.abs(f - oracle.forward(c, z)).max() / n1
    Ed = np.abs(fp - oracle.derivative(c, z)).max() / n1d
    _say("   E forward =", E, " E derivative =", Ed)
    assert E <= eps and Ed <= eps
    tol = 1e-6 if dtype == "c64" else 1e-13
    assert np.abs(f - f0).max() <= tol * n1
    assert np.abs(fp - fp0).max() <= tol * n1d


@pytest.mark.parametrize("dtype,eps", [("c64", 1e-6), ("c128", 1e-11)])
def test_autograd_gradients(torch, dtype, eps):
    """fourier_laplace through autograd: dL/dc = C^H grad_f and
    dL/dz = grad_f conj(f'(z)) for L = sum |f - t|^2 (PyTorch's conjugate
    Wirtinger convention, grad_f = 2 (f - t)), against the direct sums applied
    to the grad_f the backward receives."""
    from paper_1606_03255_amd import Plan, fourier_laplace
    rng = np.random.default_rng(5)
    N, M = 9000, 1200
    c = inputs.coefficients(rng, N)
    z = _nodes(rng, M, "mixed")
    t = inputs.coefficients(rng, M)
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    if dtype == "c64":
        c = c.astype(np.complex64).astype(np.complex128)
    plan = Plan(N, z, eps, tdt)
    ct = torch.from_numpy(c).to("cuda", tdt).requires_grad_(True)
    zt = torch.from_numpy(z).to("cuda").requires_grad_(True)
    tt = torch.from_numpy(t).to("cuda", tdt)
    f = fourier_laplace(ct, zt, plan)
    loss = (f - tt).abs().pow(2).sum()
    loss.backward()
    torch.cuda.synchronize()
    gc = ct.grad.cpu().numpy().astype(np.complex128)
    gz = zt.grad.cpu().numpy()
    fg = f.detach().cpu().numpy().astype(np.complex128)
    assert np.abs(fg - oracle.forward(c, z)).max() <= eps * np.abs(c).sum()
    gf = 2 * (fg - t.astype(np.complex64 if dtype == "c64" else np.complex128))   # the grad_f backward receives
    ref_c = oracle.adjoint(gf, z, N)
    ref_z = gf * np.conj(oracle.derivative(c, z))
    Ec = np.abs(gc - ref_c).max() / np.abs(gf).sum()
    # the bar on f' (eps times its 1-norm) carried through the product with grad_f
    Ez = np.abs(gz - ref_z).max() / (np.abs(gf).max() * np.abs(2 * np.pi * np.arange(N) * c).sum())
    _say("autograd", dtype, "E dL/dc =", Ec, " E dL/dz =", Ez)
    plan.close()
    assert Ec <= 2 * eps and Ez <= 2 * eps


def test_output_tensors_are_checked(torch):
    """A mismatched output tensor is refused before any launch: wrong dtype,
    size or layout for the transforms, the profiling calls and the Laplace
    plan."""
    from paper_1606_03255_amd import LaplacePlan, Plan
    rng = np.random.default_rng(8)
    N, M = 300, 100
    z = _nodes(rng, M, "mixed")
    plan = Plan(N, z, 1e-6, torch.complex64)
    c = torch.from_numpy(inputs.coefficients(rng, N).astype(np.complex64)).to("cuda")
    bad = [torch.empty(M, dtype=torch.complex128, device="cuda"), torch.empty(M - 1, dtype=torch.complex64, device="cuda"),
           torch.empty(2 * M, dtype=torch.complex64, device="cuda")[::2]]
    for out in bad:
        for call in (lambda o: plan.forward(c, out=o), lambda o: plan.profile_forward(c, out=o),
                     lambda o: plan.forward_derivative(c, out=o)):
            with pytest.raises((TypeError, ValueError)):
                call(out)
    with pytest.raises(ValueError):
        f = torch.empty(M, dtype=torch.complex64, device="cuda")
        plan.forward_derivative(c, out=f, out_prime=f)
    with pytest.raises((TypeError, ValueError)):
        plan.profile_adjoint(torch.empty(M, dtype=torch.complex64, device="cuda"),
                             out=torch.empty(N + 1, dtype=torch.complex64, device="cuda"))
    plan.close()
    lp = LaplacePlan(rng.random(N) * N + 1, rng.random(M), 1e-6, torch.complex64)
    fh = torch.from_numpy(inputs.coefficients(rng, N).astype(np.complex64)).to("cuda")
    for out in bad:
        with pytest.raises((TypeError, ValueError)):
            lp.forward(fh, out=out)
    lp.close()


@pytest.mark.parametrize("direct_scale", [0.0, 4.0])
@pytest.mark.parametrize("dtype,eps", [("c64", 1e-6), ("c128", 1e-10)])
def test_fixed_policy_plan_vs_direct(torch, direct_scale, dtype, eps):
    """A plan built with a given band-policy factor (flt_plan_create_policy):
    forward and adjoint meet the bar; factor 0 keeps every band whose direct
    sum the policy can avoid on the NFFT path, factor 4 sends more to the
    direct sums."""
    from paper_1606_03255_amd import Plan
    rng = np.random.default_rng(11)
    N, M = 70000, 3000
    z = _nodes(rng, M, "mixed")
    c = inputs.coefficients(rng, N)
    g = inputs.coefficients(rng, M)
    if dtype == "c64":
        c = c.astype(np.complex64).astype(np.complex128)
        g = g.astype(np.complex64).astype(np.complex128)
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    _say("fixed policy", direct_scale, dtype, N, M)
    plan = Plan(N, z, eps, tdt, direct_scale=direct_scale)
    assert plan.info()["direct_scale"] == direct_scale
    f = plan.forward(torch.from_numpy(c).to("cuda", tdt)).cpu().numpy().astype(np.complex128)
    h = plan.adjoint(torch.from_numpy(g).to("cuda", tdt)).cpu().numpy().astype(np.complex128)
    plan.close()
    assert np.abs(f - oracle.forward(c, z)).max() <= eps * np.abs(c).sum()
    k = rng.choice(N, 400, replace=False)
    assert np.abs(h[k] - oracle.adjoint(g, z, N)[k]).max() <= eps * np.abs(g).sum()
