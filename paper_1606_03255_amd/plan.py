"""Python face of the fast Fourier-Laplace transform.

``Plan`` wraps one ``flt_plan`` of the C ABI: torch supplies the device
memory (workspace, outputs) and the stream; every step of the transform runs
in the library's kernels.  ``FourierLaplace`` is the autograd Function that
pairs the forward with its hand-written backward (adjoint for dL/dc, the
derivative transform for dL/dz).
"""
import ctypes

import numpy as np

from . import _lib as L


def _as_host_z(z):
    try:
        import torch
        if isinstance(z, torch.Tensor):
            z = z.detach().to("cpu", torch.complex128).numpy()
    except ImportError:  # pragma: no cover
        pass
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).reshape(-1))
    return z


def _as_host_real(v):
    try:
        import torch
        if isinstance(v, torch.Tensor):
            v = v.detach().to("cpu", torch.float64).numpy()
    except ImportError:  # pragma: no cover
        pass
    return np.asarray(v, dtype=np.float64).reshape(-1)


def _dtype_code(dtype):
    if dtype in ("c64", "complex64", L.FLT_C64):
        return L.FLT_C64
    if dtype in ("c128", "complex128", L.FLT_C128):
        return L.FLT_C128
    try:
        import torch
        if dtype == torch.complex64:
            return L.FLT_C64
        if dtype == torch.complex128:
            return L.FLT_C128
    except ImportError:  # pragma: no cover
        pass
    raise ValueError("dtype must be complex64 or complex128")


def _check_tensor(t, n, name, dtype, device):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor on the plan's device" % name)
    if t.dtype != dtype:
        raise TypeError("%s has dtype %s, the plan computes in %s" % (name, t.dtype, dtype))
    if t.device != device:
        raise ValueError("%s is on %s, the plan lives on %s" % (name, t.device, device))
    if t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return t


def _check_out(t, n, name, dtype, device):
    _check_tensor(t, n, name, dtype, device)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous (the result is written through its data pointer)" % name)
    return t


class Plan:
    """Plan for N coefficients at the nodes z (Im z >= 0) with accuracy eps.

    dtype ``complex64`` selects the FP32 form (FP32 bulk arithmetic, FP64
    phase reduction and per-node sums); ``complex128`` the plain FP64 form.
    With ``host_only=True`` only the host-side plan is built (parameters,
    partition, byte model) and no GPU is touched.  ``nfft_only=True`` keeps
    every band on Algorithm 2's NFFT path; by default bands with few nodes and
    large grids are summed directly (exactly).  ``graph=True`` captures each
    operation's launch sequence into a hipGraph on first use and replays it.
    ``autotune=True`` chooses the band policy by timing forward + adjoint of
    candidate plans on the device (cached per size class for the process);
    ``autotune="forward"`` times the forward alone (plans for evaluation only).
    ``direct_scale=x`` builds a single plan with the band policy's factor x
    (a tuned plan's ``info()["direct_scale"]``) without timing anything.

    ``Plan.batch`` builds one plan for many independent instances; its
    transforms act on packed arrays (instance after instance).
    """

    def __init__(self, N, z, eps, dtype="complex64", device=None, host_only=False, nfft_only=False, graph=False,
                 autotune=False, direct_scale=None, _sizes=None):
        self._lib = L.load()
        self._ptr = ctypes.c_void_p()
        zh = _as_host_z(z)
        if _sizes is None:
            self.Ns = np.array([int(N)], np.int64)
            self.Ms = np.array([zh.shape[0]], np.int64)
        else:
            self.Ns, self.Ms = _sizes
        self.N = int(self.Ns.sum())
        self.M = int(self.Ms.sum())
        self.count = len(self.Ns)
        self.dtype_code = _dtype_code(dtype)
        self.host_only = bool(host_only)
        flags = ((L.FLT_FLAG_HOST_ONLY if host_only else 0) | (L.FLT_FLAG_NFFT_ONLY if nfft_only else 0)
                 | (L.FLT_FLAG_GRAPH if graph else 0) | (L.FLT_FLAG_AUTOTUNE if autotune else 0)
                 | (L.FLT_FLAG_TUNE_FORWARD if autotune == "forward" else 0))
        self._ws = None
        zp = zh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        I64 = ctypes.POINTER(ctypes.c_int64)

        if direct_scale is not None and (autotune or _sizes is not None):
            raise ValueError("direct_scale fixes the band policy of a single plan: not with autotune or a batch")

        def create():
            if direct_scale is not None:
                rc = self._lib.flt_plan_create_policy(ctypes.byref(self._ptr), self.N, self.M, zp, float(eps),
                                                      self.dtype_code, flags, float(direct_scale))
            elif _sizes is None:
                rc = self._lib.flt_plan_create(ctypes.byref(self._ptr), self.N, self.M, zp, float(eps),
                                               self.dtype_code, flags)
            else:
                rc = self._lib.flt_plan_create_batch(ctypes.byref(self._ptr), self.count,
                                                     self.Ns.ctypes.data_as(I64), self.Ms.ctypes.data_as(I64),
                                                     zp, float(eps), self.dtype_code, flags)
            L.check(rc, "flt_plan_create" if _sizes is None else "flt_plan_create_batch")

        if host_only:
            create()
            self.device = None
            return
        import torch
        self.device = torch.device(device if device is not None else "cuda", )
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            create()
            nbytes = ctypes.c_size_t()
            L.check(self._lib.flt_plan_workspace_size(self._ptr, ctypes.byref(nbytes)), "flt_plan_workspace_size")
            self._ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
            L.check(self._lib.flt_plan_set_workspace(self._ptr, ctypes.c_void_p(self._ws.data_ptr()),
                                                     self._ws.numel()), "flt_plan_set_workspace")

    @classmethod
    def batch(cls, Ns, zs, eps, dtype="complex64", device=None, host_only=False, nfft_only=False, graph=False,
              autotune=False):
        """One plan for independent instances: instance i has Ns[i] coefficients
        and the nodes zs[i].  Coefficients, results and adjoint inputs are packed
        instance after instance (offsets in ``c_offsets`` / ``f_offsets``)."""
        zl = [_as_host_z(z) for z in zs]
        Ns = np.ascontiguousarray(np.asarray(Ns, np.int64).reshape(-1))
        Ms = np.array([len(z) for z in zl], np.int64)
        if len(Ns) != len(Ms) or len(Ns) == 0:
            raise ValueError("need one coefficient count per node set, and at least one instance")
        z = np.concatenate(zl) if len(zl) > 1 else zl[0]
        return cls(None, z, eps, dtype, device, host_only, nfft_only, graph, autotune, _sizes=(Ns, Ms))

    @property
    def c_offsets(self):
        return np.concatenate([[0], np.cumsum(self.Ns)[:-1]]).astype(np.int64)

    @property
    def f_offsets(self):
        return np.concatenate([[0], np.cumsum(self.Ms)[:-1]]).astype(np.int64)

    # ---------------------------------------------------------------- queries
    @property
    def torch_dtype(self):
        import torch
        return torch.complex64 if self.dtype_code == L.FLT_C64 else torch.complex128

    def info(self):
        inf = L.FltInfo()
        L.check(self._lib.flt_plan_info(self._ptr, ctypes.byref(inf)), "flt_plan_info")
        return {name: getattr(inf, name) for name, _ in L.FltInfo._fields_}

    def bands(self):
        out = []
        for i in range(self.info()["num_bands"]):
            b = L.FltBandInfo()
            L.check(self._lib.flt_plan_band(self._ptr, i, ctypes.byref(b)), "flt_plan_band")
            out.append({name: getattr(b, name) for name, _ in L.FltBandInfo._fields_})
        return out

    def node_bands(self):
        out = np.empty(self.M, np.int32)
        L.check(self._lib.flt_plan_node_bands(self._ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
                "flt_plan_node_bands")
        return out

    # ------------------------------------------------------------- transforms
    def _prep(self, t, n, name):
        """An input tensor checked against the plan (type, device, size); a
        contiguous copy is made if needed."""
        return _check_tensor(t, n, name, self.torch_dtype, self.device).contiguous()

    def _prep_out(self, t, n, name):
        """An output tensor: as an input, and contiguous itself (the kernels
        write through its data pointer, so a copy would lose the result)."""
        return _check_out(t, n, name, self.torch_dtype, self.device)

    def _run(self, fn, x, nin, nout, out, name):
        import torch
        if self.host_only:
            raise RuntimeError("host-only plan")
        x = self._prep(x, nin, name)
        if out is None:
            out = torch.empty(nout, dtype=self.torch_dtype, device=self.device)
        else:
            out = self._prep_out(out, nout, "out")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        L.check(fn(self._ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                   ctypes.c_void_p(stream)), fn.__name__)
        return out

    def forward(self, c, out=None):
        """f_j ~ sum_k c_k exp(2 pi i k z_j); c: complex[N] on the device."""
        return self._run(self._lib.flt_forward, c, self.N, self.M, out, "c")

    def forward_noalloc(self, c, out=None):
        """The forward without the plan's workspace: its scratch is the
        library's static device array (flt_forward_noalloc); calls that
        overlap in time on one device race."""
        return self._run(self._lib.flt_forward_noalloc, c, self.N, self.M, out, "c")

    def derivative(self, c, out=None):
        """f'(z_j) ~ sum_k 2 pi i k c_k exp(2 pi i k z_j)."""
        return self._run(self._lib.flt_derivative, c, self.N, self.M, out, "c")

    def adjoint(self, g, out=None):
        """h_k ~ sum_j g_j conj(exp(2 pi i k z_j)), k < N."""
        return self._run(self._lib.flt_adjoint, g, self.M, self.N, out, "g")

    def forward_derivative(self, c, out=None, out_prime=None):
        """(f, f') in one pass: the forward and the derivative transforms of c."""
        import torch
        if self.host_only:
            raise RuntimeError("host-only plan")
        c = self._prep(c, self.N, "c")
        f = torch.empty(self.M, dtype=self.torch_dtype, device=self.device) if out is None else \
            self._prep_out(out, self.M, "out")
        fp = torch.empty(self.M, dtype=self.torch_dtype, device=self.device) if out_prime is None else \
            self._prep_out(out_prime, self.M, "out_prime")
        if f.data_ptr() == fp.data_ptr():
            raise ValueError("out and out_prime must be distinct tensors")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        L.check(self._lib.flt_forward_derivative(self._ptr, ctypes.c_void_p(c.data_ptr()),
                                                 ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(fp.data_ptr()),
                                                 ctypes.c_void_p(stream)), "flt_forward_derivative")
        return f, fp

    PROFILE_FORWARD_STAGES = ("onepass_fft", "passA_fft", "passB_fft", "gather", "direct")
    PROFILE_ADJOINT_STAGES = ("clear_sum_g", "node_prep", "cell_spread", "passB_fft", "passA_fft", "onepass_fft",
                              "direct", "finalize")

    def _profile(self, fn, x, nin, nout, out, name, nst):
        import torch
        if self.host_only:
            raise RuntimeError("host-only plan")
        x = self._prep(x, nin, name)
        out = torch.empty(nout, dtype=self.torch_dtype, device=self.device) if out is None else \
            self._prep_out(out, nout, "out")
        ms = (ctypes.c_double * nst)()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        L.check(fn(self._ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                   ctypes.c_void_p(stream), ms), fn.__name__)
        return out, list(ms)

    def profile_forward(self, c, out=None):
        """One forward with per-stage HIP-event timing; returns (f, stage_ms)
        with stage_ms for PROFILE_FORWARD_STAGES."""
        return self._profile(self._lib.flt_profile_forward, c, self.N, self.M, out, "c", 5)

    def profile_adjoint(self, g, out=None):
        """One adjoint with per-stage HIP-event timing; returns (c_out,
        stage_ms) with stage_ms for PROFILE_ADJOINT_STAGES."""
        return self._profile(self._lib.flt_profile_adjoint, g, self.M, self.N, out, "g", 8)

    def close(self):
        if getattr(self, "_ptr", None) and self._ptr.value:
            if self.device is not None:
                import torch
                torch.cuda.synchronize(self.device)
            self._lib.flt_plan_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _make_function():
    import torch

    class FourierLaplace(torch.autograd.Function):
        """f = C(z) c with C_jk = exp(2 pi i k z_j), through ``plan``.

        Backward (PyTorch's conjugate-Wirtinger convention):
            dL/dc = C^H grad_f                      (plan.adjoint)
            dL/dz = grad_f * conj(f'(z))            (f' from plan.forward_derivative)
        ``z`` must hold the values the plan was built from.  When z needs a
        gradient, the forward computes f and f' in one pass and keeps f'."""

        @staticmethod
        def forward(ctx, c, z, plan):
            ctx.plan = plan
            ctx.z_dtype = z.dtype
            if ctx.needs_input_grad[1]:
                f, fp = plan.forward_derivative(c)
                ctx.save_for_backward(fp)
                return f
            ctx.save_for_backward(None)
            return plan.forward(c)

        @staticmethod
        def backward(ctx, grad_f):
            (fp,) = ctx.saved_tensors
            plan = ctx.plan
            grad_f = grad_f.to(plan.torch_dtype).contiguous()
            gc = plan.adjoint(grad_f) if ctx.needs_input_grad[0] else None
            gz = None
            if ctx.needs_input_grad[1]:
                gz = (grad_f * fp.conj()).to(ctx.z_dtype)
            return gc, gz, None

    return FourierLaplace


_FL = None


def fourier_laplace(c, z, plan):
    """Differentiable f = C(z) c evaluated by ``plan`` (see FourierLaplace)."""
    global _FL
    if _FL is None:
        _FL = _make_function()
    return _FL.apply(c, z, plan)


KERNELS = {"exp": 0, "bessel_k_half": 1}


class LaplacePlan:
    """The discrete Laplace transform f_j = sum_k fhat_k exp(-y_j xi_k)
    (xi_k > 0, y_j >= 0) by Algorithm 1, error <= eps * sum |fhat_k|; with
    ``kernel="bessel_k_half"`` the asymptotically smooth kernel
    K_{1/2}(y xi) = sqrt(pi / (2 y xi)) exp(-y xi) of Thm 3.3's example (y_j > 0).

    ``xi`` and ``y`` are real (host arrays or tensors, copied); ``dtype``
    sets the type of fhat and f (the arithmetic is FP64 either way).  The
    plan owns its small device accumulator: calls on one plan must not
    overlap."""

    def __init__(self, xi, y, eps, dtype="complex64", device=None, host_only=False, kernel="exp"):
        self._lib = L.load()
        self._ptr = ctypes.c_void_p()
        xh = np.ascontiguousarray(_as_host_real(xi))
        yh = np.ascontiguousarray(_as_host_real(y))
        self.N, self.M = int(xh.shape[0]), int(yh.shape[0])
        self.dtype_code = _dtype_code(dtype)
        self.host_only = bool(host_only)
        D = ctypes.POINTER(ctypes.c_double)

        if kernel not in KERNELS:
            raise ValueError("kernel must be one of %s" % sorted(KERNELS))

        def create():
            L.check(self._lib.flt_laplace_plan_create_kernel(ctypes.byref(self._ptr), KERNELS[kernel], self.N,
                                                             xh.ctypes.data_as(D), self.M, yh.ctypes.data_as(D),
                                                             float(eps), self.dtype_code,
                                                             L.FLT_FLAG_HOST_ONLY if host_only else 0),
                    "flt_laplace_plan_create_kernel")

        if host_only:
            create()
            self.device = None
            return
        import torch
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            create()

    @property
    def torch_dtype(self):
        import torch
        return torch.complex64 if self.dtype_code == L.FLT_C64 else torch.complex128

    def info(self):
        o = L.FltLaplaceInfo()
        L.check(self._lib.flt_laplace_plan_info(self._ptr, ctypes.byref(o)), "flt_laplace_plan_info")
        return {k: getattr(o, k) for k, _ in L.FltLaplaceInfo._fields_}

    def forward(self, fhat, out=None):
        """f_j ~ sum_k fhat_k exp(-y_j xi_k); fhat: complex[N] on the device."""
        import torch
        if self.host_only:
            raise RuntimeError("host-only plan")
        fhat = _check_tensor(fhat, self.N, "fhat", self.torch_dtype, self.device).contiguous()
        if out is None:
            out = torch.empty(self.M, dtype=self.torch_dtype, device=self.device)
        else:
            out = _check_out(out, self.M, "out", self.torch_dtype, self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        L.check(self._lib.flt_laplace_forward(self._ptr, ctypes.c_void_p(fhat.data_ptr()),
                                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream)),
                "flt_laplace_forward")
        return out

    def close(self):
        if getattr(self, "_ptr", None) and self._ptr.value:
            if self.device is not None:
                import torch
                torch.cuda.synchronize(self.device)
            self._lib.flt_laplace_plan_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class XiPlan:
    """Real exponents: f_j = sum_k c_k w_j^{xi_k} (eq. 4.1 with real xi_k >= 1),
    its transposed h_k = sum_j g_j w_j^{xi_k} (the g(xi) of Sect. 4) and its
    adjoint h_k = sum_j g_j conj(w_j^{xi_k}); w_j = exp(2 pi i z_j), principal
    power with Re z reduced to (-1/2, 1/2].  Error <= eps * sum |coefficients|.

    ``xi`` (real) and ``z`` (complex, Im z >= 0) are host arrays or tensors,
    copied.  The plan owns its device memory (tables, the inner batched
    integer plan, its buffers): calls on one plan must not overlap."""

    def __init__(self, xi, z, eps, dtype="complex64", device=None, host_only=False):
        self._lib = L.load()
        self._ptr = ctypes.c_void_p()
        xh = np.ascontiguousarray(_as_host_real(xi))
        zh = _as_host_z(z)
        self.N, self.M = int(xh.shape[0]), int(zh.shape[0])
        self.dtype_code = _dtype_code(dtype)
        self.host_only = bool(host_only)
        D = ctypes.POINTER(ctypes.c_double)

        def create():
            L.check(self._lib.flt_xi_plan_create(ctypes.byref(self._ptr), self.N, xh.ctypes.data_as(D), self.M,
                                                 zh.ctypes.data_as(D), float(eps), self.dtype_code,
                                                 L.FLT_FLAG_HOST_ONLY if host_only else 0),
                    "flt_xi_plan_create")

        if host_only:
            create()
            self.device = None
            return
        import torch
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            create()

    @property
    def torch_dtype(self):
        import torch
        return torch.complex64 if self.dtype_code == L.FLT_C64 else torch.complex128

    def info(self):
        o = L.FltXiInfo()
        L.check(self._lib.flt_xi_plan_info(self._ptr, ctypes.byref(o)), "flt_xi_plan_info")
        return {k: getattr(o, k) for k, _ in L.FltXiInfo._fields_}

    def _call(self, fn, x, nin, nout, out, name):
        import torch
        if self.host_only:
            raise RuntimeError("host-only plan")
        x = _check_tensor(x, nin, "input", self.torch_dtype, self.device).contiguous()
        if out is None:
            out = torch.empty(nout, dtype=self.torch_dtype, device=self.device)
        else:
            out = _check_out(out, nout, "out", self.torch_dtype, self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        L.check(fn(self._ptr, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                   ctypes.c_void_p(stream)), name)
        return out

    def forward(self, c, out=None):
        """f_j = sum_k c_k w_j^{xi_k}; c: complex[N] on the device, order of xi."""
        return self._call(self._lib.flt_xi_forward, c, self.N, self.M, out, "flt_xi_forward")

    def transposed(self, g, out=None):
        """h_k = sum_j g_j w_j^{xi_k}; g: complex[M] on the device."""
        return self._call(self._lib.flt_xi_transposed, g, self.M, self.N, out, "flt_xi_transposed")

    def adjoint(self, g, out=None):
        """h_k = sum_j g_j conj(w_j^{xi_k}); g: complex[M] on the device."""
        return self._call(self._lib.flt_xi_adjoint, g, self.M, self.N, out, "flt_xi_adjoint")

    def close(self):
        if getattr(self, "_ptr", None) and self._ptr.value:
            if self.device is not None:
                import torch
                torch.cuda.synchronize(self.device)
            self._lib.flt_xi_plan_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
