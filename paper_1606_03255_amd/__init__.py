"""MI355X-native fast Fourier-Laplace transform.

Kunis & Melzer, "Fast evaluation of real and complex exponential sums":
evaluate f(z_j) = sum_{k<N} c_k exp(2 pi i k z_j) for Im z_j >= 0 (a polynomial
at nodes in the unit disk) with Algorithm 2, in hand-written HIP kernels for
gfx950 behind the C ABI of ``include/flt.h``.
"""
from .plan import LaplacePlan, Plan, XiPlan, fourier_laplace  # noqa: F401
from . import inputs  # noqa: F401
