"""ORACLE (test infrastructure only): brute-force evaluations used to pin the
FP64 oracle.  Each power w^k = e^{-k y} e^{2 pi i k x} is formed on its own
(no recurrence, no anchors), either in 80-bit extended precision (numpy
longdouble, unit roundoff 5.4e-20) or in mpmath at a chosen number of digits.
"""
import numpy as np

try:
    import mpmath
except ImportError:  # pragma: no cover
    mpmath = None

_TWO_PI_L = np.longdouble("6.28318530717958647692528676655900577")


def forward_longdouble(c, z):
    """sum_k c_k w^k for each node, every term formed directly in longdouble."""
    c = np.asarray(c, np.complex128)
    z = np.asarray(z, np.complex128)
    N = c.shape[0]
    k = np.arange(N, dtype=np.longdouble)
    cr = c.real.astype(np.longdouble)
    ci = c.imag.astype(np.longdouble)
    out = np.empty(z.shape[0], np.complex128)
    for j, zj in enumerate(z):
        re = np.longdouble(zj.real)
        im = np.longdouble(zj.imag)
        if np.isinf(zj.imag):
            out[j] = c[0]
            continue
        x = float(zj.real) - np.floor(float(zj.real))
        # split x = xh + xl with xh a multiple of 2^-40: k*xh is then exact in the
        # 64-bit longdouble mantissa for k < 2^24, so frac(k*x) carries no k-amplified error
        xh = np.floor(x * 2.0 ** 40) / 2.0 ** 40
        xl = np.longdouble(x - xh)
        ph = k * np.longdouble(xh)
        ph = (ph - np.round(ph)) + k * xl
        mag = np.exp(-k * (_TWO_PI_L * im))
        wr = mag * np.cos(_TWO_PI_L * ph)
        wi = mag * np.sin(_TWO_PI_L * ph)
        sr = np.sum(cr * wr - ci * wi)
        si = np.sum(cr * wi + ci * wr)
        out[j] = complex(float(sr), float(si))
    return out


def forward_mpmath(c, z, dps=40):
    """sum_k c_k exp(2 pi i k z) in mpmath at ``dps`` digits (tiny N, M only)."""
    if mpmath is None:
        raise RuntimeError("mpmath unavailable")
    out = []
    with mpmath.workdps(dps):
        for zj in z:
            zz = mpmath.mpc(float(zj.real), float(zj.imag)) if not np.isinf(zj.imag) else None
            if zz is None:
                out.append(complex(c[0]))
                continue
            w = mpmath.exp(2j * mpmath.pi * zz)
            s = mpmath.mpc(0)
            p = mpmath.mpc(1)
            for ck in c:
                s += mpmath.mpc(float(ck.real), float(ck.imag)) * p
                p *= w
            out.append(complex(s))
    return np.array(out, np.complex128)


def adjoint_mpmath(g, z, N, dps=40):
    """sum_j g_j conj(exp(2 pi i k z_j)) for k < N in mpmath (tiny sizes)."""
    if mpmath is None:
        raise RuntimeError("mpmath unavailable")
    out = []
    with mpmath.workdps(dps):
        ws = []
        for zj in z:
            if np.isinf(zj.imag):
                ws.append(mpmath.mpc(0))
            else:
                ws.append(mpmath.conj(mpmath.exp(2j * mpmath.pi * mpmath.mpc(float(zj.real), float(zj.imag)))))
        gs = [mpmath.mpc(float(v.real), float(v.imag)) for v in g]
        for k in range(N):
            s = mpmath.mpc(0)
            for gj, wj in zip(gs, ws):
                s += gj * (wj ** k if k else 1)
            out.append(complex(s))
    return np.array(out, np.complex128)
