"""ORACLE (test infrastructure only): the discrete Laplace transform.

Kunis & Melzer, "Fast evaluation of real and complex exponential sums",
Sect. 3: f = K fhat with K = (exp(-y_j xi_k)) for real frequencies xi_k > 0
and real nodes y_j >= 0.

``direct``  the plain definition, f_j = sum_k fhat_k exp(-y_j xi_k), FP64.
``direct_kernel``  the same sum for another kernel kappa(y_j, xi_k) (Thm 3.3):
            "bessel_k_half", the example K_{1/2}(y xi) = sqrt(pi / (2 y xi)) e^{-y xi}.
``alg1``    the paper's Algorithm 1 step by step in numpy FP64 (partition of
            Def. 3.2, the approximant of Thm A.3): cumulative block sums g_m,
            block moments v = (L^Omega)^T fhat, h^{Y_m} = sum_l K^{Y_m,Omega_l} v,
            then L^{Y_m} h + g_{L_m+1}.

Readings (also listed in the design notes of the repository):
* y_1 = max_j y_j and xi_1 = max_k xi_k (the interval lengths of Def. 3.2);
  if every y_j is 0, all nodes lie in Y_M;
* the log inside l_m is the natural logarithm (as in the hot path's reading);
* Y_m = (y_1 2^-m, y_1 2^(1-m)] half open, Y_M = [0, y_1 2^(1-M)]; the same
  for Omega_l; the Chebyshev nodes of a block are those of its closure.
"""
import math

import numpy as np

from .method import interval_nodes, lagrange_bary


def direct(fhat, xi, y, block=2048):
    """f_j = sum_k fhat_k exp(-y_j xi_k) in FP64, rows in blocks."""
    fhat = np.asarray(fhat, np.complex128)
    xi = np.asarray(xi, np.float64)
    y = np.asarray(y, np.float64)
    out = np.zeros(len(y), np.complex128)
    for s in range(0, len(y), block):
        out[s:s + block] = np.exp(-np.outer(y[s:s + block], xi)) @ fhat
    return out


def bessel_k_half(x):
    """K_{1/2}(x) = sqrt(pi / (2 x)) e^{-x} (x > 0), the closed form the paper's
    example states for its integral definition."""
    x = np.asarray(x, np.float64)
    return np.sqrt(np.pi / (2.0 * x)) * np.exp(-x)


def direct_kernel(fhat, xi, y, kernel, block=2048):
    """f_j = sum_k fhat_k kappa(y_j, xi_k) in FP64, rows in blocks."""
    fhat = np.asarray(fhat, np.complex128)
    xi = np.asarray(xi, np.float64)
    y = np.asarray(y, np.float64)
    if kernel == "exp":
        return direct(fhat, xi, y, block)
    if kernel != "bessel_k_half":
        raise ValueError(kernel)
    out = np.zeros(len(y), np.complex128)
    for s in range(0, len(y), block):
        out[s:s + block] = bessel_k_half(np.outer(y[s:s + block], xi)) @ fhat
    return out


def params(xi, y, eps):
    """Def. 3.2: q, the number of levels M, y_1, xi_1, l_m and L_m."""
    y1 = float(np.max(y))
    xi1 = float(np.max(xi))
    q = int(math.ceil(0.5 + math.log(1.0 / eps) / math.log(4.0)))
    if y1 <= 0.0:
        return dict(q=q, M=1, y1=0.0, xi1=xi1, lm={}, Lm={})
    M = int(math.ceil(math.log2(y1 * xi1 / eps))) + 1
    lm = {m: max(1, int(math.floor(math.log2(y1 * xi1) - m - math.log2(math.log(1.0 / eps)))) + 1)
          for m in range(1, M)}
    Lm = {m: M - m for m in range(1, M)}
    return dict(q=q, M=M, y1=y1, xi1=xi1, lm=lm, Lm=Lm)


def level(v, v1, M):
    """Index i of the dyadic interval holding v: (v1 2^-i, v1 2^(1-i)] for
    i < M, [0, v1 2^(1-M)] for i = M (Def. 3.2)."""
    if M == 1 or v <= v1 * 2.0 ** (1 - M):
        return M
    i = max(1, min(M - 1, int(math.floor(math.log2(v1 / v))) + 1))
    while i > 1 and v > v1 * 2.0 ** (1 - i):
        i -= 1
    while i < M - 1 and v <= v1 * 2.0 ** (-i):
        i += 1
    return i


def alg1(fhat, xi, y, eps, trace=None):
    """Algorithm 1 (Sect. 3) in the paper's order; the result is the
    approximant f~ of Thm A.3, |f - f~| <= eps ||fhat||_1."""
    fhat = np.asarray(fhat, np.complex128)
    xi = np.asarray(xi, np.float64)
    y = np.asarray(y, np.float64)
    P = params(xi, y, eps)
    q, M, y1, xi1 = P["q"], P["M"], P["y1"], P["xi1"]
    out = np.zeros(len(y), np.complex128)
    if M == 1:                                   # every node in Y_M = {0}
        out[:] = fhat.sum()
        return out
    blk = np.array([level(v, xi1, M) for v in xi])
    band = np.array([level(v, y1, M) for v in y])
    # g_M = sum over Omega_M; g_m = g_{m+1} + sum over Omega_m
    g = np.zeros(M + 2, np.complex128)
    g[M] = fhat[blk == M].sum()
    for m in range(M - 1, 0, -1):
        g[m] = g[m + 1] + fhat[blk == m].sum()
    out[band == M] = g[1]
    # v^{Omega_l} = (L^{Omega_l})^T fhat^{Omega_l}
    v = {}
    for l in range(1, M):
        a, b = xi1 * 2.0 ** (-l), xi1 * 2.0 ** (1 - l)
        sel = blk == l
        nodes = interval_nodes(a, b, q)
        v[l] = lagrange_bary(xi[sel], nodes).T @ fhat[sel] if sel.any() else np.zeros(q, np.complex128)
    for m in range(1, M):
        sel = band == m
        if not sel.any():
            continue
        ym = interval_nodes(y1 * 2.0 ** (-m), y1 * 2.0 ** (1 - m), q)
        h = np.zeros(q, np.complex128)
        for l in range(P["lm"][m], P["Lm"][m] + 1):
            xl = interval_nodes(xi1 * 2.0 ** (-l), xi1 * 2.0 ** (1 - l), q)
            K = np.exp(-np.outer(ym, xl))        # K^{Y_m,Omega_l}[s, r] = kappa(y_s, xi_r)
            h += K @ v[l]
        out[sel] = lagrange_bary(y[sel], ym) @ h + g[P["Lm"][m] + 1]
    if trace is not None:
        trace.update(P=P, g=g, v=v, blk=blk, band=band)
    return out
