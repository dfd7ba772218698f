"""ORACLE (test infrastructure only): the paper's Algorithm 2 step by step.

Kunis & Melzer, "Fast evaluation of real and complex exponential sums".
Everything is plain numpy FP64 and follows the paper's order and notation;
no blocking, fusion or reordering beyond what the paper states.  Sizes must be
small enough for dense per-band products.

Readings of points the paper leaves open (each is also listed in the design
notes of the repository):

* exponents are k = 0..N-1; the k = 0 term (kernel exactly 1) is added as the
  constant c_0 at every node, so Z^0 nodes receive c_0 rather than 0;
* accuracy split of Lemma 4.1: eps_K = eps_A = eps/3; q and the levels D (the
  paper's M) are taken from eps_K, the Fourier black box is held to eps_A;
* y_1 := ln(1/eps_K) (nodes with y > y_1 form Z^0, |w| < eps_K), and
  xi_1 := 2^ceil(log2(N-1)) >= N-1, so that with the natural log the index of
  Def. 3.2 reduces exactly to l_m = max(1, n - m + 1), xi_1 = 2^n;
* intervals: Y_m = (y_1 2^-m, y_1 2^(1-m)] half open, Y_D = [0, y_1 2^(1-D)];
  the same for Omega_l;
* the Fourier black box on band m acts on the frequencies 1..min(N-1, K_m),
  K_m = xi_1 2^(1-l_m) (the band's support); the "nfft" box is the
  Kaiser-Bessel NFFT (oversampling 2) with grid n_m = max(2 K_m, 16), the
  frequencies centred at k_0 = floor(K_m/2), and window half-width m_w from
  the Kaiser-Bessel error bound at eps_A.
"""
import math

import numpy as np

TWO_PI = 2.0 * np.pi


# ----------------------------------------------------------------------------
# Sect. 2: Chebyshev nodes and barycentric Lagrange polynomials
# ----------------------------------------------------------------------------
def chebyshev_points(q):
    """t_j = cos((2j+1) pi / (2q)), j = 0..q-1 (zeros of T_q), Sect. 2."""
    j = np.arange(q)
    return np.cos((2 * j + 1) * np.pi / (2 * q))


def interval_nodes(a, b, q):
    """y_j^A = c^A + diam(A)/2 * t_j for A = [a, b], Sect. 2."""
    return 0.5 * (a + b) + 0.5 * (b - a) * chebyshev_points(q)


def bary_weights(q):
    """lambda_r = (-1)^r sin((2r+1) pi / (2q)), Sect. 2."""
    r = np.arange(q)
    return (-1.0) ** r * np.sin((2 * r + 1) * np.pi / (2 * q))


def lagrange_bary(y, nodes):
    """Matrix L[i, r] = L_r(y_i) by the barycentric formula of Sect. 2.
    A point equal to a node gets the Kronecker delta."""
    y = np.atleast_1d(np.asarray(y, np.float64))
    q = len(nodes)
    lam = bary_weights(q)
    d = y[:, None] - nodes[None, :]
    hit = d == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        w = lam[None, :] / d
        L = w / w.sum(axis=1, keepdims=True)
    rows = hit.any(axis=1)
    if rows.any():
        L[rows] = hit[rows].astype(np.float64)
    return L


def lagrange_product(y, nodes):
    """Matrix L[i, r] = prod_{j != r} (y_i - y_j)/(y_r - y_j) (first form, Sect. 2)."""
    y = np.atleast_1d(np.asarray(y, np.float64))
    q = len(nodes)
    L = np.ones((len(y), q))
    for r in range(q):
        for j in range(q):
            if j != r:
                L[:, r] *= (y - nodes[j]) / (nodes[r] - nodes[j])
    return L


# ----------------------------------------------------------------------------
# Def. 3.2, Lemma 4.1, Alg. 2: parameters and partitions
# ----------------------------------------------------------------------------
class Params:
    def __init__(self, N, eps):
        if not (0.0 < eps < 1.0):
            raise ValueError("eps must lie in (0, 1)")
        self.N = int(N)
        self.eps = float(eps)
        self.eps_K = eps / 3.0                      # Lemma 4.1 split
        self.eps_A = eps / 3.0
        self.q = int(math.ceil(0.5 + math.log(1.0 / self.eps_K) / math.log(4.0)))   # Def. 3.2
        self.y1 = math.log(1.0 / self.eps_K)        # |z| < eps_K  <=>  y > y_1
        kmax = max(self.N - 1, 1)
        self.n = int(math.ceil(math.log2(kmax))) if kmax > 1 else 0
        while (1 << self.n) < kmax:
            self.n += 1
        while self.n > 0 and (1 << (self.n - 1)) >= kmax:
            self.n -= 1
        self.xi1 = float(1 << self.n)
        self.D = int(math.ceil(math.log2(self.y1 * self.xi1 / self.eps_K))) + 1   # Def. 3.2 "M"
        self.mw = kb_halfwidth(self.eps_A)

    def ell(self, m):
        """l_m of Def. 3.2; with y_1 = ln(1/eps_K) it is max(1, n - m + 1) exactly."""
        return max(1, self.n - m + 1)

    def L(self, m):
        """L_m = D - m (Def. 3.2)."""
        return self.D - m

    def Y(self, m):
        """(lo, hi) of Y_m; Y_D = [0, y_1 2^(1-D)]."""
        m = int(m)
        if m >= self.D:
            return 0.0, math.ldexp(self.y1, 1 - self.D)
        return math.ldexp(self.y1, -m), math.ldexp(self.y1, 1 - m)

    def Omega(self, l):
        """(lo, hi) of Omega_l; Omega_D = [0, xi_1 2^(1-D)]."""
        l = int(l)
        if l >= self.D:
            return 0.0, math.ldexp(self.xi1, 1 - self.D)
        return math.ldexp(self.xi1, -l), math.ldexp(self.xi1, 1 - l)

    def K_band(self, m):
        """Upper end of band m's frequency support: xi_1 2^(1 - l_m)."""
        m = int(m)
        if m >= self.D:
            return int(self.xi1)
        return int(math.ldexp(self.xi1, 1 - self.ell(m)))

    def grid(self, m):
        """NFFT grid size and centre for band m (reading stated in the header)."""
        K = self.K_band(m)
        n = max(2 * K, 16)
        return n, K // 2


def polar(z):
    """Eq. 4.2: w = e^{-y} e^{2 pi i x}, x = Re z mod 1, y = 2 pi Im z."""
    z = np.asarray(z, np.complex128)
    x = z.real - np.floor(z.real)
    x = np.where(x >= 1.0, 0.0, x)
    y = TWO_PI * z.imag
    return x, y


def node_band(P, y):
    """Band index per node: 0 for Z^0 (y > y_1), m in 1..D-1 for Y_m, D for Y_D.
    Membership is decided by exact comparisons with y_1 2^-m (a first guess
    from log2 is corrected until y_1 2^-m < y <= y_1 2^(1-m) holds)."""
    y = np.asarray(y, np.float64)
    out = np.full(y.shape, P.D, np.int64)
    out[y > P.y1] = 0
    inner = (y <= P.y1) & (y > 0)
    with np.errstate(divide="ignore"):
        m = np.floor(np.log2(P.y1 / np.where(inner, y, 1.0))).astype(np.int64) + 1
    m = np.clip(m, 1, P.D)
    for _ in range(3):
        lo = np.ldexp(P.y1, -m)
        hi = np.ldexp(P.y1, 1 - m)
        m = np.where(~(y > lo) & (m < P.D), m + 1, m)
        m = np.where((y > hi) & (m > 1), m - 1, m)
    out[inner] = m[inner]
    return out


def freq_block(P, k):
    """l with k in Omega_l = (xi_1 2^-l, xi_1 2^(1-l)] (k >= 1)."""
    l = 1
    while not (k > math.ldexp(P.xi1, -l)):
        l += 1
    return l


# ----------------------------------------------------------------------------
# Laplace factor: K^{Y_m, Omega_l}, the contraction F^ K^T, and K~ (eq. A.2)
# ----------------------------------------------------------------------------
def K_block(P, m, l):
    """K^{Y_m,Omega_l}[s, r] = exp(-y_s xi_r) on the Chebyshev nodes (Def. 3.2)."""
    ys = interval_nodes(*P.Y(m), P.q)
    xr = interval_nodes(*P.Omega(l), P.q)
    return np.exp(-ys[:, None] * xr[None, :])


def contraction(P, m, c):
    """Rows k of (F^{Omega_l} K^{Y_m,Omega_l T}) for l_m <= l <= L_m, with
    F^{Omega_l} = diag(c^{Omega_l}) L^{Omega_l} (Alg. 2).  Returns (ks, G)
    with G[i, s] for frequency ks[i]; frequencies of blocks l > L_m are not
    included (they form the kernel ~ 1 part)."""
    ks, rows = [], []
    Kmax = min(P.K_band(m), P.N - 1)
    for l in range(P.ell(m), P.L(m) + 1):
        lo, hi = P.Omega(l)
        kk = np.arange(int(math.floor(lo)) + 1, min(int(math.floor(hi)), Kmax) + 1)
        if kk.size == 0:
            continue
        Lo = lagrange_bary(kk.astype(np.float64), interval_nodes(lo, hi, P.q))
        Fhat = c[kk][:, None] * Lo
        rows.append(Fhat @ K_block(P, m, l).T)
        ks.append(kk)
    if not ks:
        return np.zeros(0, np.int64), np.zeros((0, P.q), np.complex128)
    return np.concatenate(ks), np.concatenate(rows)


def ones_part(P, m):
    """Frequencies of the blocks l > L_m of band m (kernel ~ 1, Lemma A.2 iv)."""
    Kmax = min(P.K_band(m), P.N - 1)
    top = min(int(math.floor(math.ldexp(P.xi1, -P.L(m)))), Kmax)
    return np.arange(1, top + 1) if top >= 1 else np.zeros(0, np.int64)


def Ktilde(P, y, N):
    """Dense approximate Laplace matrix K~[j, k] of Thm A.3 (eq. A.2), with the
    k = 0 column equal to 1 and Z^0 rows equal to e_0 (see header)."""
    y = np.asarray(y, np.float64)
    bands = node_band(P, y)
    Kt = np.zeros((len(y), N))
    Kt[:, 0] = 1.0
    blk = np.array([freq_block(P, k) for k in range(1, N)], np.int64)
    for j, (v, m) in enumerate(zip(y, bands)):
        if m == 0:
            continue
        if m == P.D:
            Kt[j, 1:] = 1.0
            continue
        Ly = lagrange_bary([v], interval_nodes(*P.Y(m), P.q))[0]
        for l in range(1, P.D):
            sel = np.nonzero(blk == l)[0] + 1
            if sel.size == 0:
                continue
            if l < P.ell(m):
                continue                                   # Lemma A.2 ii: ~ 0
            if l > P.L(m):
                Kt[j, sel] = 1.0                           # Lemma A.2 iv: ~ 1
                continue
            lo, hi = P.Omega(l)
            Lo = lagrange_bary(sel.astype(np.float64), interval_nodes(lo, hi, P.q))
            Kt[j, sel] = Lo @ (K_block(P, m, l).T @ Ly)    # Lemma A.2 iii: I_q^{Y x Omega}
    return Kt


def dense_forward(c, z, eps):
    """(A o K~) c with the exact Fourier factor A (eq. 4.3)."""
    c = np.asarray(c, np.complex128)
    P = Params(len(c), eps)
    x, y = polar(z)
    k = np.arange(len(c))
    A = np.exp(2j * np.pi * np.outer(x, k))
    return (A * Ktilde(P, y, len(c))) @ c


def dense_adjoint(g, z, N, eps):
    """(A o K~)^H g."""
    P = Params(N, eps)
    x, y = polar(z)
    k = np.arange(N)
    A = np.exp(2j * np.pi * np.outer(x, k))
    return (A * Ktilde(P, y, N)).conj().T @ np.asarray(g, np.complex128)


# ----------------------------------------------------------------------------
# Fourier black box: exact NDFT or Kaiser-Bessel NFFT (oversampling 2)
# ----------------------------------------------------------------------------
SIGMA = 2.0
KB_B = np.pi * (2.0 - 1.0 / SIGMA)


def kb_error_bound(m, sigma=SIGMA):
    """Kaiser-Bessel NFFT error bound relative to ||a||_1 (Potts-Steidl):
    4 pi (sqrt(m) + m) (1 - 1/sigma)^(1/4) exp(-2 pi m sqrt(1 - 1/sigma))."""
    s = math.sqrt(1.0 - 1.0 / sigma)
    return 4.0 * math.pi * (math.sqrt(m) + m) * math.sqrt(s) * math.exp(-2.0 * math.pi * m * s)


def kb_halfwidth(eps_A):
    m = 2
    while kb_error_bound(m) > eps_A:
        m += 1
    return m


def kb_phi(u, m, b=KB_B):
    """Window in grid units u = n x - l, |u| <= m:  sinh(b sqrt(m^2-u^2)) / (pi sqrt(m^2-u^2))."""
    u = np.asarray(u, np.float64)
    v = np.sqrt(np.maximum(m * m - u * u, 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        r = np.where(v > 1e-8, np.sinh(b * v) / np.where(v > 1e-8, v, 1.0), b)
    return np.where(np.abs(u) <= m, r / np.pi, 0.0)


def kb_nphihat(k, n, m, b=KB_B):
    """n * phi_hat(k) = I_0(m sqrt(b^2 - (2 pi k / n)^2)) for |k| <= n (1 - 1/(2 sigma))."""
    k = np.asarray(k, np.float64)
    return np.i0(m * np.sqrt(b * b - (2.0 * np.pi * k / n) ** 2))


def ndft(a, ks, x):
    """sum_k a_k e^{2 pi i k x_j} exactly."""
    if len(ks) == 0:
        return np.zeros((len(x),) + a.shape[1:], np.complex128)
    return np.exp(2j * np.pi * np.outer(x, ks)) @ a


def ndft_adjoint(v, ks, x):
    if len(ks) == 0:
        return np.zeros((0,) + v.shape[1:], np.complex128)
    return np.exp(-2j * np.pi * np.outer(ks, x)) @ v


def nfft(a, ks, x, n, m, k0):
    """Kaiser-Bessel NFFT of the columns of a (frequencies ks, |ks - k0| <= n/4)."""
    a = np.asarray(a, np.complex128)
    squeeze = a.ndim == 1
    if squeeze:
        a = a[:, None]
    kp = np.asarray(ks) - k0
    ghat = np.zeros((n, a.shape[1]), np.complex128)
    ghat[np.mod(kp, n)] = a / kb_nphihat(kp, n, m)[:, None]
    g = np.fft.ifft(ghat, axis=0) * n            # g[l] = sum ghat[k'] e^{2 pi i k' l / n}
    nx = n * np.asarray(x, np.float64)
    l0 = np.floor(nx).astype(np.int64)
    out = np.zeros((len(x), a.shape[1]), np.complex128)
    for t in range(2 * m):
        l = l0 - m + 1 + t
        out += g[np.mod(l, n)] * kb_phi(nx - l, m)[:, None]
    out *= np.exp(2j * np.pi * k0 * np.asarray(x))[:, None]
    return out[:, 0] if squeeze else out


def nfft_adjoint(v, ks, x, n, m, k0):
    """Transpose-conjugate of ``nfft``: h_k = sum_j v_j e^{-2 pi i k x_j} (approx.)."""
    v = np.asarray(v, np.complex128)
    squeeze = v.ndim == 1
    if squeeze:
        v = v[:, None]
    nx = n * np.asarray(x, np.float64)
    l0 = np.floor(nx).astype(np.int64)
    u = v * np.exp(-2j * np.pi * k0 * np.asarray(x))[:, None]
    G = np.zeros((n, v.shape[1]), np.complex128)
    for t in range(2 * m):
        l = l0 - m + 1 + t
        np.add.at(G, np.mod(l, n), u * kb_phi(nx - l, m)[:, None])
    H = np.fft.fft(G, axis=0)                    # sum_l G[l] e^{-2 pi i k' l / n}
    kp = np.asarray(ks) - k0
    out = H[np.mod(kp, n)] / kb_nphihat(kp, n, m)[:, None]
    return out[:, 0] if squeeze else out


# ----------------------------------------------------------------------------
# Algorithm 2
# ----------------------------------------------------------------------------
def _box(P, m, fourier):
    if fourier == "ndft":
        return (lambda a, ks, x: ndft(a, ks, x)), (lambda v, ks, x: ndft_adjoint(v, ks, x))
    if fourier == "nfft":
        n, k0 = P.grid(m)
        return ((lambda a, ks, x: nfft(a, ks, x, n, P.mw, k0)),
                (lambda v, ks, x: nfft_adjoint(v, ks, x, n, P.mw, k0)))
    raise ValueError(fourier)


def alg2_forward(c, z, eps, fourier="ndft", trace=None):
    """Algorithm 2 (alg:XFLT) evaluated step by step; returns f~.
    ``trace`` (a dict) receives per-band intermediates if given."""
    c = np.asarray(c, np.complex128)
    N = len(c)
    P = Params(N, eps)
    x, y = polar(z)
    bands = node_band(P, y)
    f = np.full(len(x), c[0], np.complex128)           # k = 0 term; f~^{Z^0} = c_0
    if N == 1:
        return f
    # f~^{Z_D} = A~^{X_D, [1, xi_1]} c
    sel = np.nonzero(bands == P.D)[0]
    ks_all = np.arange(1, N)
    if sel.size:
        A, _ = _box(P, P.D, fourier)
        f[sel] += A(c[ks_all], ks_all, x[sel])
    for m in range(1, P.D):
        sel = np.nonzero(bands == m)[0]
        if sel.size == 0:
            continue
        A, _ = _box(P, m, fourier)
        ones = ones_part(P, m)                              # Omega = U_{l > L_m} Omega_l
        part1 = A(c[ones], ones, x[sel]) if ones.size else 0.0
        ks, G = contraction(P, m, c)                        # (F^{Omega_l} K^{Y_m,Omega_l T})_l
        F = A(G, ks, x[sel])                                # F = A~^{X_m,Omega}(...)
        Ly = lagrange_bary(y[sel], interval_nodes(*P.Y(m), P.q))
        f[sel] += part1 + (Ly * F).sum(axis=1)              # f~ += (L^{Y_m} o F) 1
        if trace is not None:
            trace[m] = dict(nodes=sel, ks=ks, G=G, F=F, Ly=Ly, ones=ones)
    return f


def alg2_adjoint(g, z, N, eps, fourier="ndft"):
    """Adjoint of ``alg2_forward`` factor by factor (Sect. 4, closing remarks)."""
    g = np.asarray(g, np.complex128)
    P = Params(N, eps)
    x, y = polar(z)
    bands = node_band(P, y)
    h = np.zeros(N, np.complex128)
    h[0] = g.sum()
    if N == 1:
        return h
    ks_all = np.arange(1, N)
    sel = np.nonzero(bands == P.D)[0]
    if sel.size:
        _, AH = _box(P, P.D, fourier)
        h[ks_all] += AH(g[sel], ks_all, x[sel])
    for m in range(1, P.D):
        sel = np.nonzero(bands == m)[0]
        if sel.size == 0:
            continue
        _, AH = _box(P, m, fourier)
        ones = ones_part(P, m)
        if ones.size:
            h[ones] += AH(g[sel], ones, x[sel])
        Ly = lagrange_bary(y[sel], interval_nodes(*P.Y(m), P.q))
        for l in range(P.ell(m), P.L(m) + 1):
            lo, hi = P.Omega(l)
            Kmax = min(P.K_band(m), N - 1)
            kk = np.arange(int(math.floor(lo)) + 1, min(int(math.floor(hi)), Kmax) + 1)
            if kk.size == 0:
                continue
            Hs = AH(g[sel][:, None] * Ly, kk, x[sel])               # |kk| x q
            Lo = lagrange_bary(kk.astype(np.float64), interval_nodes(lo, hi, P.q))
            h[kk] += ((Hs @ K_block(P, m, l)) * Lo).sum(axis=1)      # L^Omega K^T transposed
    return h


def alg2_derivative(c, z, eps, fourier="ndft"):
    """f'(z) = sum_k 2 pi i k c_k w^k: Algorithm 2 applied to c'_k = 2 pi i k c_k."""
    c = np.asarray(c, np.complex128)
    k = np.arange(len(c))
    return alg2_forward(2j * np.pi * k * c, z, eps, fourier)
