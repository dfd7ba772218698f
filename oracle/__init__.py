"""ORACLE — test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_1606_03255_amd``)
never imports it and shares no code with it.

Contents
--------
``direct``   plain FP64 definition of the sums (C + OpenMP, ``direct.c``):
             forward f_j = sum_k c_k w_j^k (eq. 4.1 with xi_k = k),
             adjoint h_k = sum_j g_j conj(w_j)^k (the C^* of Sect. 4), also on
             chosen blocks of consecutive k only,
             derivative f'_j = sum_k 2 pi i k c_k w_j^k,
             and a compensated-Horner cross-check; with real exponents
             (principal power w^xi, Re z reduced to (-1/2, 1/2]) the forward
             f_j = sum_k c_k w_j^{xi_k} and the transposed evaluation
             g(xi_k) = sum_j g_j w_j^{xi_k} of Sect. 4.
``brute``    independent brute force: every power w^k formed on its own in
             80-bit extended precision (numpy longdouble) or with mpmath.
``laplace``  the discrete Laplace transform of Sect. 3: its plain FP64
             definition and Algorithm 1 step by step (Def. 3.2, Thm A.3).
``method``   the paper's Algorithm 2 (Sect. 4) step by step in numpy FP64,
             with the Laplace-side factorisation of Def. 3.2 / Lemma A.2 and
             the Fourier "black box" either exact (dense NDFT) or a
             Kaiser-Bessel NFFT.
"""
from .direct import (forward, adjoint, adjoint_blocks, derivative, horner, num_threads, load,  # noqa: F401
                     forward_xi, transposed_xi)
