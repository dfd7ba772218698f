"""Writes forward_small.json: the oracle's FP64 direct sums (forward,
adjoint, derivative) for a small seeded case.  The paper prints no worked
example with numeric values, so the stored values come from the oracle only;
test_golden.py checks that the oracle still reproduces them and that the HIP
path meets its bar against them.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def case():
    rng = np.random.default_rng(2024)
    N, M = 64, 24
    c = rng.standard_normal((N, 2)) @ np.array([1.0, 1j])
    g = rng.standard_normal((M, 2)) @ np.array([1.0, 1j])
    x = rng.random(M)
    r2 = 1.0 - rng.random(M)                      # |w|^2 uniform by area in the disk
    z = x + 1j * (-np.log(r2) / (4 * np.pi))
    z[0] = 0.125 + 0j                             # on the circle
    z[1] = 0.5 + 1j * np.log(2.0) / (2 * np.pi)   # |w| = 1/2
    return N, M, c, g, z


def main():
    N, M, c, g, z = case()
    rec = {
        "what": "FP64 direct sums f = sum_k c_k w^k, C^H g, f' = sum_k 2 pi i k c_k w^k, w = exp(2 pi i z)",
        "N": N, "M": M,
        "c": [[v.real, v.imag] for v in c], "g": [[v.real, v.imag] for v in g],
        "z": [[v.real, v.imag] for v in z],
        "forward": [[v.real, v.imag] for v in oracle.forward(c, z)],
        "adjoint": [[v.real, v.imag] for v in oracle.adjoint(g, z, N)],
        "derivative": [[v.real, v.imag] for v in oracle.derivative(c, z)],
    }
    with open(os.path.join(HERE, "forward_small.json"), "w") as fh:
        json.dump(rec, fh, indent=0)


if __name__ == "__main__":
    main()
