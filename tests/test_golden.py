"""Stored oracle values (tests/golden/forward_small.json, written by
tests/golden/make_golden.py from the oracle's FP64 direct sums): the oracle
must still reproduce them, and the HIP path must meet its bar against them."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "forward_small.json")


def _load():
    with open(GOLDEN) as fh:
        r = json.load(fh)
    cx = lambda a: np.array([complex(u, v) for u, v in a])
    return r, cx(r["c"]), cx(r["g"]), cx(r["z"]), cx(r["forward"]), cx(r["adjoint"]), cx(r["derivative"])


def test_oracle_reproduces_the_stored_values():
    r, c, g, z, f, h, fp = _load()
    n1 = np.abs(c).sum()
    assert np.abs(oracle.forward(c, z) - f).max() <= 1e-14 * n1
    assert np.abs(oracle.adjoint(g, z, r["N"]) - h).max() <= 1e-14 * np.abs(g).sum()
    assert np.abs(oracle.derivative(c, z) - fp).max() <= 1e-14 * np.abs(2 * np.pi * np.arange(r["N"]) * c).sum()
    # the two planted special nodes: |w| = 1 at Re z = 1/8, and |w| = 1/2
    w1 = np.exp(2j * np.pi * z[1])
    assert abs(abs(w1) - 0.5) < 1e-15
    assert abs(f[1] - np.polyval(c[::-1], w1)) <= 1e-13 * n1


@pytest.mark.gpu
@pytest.mark.parametrize("dtype,eps", [("c128", 1e-12), ("c64", 1e-6)])
def test_hip_path_against_the_stored_values(dtype, eps):
    import torch
    from paper_1606_03255_amd import Plan
    r, c, g, z, f, h, fp = _load()
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    p = Plan(r["N"], z, eps, tdt)
    cc = c.astype(np.complex64).astype(np.complex128) if dtype == "c64" else c
    gg = g.astype(np.complex64).astype(np.complex128) if dtype == "c64" else g
    fr = oracle.forward(cc, z) if dtype == "c64" else f
    hr = oracle.adjoint(gg, z, r["N"]) if dtype == "c64" else h
    got_f = p.forward(torch.from_numpy(cc).to("cuda", tdt)).cpu().numpy()
    got_h = p.adjoint(torch.from_numpy(gg).to("cuda", tdt)).cpu().numpy()
    p.close()
    assert np.abs(got_f - fr).max() <= eps * np.abs(cc).sum()
    assert np.abs(got_h - hr).max() <= eps * np.abs(gg).sum()
