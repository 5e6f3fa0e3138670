"""Input generators (no GPU): determinism and the stated shapes and value
ranges."""
import numpy as np
import pytest

from paper_1401_6235_amd import workloads as W


def test_generators_are_deterministic_and_shaped():
    for dt in (np.float64, np.float32):
        a, b = W.chain_case("mul", 1000, seed=3, dtype=dt), W.chain_case("mul", 1000, seed=3, dtype=dt)
        assert all((a[k] == b[k]).all() and a[k].dtype == dt for k in a)
        assert np.all(np.abs(a["y0"] - 1) <= 2.0 ** -12)
        c = W.trsv_case(5, 10, seed=1, dtype=dt, kind="dense")
        U = c["U0"].reshape(5, 5, 10)
        assert (np.tril(np.ones((5, 5)), -1)[:, :, None] * U == 0).all()
        assert np.all(np.abs(np.diagonal(U, axis1=0, axis2=1)) >= 1)
        q = W.quadratic_case(3000, seed=1, dtype=dt)
        disc = q["b0"].astype(np.float64) ** 2 - 4 * q["a0"].astype(np.float64) * q["c0"].astype(np.float64)
        assert (disc < 0).any() and (disc > 0).any()
        f = W.fma_case(3000, seed=1, dtype=dt)
        assert f["w0"].dtype == dt and f["w1"].dtype == dt
