"""Helpers shared by the GPU tests: device transfer, bitwise comparison and
a report line printed before each GPU step (so a failing step is named even
if the process dies)."""
import sys

import numpy as np

from exact import bits_equal


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def step(msg: str):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def to_gpu(a):
    torch = torch_cuda()
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_np(t):
    return t.detach().cpu().numpy()


def assert_bits(got, want, what=""):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    eq = bits_equal(got, want)
    if not eq.all():
        bad = np.flatnonzero(~eq)
        i = bad[0]
        raise AssertionError("%s: %d of %d differ; first at %d: got %r want %r"
                             % (what, bad.size, eq.size, i, got.flat[i], want.flat[i]))
