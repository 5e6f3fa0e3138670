"""GPU parity past 2^31 elements, binary32 and binary64: 64-bit indexing in
the elementwise and reduction kernels and the multi-level partial join at
that size.

Inputs are seeded on the device with torch's generator (sign-uniform high
parts in [0.5, 1.5), low parts about one unit in the last place); the
oracle recomputes sampled elements, including the ones around 2^31 and the
ragged tail.  The sum is checked three ways: the 1000003-leaf tail's sum
against the oracle; the whole sum against the oracle run on the host over
all 2^31 + 1000003 leaves (16 or 32 GiB of host memory, when available);
and the tree's shape: with n = 2^31 + m the root joins the first 2^31
leaves (an exact power of two of tiles, no padding) with the rest, whose
subtree is the tail's own tree joined with zero subtrees, and
ATF1(v, (+0, +0)) = v, so the whole sum must equal ATF1 of the library's
sums of the two parts.
"""
import numpy as np
import pytest

import oracle
import paper_1401_6235_amd as tf
from gpu_util import assert_bits, step, torch_cuda

pytestmark = pytest.mark.gpu

N_BIG = (1 << 31) + 1000003  # 8 GiB per binary32 array, 16 GiB per binary64 array
GIB = 1 << 30


def _operands(torch, n, seed, dtype, with_y=True):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    dt = torch.float32 if dtype == "f32" else torch.float64
    ulp = 2.0 ** -24 if dtype == "f32" else 2.0 ** -53

    def hi():
        v = torch.rand(n, generator=g, device="cuda", dtype=dt) + 0.5
        sign = torch.randint(0, 2, (n,), generator=g, device="cuda", dtype=torch.int8)
        return torch.where(sign == 1, -v, v)

    def lo(h):
        return h * ((torch.rand(n, generator=g, device="cuda", dtype=dt) * 2 - 1) * ulp)

    x0 = hi()
    x1 = lo(x0)
    if not with_y:
        return x0, x1, None, None
    y0 = hi()
    y1 = lo(y0)
    return x0, x1, y0, y1


def _sample_indices(n, rng):
    edge = [0, 1, 2, 3, (1 << 31) - 2, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, n - 5, n - 4, n - 3, n - 2, n - 1]
    return np.unique(np.concatenate([np.array(edge, np.int64), rng.integers(0, n, 4096)]))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_add_past_2e31_elements(dtype):
    torch = torch_cuda()
    torch.cuda.empty_cache()  # memory cached by earlier tests
    free, _ = torch.cuda.mem_get_info()
    need = (60 if dtype == "f32" else 120) * GIB
    if free < need:
        pytest.skip("needs about %d GiB of free device memory" % (need // GIB))
    step("twofold add %s n = 2^31 + 1000003" % dtype)
    x0, x1, y0, y1 = _operands(torch, N_BIG, 20, dtype)
    z0, z1 = tf.tf_add(x0, x1, y0, y1)
    torch.cuda.synchronize()
    idx = _sample_indices(N_BIG, np.random.default_rng(3))
    ti = torch.from_numpy(idx).cuda()
    host = [t.index_select(0, ti).cpu().numpy() for t in (x0, x1, y0, y1, z0, z1)]
    del x0, x1, y0, y1, z0, z1
    torch.cuda.empty_cache()
    want = oracle.add(*host[:4])
    assert_bits(host[4], want[0], "z0")
    assert_bits(host[5], want[1], "z1")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sum_past_2e31_elements(dtype):
    import psutil
    torch = torch_cuda()
    torch.cuda.empty_cache()  # memory cached by earlier tests
    free, _ = torch.cuda.mem_get_info()
    need = (40 if dtype == "f32" else 80) * GIB
    if free < need:
        pytest.skip("needs about %d GiB of free device memory" % (need // GIB))
    step("twofold sum %s n = 2^31 + 1000003" % dtype)
    x0, x1, _, _ = _operands(torch, N_BIG, 21, dtype, with_y=False)
    whole = tf.tf_sum(x0, x1).cpu().numpy()
    half = 1 << 31
    left = tf.tf_sum(x0[:half], x1[:half]).cpu().numpy()
    right = tf.tf_sum(x0[half:].contiguous(), x1[half:].contiguous()).cpu().numpy()
    # the 1000003-leaf tail straight against the oracle
    step("tail sum %s against the oracle" % dtype)
    tail = [t[half:].cpu().numpy() for t in (x0, x1)]
    assert_bits(right, np.array(oracle.sum(*tail)), "tail sum")
    del tail
    # the whole sum against the oracle on the host, when the host holds both
    # arrays (16 or 32 GiB); otherwise the decomposition below stands alone
    es = 4 if dtype == "f32" else 8
    host_need = 2 * N_BIG * es + 4 * GIB
    if psutil.virtual_memory().available > host_need:
        step("whole sum %s against the oracle on the host" % dtype)
        xh = [t.cpu().numpy() for t in (x0, x1)]
        del x0, x1
        torch.cuda.empty_cache()
        assert_bits(whole, np.array(oracle.sum(*xh)), "whole sum")
        del xh
    else:
        del x0, x1
        torch.cuda.empty_cache()
    assert right[0] != 0 and right[1] != 0  # ATF1(v, 0) = v needs no signed-zero low part
    want = oracle.add(left[:1], left[1:], right[:1], right[1:])
    assert_bits(whole[:1], want[0], "sum z0")
    assert_bits(whole[1:], want[1], "sum z1")
