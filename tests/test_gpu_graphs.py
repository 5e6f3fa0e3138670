"""GPU: twofold calls captured once in a HIP graph (torch.cuda.CUDAGraph)
and replayed.  The library launches only kernels (no memset, no
allocation, no synchronisation), so a sequence of calls can be captured on
the caller's stream; every replay must equal the eager calls bit for bit,
with fresh inputs copied in and eager work in between the replays."""
import numpy as np
import pytest

import paper_1401_6235_amd as tf
from gpu_util import assert_bits, step, to_gpu, to_np, torch_cuda
from paper_1401_6235_amd import workloads as W

pytestmark = pytest.mark.gpu


def _pipeline(d, o):
    """add -> Dekker mul -> twofold sum of the product, plus a chain."""
    tf.tf_add(d["x0"], d["x1"], d["y0"], d["y1"], o["a0"], o["a1"])
    tf.tf_coupled("mul", o["a0"], o["a1"], d["y0"], d["y1"], renorm=True, z0=o["m0"], z1=o["m1"])
    tf.tf_sum(o["m0"], o["m1"], o["s"], o["work"])
    tf.tf_chain("div", "twofold", 16, d["x0"], d["x1"], d["y0"], d["y1"], o["c0"], o["c1"])


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_graph_replays_equal_eager_calls(dtype):
    torch = torch_cuda()
    n = (1 << 20) + 37
    c = W.elementwise("div", n, seed=31, dtype=dtype)
    d = {k: to_gpu(v) for k, v in c.items()}

    def outputs():
        o = {k: torch.empty_like(d["x0"]) for k in ("a0", "a1", "m0", "m1", "c0", "c1")}
        o["s"] = torch.empty(2, dtype=d["x0"].dtype, device="cuda")
        o["work"] = tf.workspace(d["x0"])
        return o

    eager, graphed = outputs(), outputs()
    step("graph eager reference %s" % np.dtype(dtype))
    _pipeline(d, eager)  # also loads every kernel before the capture
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            _pipeline(d, graphed)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()

    for rep in range(4):
        fresh = W.elementwise("div", n, seed=100 + rep, dtype=dtype)
        for k, v in fresh.items():
            d[k].copy_(torch.from_numpy(v))
        step("graph replay %d %s" % (rep, np.dtype(dtype)))
        g.replay()
        torch.cuda.synchronize()
        _pipeline(d, eager)  # eager work between replays
        torch.cuda.synchronize()
        for k in ("a0", "a1", "m0", "m1", "s", "c0", "c1"):
            assert_bits(to_np(graphed[k]), to_np(eager[k]), "replay %d %s" % (rep, k))
