"""One persistent transform launch over limbs of several parameter sets (N = 4096,
8192, 16384, each with its own primes): the result equals each context's own
transform, the inverse restores the input, and a captured hipGraph replays it."""
import numpy as np
import pytest

import synthetic

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def _contexts():
    from paper_2402_01296_amd import bcn
    from synthetic import workloads as W
    out = []
    for name in ("t4k", "cfg2", "cfg3"):
        p = W.PARAMS[name]
        out.append(bcn.Context(p["n"], p["bits"], p["L"], p["K"], p["alpha"], p["t"]))
    return out


def _data(torch, ctx, n_polys, seed):
    res = np.stack([synthetic.test_poly(seed, i, ctx.primes[:ctx.L + ctx.K], ctx.n) for i in range(n_polys)])
    return torch.from_numpy(res.astype(np.float64)).cuda()


def test_multi_context_transform_equals_per_context():
    torch = torch_cuda()
    from paper_2402_01296_amd import bcn
    ctxs = _contexts()
    xs = [_data(torch, c, 3 + i, 40 + i) for i, c in enumerate(ctxs)]
    ref = [x.clone() for x in xs]
    for c, r in zip(ctxs, ref):
        c.ntt(r, 0)
    multi = [x.clone() for x in xs]
    bcn.ntt_multi([(c, m, 0) for c, m in zip(ctxs, multi)])
    torch.cuda.synchronize()
    for k in range(3):
        assert bool((multi[k] == ref[k]).all()), "context %d" % k
    bcn.ntt_multi([(c, m, 0) for c, m in zip(ctxs, multi)], inverse=True)
    torch.cuda.synchronize()
    for k in range(3):
        assert bool((multi[k] == xs[k]).all()), "inverse, context %d" % k
    # an item with an offset prime range (the P primes of the middle context)
    c = ctxs[1]
    y = _data(torch, c, 2, 50)[:, c.L:c.L + c.K].contiguous()
    yr = y.clone()
    c.ntt(yr, c.L)
    bcn.ntt_multi([(c, y, c.L)])
    torch.cuda.synchronize()
    assert bool((y == yr).all())


def test_multi_context_transform_graph_replays():
    torch = torch_cuda()
    from paper_2402_01296_amd import bcn
    ctxs = _contexts()
    xs = [_data(torch, c, 2, 60 + i) for i, c in enumerate(ctxs)]
    ref = [x.clone() for x in xs]
    for c, r in zip(ctxs, ref):
        c.ntt(r, 0)
    work = [x.clone() for x in xs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bcn.ntt_multi([(c, w, 0) for c, w in zip(ctxs, work)])      # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bcn.ntt_multi([(c, w, 0) for c, w in zip(ctxs, work)])
    for rep in range(3):
        for w, x in zip(work, xs):
            w.copy_(x)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(3):
            assert bool((work[k] == ref[k]).all()), "replay %d context %d" % (rep, k)
