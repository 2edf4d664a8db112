"""Continuous-batching server: every request's result is identical to the same
request evaluated alone (tolerance zero, the arithmetic is exact), batching
does happen under load, and HBM admission limits the batch size."""
import numpy as np
import pytest

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

SMALL_MIX = ("cfg1_small", "cfg2_small", "cfg3_small")


@pytest.fixture(scope="module")
def server():
    torch_cuda()
    from paper_2402_01296_amd.serve import Server
    return Server(mix=SMALL_MIX, pool=4, autotune=False)


def test_served_results_equal_alone(server):
    from paper_2402_01296_amd.serve import poisson_arrivals
    arrivals = poisson_arrivals(2000.0, 40, seed=5, mix=SMALL_MIX)
    res = server.serve(arrivals, keep_outputs=True)
    assert len(res["latency"]) == 40 and (res["latency"] > 0).all()
    assert max(res["mean_batch"].values()) > 1.0, "no batching happened under load"
    for i, (t, name) in enumerate(arrivals):
        grp = server.pools[name]
        alone = grp.run_alone(i % len(grp))
        assert bool((res["outputs"][i] == alone).all()), "request %d (%s)" % (i, name)


def test_admission_respects_budget(server):
    from paper_2402_01296_amd.serve import poisson_arrivals
    arrivals = poisson_arrivals(5000.0, 12, seed=6, mix=SMALL_MIX)
    name = SMALL_MIX[1]
    # a budget that fits the keys plus exactly two requests of the middle workload
    budget = server.budget
    server.budget = server.key_bytes + 2 * server.req_bytes[name] + 1
    try:
        res = server.serve(arrivals, max_batch={n: 64 for n in SMALL_MIX})
    finally:
        server.budget = budget
    assert len(res["latency"]) == 12
    assert res["mean_batch"].get(name, 1.0) <= 2.0
