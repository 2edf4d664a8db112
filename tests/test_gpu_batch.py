"""Batched multi-request evaluation: every request's ciphertexts are identical
whether it runs alone, stacked with others of its parameter set, on its own
stream next to other parameter sets, or replayed from a captured hipGraph;
and each request decrypts to its own integer network."""
import numpy as np
import pytest

from oracle import network

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

SMALL_MIX = ("cfg1_small", "cfg2_small", "cfg3_small")


@pytest.fixture(scope="module")
def mix():
    torch_cuda()
    from paper_2402_01296_amd.batch import Mix
    return Mix(8, seed=3, mix=SMALL_MIX, autotune=False)


def test_batched_equals_alone(mix):
    alone = mix.run_per_request()
    batched = mix.run_batched(chunks={"cfg2_small": 2})
    for rid in range(len(mix.names)):
        a = alone[rid]
        b = mix.request_output(batched, rid)
        assert a.shape == b.shape
        assert bool((a == b).all()), "request %d (%s)" % (rid, mix.names[rid])


def test_requests_decrypt_to_their_networks(mix):
    batched = mix.run_batched()
    for rid, name in enumerate(mix.names):
        s = mix.sessions[name]
        vals = s.output_values(mix.request_output(batched, rid))
        want = network.run_mod_t(name, s.request_inputs(rid), s.ctx.t)
        assert (vals == want).all(), "request %d (%s)" % (rid, name)


def test_graph_replays_equal_eager(mix):
    torch = mix.torch
    eager = mix.run_batched()
    eager = {k: v.clone() for k, v in eager.items()}
    mix.capture()
    for rep in range(3):
        out = mix.run_batched(graphs=True)
        for name in eager:
            assert bool((out[name] == eager[name]).all()), "replay %d of %s" % (rep, name)
        # eager work and a synchronisation between replays
        _ = mix.run_batched()
        torch.cuda.synchronize()
