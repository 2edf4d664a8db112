"""The context's scratch arena and captured graphs.  A graph captured once the
arena has settled must keep working after a later, larger call has moved the
arena to a bigger block: the old block is retired, not freed, until the caller
releases it."""
import numpy as np
import pytest

from gpu_util import context, key_randomness, random_ct_residues, torch_cuda

pytestmark = pytest.mark.gpu


def test_graph_survives_arena_growth():
    torch = torch_cuda()
    from paper_2402_01296_amd import bcn
    import synthetic
    prm, ctx = context("t2k")
    sk = ctx.secret_key(synthetic.ternary_secret(41, prm.n))
    ek = ctx.eval_keys()
    a, e = key_randomness(prm, 41, 0)
    ctx.keygen(sk, ek, bcn.BCN_KEY_RELIN, 0, np.stack(a), np.stack(e))
    level = prm.L
    small = ctx.import_(random_ct_residues(prm, level, 2, 901))
    # two eager calls of the captured shape: the first may grow the arena, the second settles it
    ref = ctx.square_relin(ek, small, modswitch=True)
    ref = ctx.square_relin(ek, small, modswitch=True).clone()
    torch.cuda.synchronize()
    before = ctx.scratch_info()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = ctx.square_relin(ek, small, modswitch=True)
    g.replay()
    torch.cuda.synchronize()
    assert bool((out == ref).all())
    assert ctx.scratch_info()["generation"] == before["generation"]
    # a much larger call (about 300 MB of scratch) outgrows the block twice over
    big = ctx.import_(random_ct_residues(prm, level, 256, 902))
    ctx.square_relin(ek, big, modswitch=True)
    ctx.square_relin(ek, big, modswitch=True)
    torch.cuda.synchronize()
    after = ctx.scratch_info()
    assert after["generation"] != before["generation"]
    assert after["base"] != before["base"]
    assert after["retired_bytes"] >= before["bytes"]
    assert after["high_bytes"] > before["bytes"]   # the big calls, since the query before the capture
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert bool((out == ref).all()), "replay %d after the arena moved" % rep
        ctx.square_relin(ek, big[:64], modswitch=True)
        torch.cuda.synchronize()
    del g
    torch.cuda.synchronize()
    ctx.scratch_release()
    assert ctx.scratch_info()["retired_bytes"] == 0
    assert bool((ctx.square_relin(ek, small, modswitch=True) == ref).all())
