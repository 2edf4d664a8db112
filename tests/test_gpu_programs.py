"""End-to-end GPU parity of the workloads' homomorphic programs: every
output ciphertext bit-equal to the oracle's, and Dec(Eval(c)) equal to the
integer-quantised network mod t."""
import numpy as np
import pytest

from oracle import bfv, network, programs

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["cfg1_small", "cfg2_small", "cfg3_small", "cfg3_bhw_small"])
def test_program_parity(name):
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    g = GpuSession(name)
    O = programs.OracleSession(name)
    assert g.steps == O.plan["steps"]
    ct = g.encrypt_inputs()
    ref_in = O.encrypt_inputs()
    got_in = g.ctx.export(ct)
    for i in range(len(ref_in)):
        assert (got_in[i] == bfv.ct_to_rns(O.prm, ref_in[i])).all(), "input %d" % i
    # layer by layer
    cur_o = ref_in
    cur_g = ct
    for li in range(len(g.layers)):
        cur_g = g.layers[li](g.ek, cur_g, g.features[li])
        cur_o = _oracle_layer(O, li, cur_o)
        got = g.ctx.export(cur_g)
        assert got.shape[0] == len(cur_o)
        for k in range(len(cur_o)):
            assert (got[k] == bfv.ct_to_rns(O.prm, cur_o[k])).all(), "layer %d output %d" % (li, k)
    vals = g.output_values(cur_g)
    want = network.run_mod_t(name, g.inputs, O.prm.t)
    assert (vals == want).all()


def _oracle_layer(O, li, cts):
    info = O.plan["layers"][li]
    hw = O.wl["packing"] in ("hw", "bhw")
    if info["kind"] == "conv":
        return O.conv_hw(li, cts) if hw else O.conv_batch(li, cts)
    if hw and "in_slots" in info:
        return O.dense_hw(li, cts)
    return O.dense_scalar(li, cts)
