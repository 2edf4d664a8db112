"""End-to-end GPU parity of the workloads' homomorphic programs: every
output ciphertext bit-equal to the oracle's, and Dec(Eval(c)) equal to the
integer-quantised network mod t."""
import numpy as np
import pytest

from oracle import bfv, network, programs

from gpu_util import export_rows, oracle_rows, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["cfg1_small", "cfg2_small", "cfg3_small", "cfg3_bhw_small", "cfg2_bi_small",
                                  "fc_diag_small", "cfg3_pool_small"])
def test_program_parity(name):
    torch_cuda()
    from paper_2402_01296_amd.workload import GpuSession
    from synthetic import workloads as W
    g = GpuSession(name)
    # a plaintext branch's FP32 outputs are inputs of the ciphertext branch: both sides take the
    # same ones (the plaintext branch itself is checked against its FP64 reference)
    pf = {key: g.inputs["features"][li] for li, key in W.plain_feature_layers(name).items()} or None
    O = programs.OracleSession(name, plain_features=pf)
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
        got = export_rows(g.ctx, cur_g)
        assert got.shape[0] == len(cur_o)
        for k in range(len(cur_o)):
            assert (got[k] == oracle_rows(O.prm, cur_o[k])).all(), "layer %d output %d" % (li, k)
    vals = g.output_values(cur_g)
    want = network.run_mod_t(name, g.inputs, O.prm.t)
    assert (vals == want).all()


def _oracle_layer(O, li, cts):
    info = O.plan["layers"][li]
    hw = O.wl["packing"] in ("hw", "bhw")
    if info["kind"] == "pool":
        return O.pool_hw(li, cts)
    if info.get("method") == "diag":
        return O.dense_diag(li, cts)
    if info["kind"] == "conv":
        return O.conv_hw(li, cts) if hw else O.conv_batch(li, cts)
    if hw and "in_slots" in info:
        return O.dense_hw(li, cts)
    return O.dense_scalar(li, cts)


def test_bi_model_overlapped_equals_serial_and_network():
    """The whole bi-CryptoNets model: plaintext branch (FP32) on a side stream in parallel with
    the ciphertext branch; the same ciphertexts as the serial run, the plaintext side within FP32
    rounding of its FP64 reference, and Dec(Eval) equal to the integer network mod t."""
    torch = torch_cuda()
    from oracle import plain
    from paper_2402_01296_amd.workload import GpuSession
    name = "cfg2_bi_small"
    g = GpuSession(name)
    ref = plain.run(name, g.inputs)
    outs = g.plain(*g.plain_inputs(g.inputs))
    for k in ("z1", "u1", "u2"):
        a = outs[k].cpu().numpy().astype(np.float64)
        assert np.abs(a - ref[k]).max() <= 1e-4 * max(1.0, np.abs(ref[k]).max()), k
    ct = g.encrypt_inputs()
    serial = g.run(ct)
    side = torch.cuda.Stream()
    images, noise = g.plain_inputs(g.inputs)
    for _ in range(2):
        over = g.run_bi(ct, images, noise, side)
        torch.cuda.synchronize()
        assert bool((over == serial).all())
    vals = g.output_values(over)
    want = network.run_mod_t(name, g.inputs, g.ctx.t)
    assert (vals == want).all()


@pytest.mark.parametrize("tile", [2, 4, 8, 16])
@pytest.mark.parametrize("fused", [1, 0])
def test_batch_square_layer_mac_tiles(tile, fused, monkeypatch):
    """A slot-batched square layer's MAC at each tile, with the extension to Q+B fused into its
    stores or run as its own kernel: the layer's outputs bit-equal to the oracle's."""
    torch_cuda()
    monkeypatch.setenv("BCN_MAC_TILE", str(tile))
    monkeypatch.setenv("BCN_MAC_EXT", str(fused))
    from paper_2402_01296_amd.workload import GpuSession
    name = "cfg2_small"
    g = GpuSession(name)
    O = programs.OracleSession(name)
    ct = g.encrypt_inputs()
    cur_o = O.encrypt_inputs()
    for li in range(2):
        ct = g.layers[li](g.ek, ct, g.features[li])
        cur_o = _oracle_layer(O, li, cur_o)
        got = export_rows(g.ctx, ct)
        for k in range(len(cur_o)):
            assert (got[k] == oracle_rows(O.prm, cur_o[k])).all(), "layer %d output %d" % (li, k)
