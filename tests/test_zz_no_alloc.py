"""The allocation-free square + relinearisation (bcn_square_relin_noalloc) against
bcn_square_relin: the same inputs give bit-identical ciphertexts, on two calls in
a row with the second smaller (the fixed scratch array keeps the first call's
contents), and a call too large for the fixed array is refused."""
import numpy as np
import pytest

import synthetic

from gpu_util import context, key_randomness, random_ct_residues, torch_cuda

pytestmark = pytest.mark.gpu


def _setup(pname, seed):
    from paper_2402_01296_amd import bcn
    prm, ctx = context(pname)
    sk = ctx.secret_key(synthetic.ternary_secret(seed, prm.n))
    ek = ctx.eval_keys()
    a, e = key_randomness(prm, seed, 0)
    ctx.keygen(sk, ek, bcn.BCN_KEY_RELIN, 0, np.stack(a), np.stack(e))
    return prm, ctx, ek


@pytest.mark.parametrize("pname,modsw", [("cfg2", True), ("t2k", False)])
def test_noalloc_matches_square_relin(pname, modsw):
    torch = torch_cuda()
    prm, ctx, ek = _setup(pname, 51)
    level = prm.L
    for n, seed in ((5, 911), (2, 912)):
        print("noalloc %s n=%d level=%d modswitch=%s" % (pname, n, level, modsw), flush=True)
        x = ctx.import_(random_ct_residues(prm, level, n, seed))
        ref = ctx.square_relin(ek, x, modswitch=modsw)
        out = ctx.empty_ct(n, level - 1 if modsw else level)
        out.fill_(-1.0)
        ctx.square_relin_noalloc(ek, x, out, modswitch=modsw)
        torch.cuda.synchronize()
        assert bool((out == ref).all()), "n=%d" % n


def test_noalloc_refuses_oversize_calls():
    torch = torch_cuda()
    from paper_2402_01296_amd import bcn
    prm, ctx, ek = _setup("cfg2", 52)
    level = prm.L
    x = torch.zeros((40, 2, level, prm.n), dtype=torch.float64, device="cuda")
    out = ctx.empty_ct(40, level)
    with pytest.raises(bcn.BcnError) as ei:
        ctx.square_relin_noalloc(ek, x, out)
    assert ei.value.code == bcn.BCN_ERR_INVALID
    assert "fixed buffer" in str(ei.value)
