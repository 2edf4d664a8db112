"""Helpers shared by the GPU parity tests."""
import numpy as np
import pytest

import synthetic
from oracle import bfv, params


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def context(pname):
    from paper_2402_01296_amd import bcn
    spec = params.get(pname)
    bits = spec.q[0].bit_length()
    ctx = bcn.Context(spec.n, bits, spec.L, spec.K, spec.alpha, spec.t)
    assert ctx.q == list(spec.q) and ctx.p_primes == list(spec.p), "prime rule differs from the oracle's"
    return spec, ctx


def random_ct_residues(prm, level, n, seed):
    """[n][2][level][N] uniform residues (a random element of R_Q^2, not an encryption)."""
    out = np.zeros((n, 2, level, prm.n), dtype=np.uint64)
    for i in range(n):
        for part in range(2):
            out[i, part] = synthetic.test_poly(seed, 2 * i + part, prm.q[:level], prm.n)
    return out


def oracle_ct(prm, res):
    """Oracle Ct from [2][level][N] residues."""
    level = res.shape[1]
    return bfv.Ct(bfv.from_rns(res[0], prm.q[:level]), bfv.from_rns(res[1], prm.q[:level]), level)


def key_randomness(prm, seed, key_id):
    moduli = list(prm.q) + list(prm.p)
    d = prm.dnum(prm.L)
    a = [synthetic.uniform_residues(seed, "ksk_a", (key_id, j), moduli, prm.n) for j in range(d)]
    e = [synthetic.gaussian_error(seed, "ksk_e", (key_id, j), prm.n) for j in range(d)]
    return a, e


def export_rows(ctx, t):
    """Coefficient-form residues of device rows [n][parts][level][N] (parts 2, or 3 for
    unrelinearised products) as uint64 [n][parts][level][N]."""
    parts = t.shape[1]
    if parts == 2:
        return ctx.export(t)
    a = ctx.export(t[:, 0:2].contiguous())
    b = ctx.export(t[:, 1:3].contiguous())
    return np.concatenate([a, b[:, 1:2]], axis=1)


def oracle_rows(prm, ct):
    """[parts][level][N] residues of an oracle Ct or Ct3."""
    parts = [ct.c0, ct.c1] + ([ct.c2] if hasattr(ct, "c2") else [])
    return np.stack([bfv.to_rns(p, prm.q[:ct.level]) for p in parts])
