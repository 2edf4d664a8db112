"""Writes tests/golden/<workload>_fullsize.json: SHA-256 digests of every ciphertext the
oracle computes for a workload at its full size (the encrypted inputs and every layer's
outputs), from the workload's seeded synthetic inputs.  Only oracle/ and the seeded input
generators are called.  The GPU tests compare the digests of their own exported
ciphertexts (coefficient form, [2][level][N] little-endian uint64) with these.

Usage: python tests/golden/make_fullsize_digests.py cfg2|cfg3 [workers]
The oracle is slow at these sizes: the work is spread over worker processes (fork).
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bfv, programs  # noqa: E402

_S = {}


def digest(prm, ct) -> str:
    """Of the [parts][level][N] residues (two parts, or three for an unrelinearised product)."""
    parts = [ct.c0, ct.c1] + ([ct.c2] if hasattr(ct, "c2") else [])
    res = np.stack([bfv.to_rns(p, prm.q[:ct.level]) for p in parts])
    return hashlib.sha256(np.ascontiguousarray(res, dtype="<u8").tobytes()).hexdigest()


def _encrypt(i):
    O = _S["O"]
    return i, O.encrypt_slots(_S["slots"][i], i)


def _extend(c):
    O = _S["O"]
    return c, O.extended_input(_S["li"], _S["cts"][c])


def _layer_output(o):
    O, li, kind = _S["O"], _S["li"], _S["kind"]
    if kind == "conv_hw":
        return o, O.conv_hw(li, _S["cts"], outputs=[o], ext=_S["ext"])[o]
    if kind == "conv_batch":
        return o, O.conv_batch(li, _S["cts"], outputs=[o])[o]
    if kind == "dense_hw":
        return o, O.dense_hw(li, _S["cts"], outputs=[o])[o]
    return o, O.dense_scalar(li, _S["cts"], outputs=[o])[o]


def _pool_map(fn, items, workers):
    with mp.get_context("fork").Pool(workers) as pool:
        return dict(pool.map(fn, items, chunksize=1))


def main():
    name = sys.argv[1]
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    t0 = time.time()
    O = programs.OracleSession(name)
    prm = O.prm
    print("%s: keys ready in %.0fs" % (name, time.time() - t0), flush=True)
    _S.update(O=O, slots=O.input_slots())
    cts = _pool_map(_encrypt, list(range(len(_S["slots"]))), workers)
    out = {"workload": name, "n": prm.n, "format": "sha256 of the [parts][level][N] little-endian uint64 residues (parts 3: unrelinearised)",
           "layers": [{"what": "encrypted inputs", "level": prm.L,
                       "digests": [digest(prm, cts[i]) for i in sorted(cts)]}]}
    print("%s: %d inputs encrypted at %.0fs" % (name, len(cts), time.time() - t0), flush=True)
    hw = O.wl["packing"] == "hw"
    spatial = True
    for li, info in enumerate(O.plan["layers"]):
        _S.update(li=li, cts=cts)
        if info["kind"] == "conv":
            n_out = info["out_shape"][0] if hw else int(np.prod(info["out_shape"]))
            if hw:
                _S["ext"] = _pool_map(_extend, sorted(cts), workers)
                _S["kind"] = "conv_hw"
                if info.get("sum"):
                    spatial = False
            else:
                _S["kind"] = "conv_batch"
        elif hw and spatial:
            n_out, _S["kind"] = info["out"], "dense_hw"
            spatial = False
        else:
            n_out, _S["kind"] = info["out"], "dense_scalar"
        cts = _pool_map(_layer_output, list(range(n_out)), workers)
        _S.pop("ext", None)
        level = cts[0].level
        out["layers"].append({"what": "outputs of layer %d (%s)" % (li + 1, _S["kind"]), "level": level,
                              "digests": [digest(prm, cts[o]) for o in range(n_out)]})
        print("%s: layer %d (%d outputs, level %d) at %.0fs" % (name, li + 1, n_out, level, time.time() - t0),
              flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "%s_fullsize.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote %s in %.0fs" % (path, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
