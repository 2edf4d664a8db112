"""Batched evaluation of many independent encrypted-inference requests.

A request is one run of a workload's ciphertext branch on its own encrypted
inputs (one HW-packed image, or one slot-batched group of images).  The mix
draws each request's workload uniformly from the three parameter sets
(N, primes) = (4096, 2), (8192, 4), (16384, 6).

* per-request path: every request alone, layer by layer, one request at a time;
* batched path: requests of one parameter set share the model (context, keys,
  layers) and are stacked, so each layer runs once over all of them (one launch
  per kernel for the whole group); the groups run on separate streams, so
  kernels of different parameter sets overlap on the device; each group's
  layer pipeline can be captured once into a hipGraph and replayed.

Results are exact, so every request's ciphertexts are identical in both paths.
"""
from __future__ import annotations

import time

import numpy as np

import synthetic

from .workload import GpuSession

MIX = ("cfg1", "cfg2", "cfg3")


def draw_mix(n_requests: int, seed: int = 7, mix=MIX):
    """Workload name of each request, drawn uniformly (stream 'req')."""
    g = synthetic.rng(seed, "req", 0)
    return [mix[i] for i in g.integers(0, len(mix), size=n_requests)]


class Group:
    """Requests of one parameter set: shared model, stacked ciphertexts and features."""

    def __init__(self, session: GpuSession, rids):
        self.s = session
        self.rids = list(rids)
        torch = session.torch
        self.inputs = {r: session.request_inputs(r) for r in self.rids}
        cts = [session.encrypt_request(r, self.inputs[r]) for r in self.rids]
        self.ct = torch.cat(cts) if cts else None
        feats = [session.request_features(self.inputs[r]) for r in self.rids]
        self.features = []
        for li in range(len(session.layers)):
            per = [f[li] for f in feats]
            self.features.append(None if per[0] is None else torch.cat(per))
        self.graph = None
        self.graph_out = None

    def __len__(self):
        return len(self.rids)

    def run_batched(self, chunk: int | None = None):
        """All requests of the group, `chunk` requests per launch group (default: all)."""
        R = len(self.rids)
        chunk = R if not chunk else chunk
        outs = []
        n_in = self.s.n_inputs()
        for lo in range(0, R, chunk):
            hi = min(R, lo + chunk)
            ct = self.ct[lo * n_in:hi * n_in]
            feats = [None if f is None else f[lo * (f.shape[0] // R):hi * (f.shape[0] // R)]
                     for f in self.features]
            outs.append(self.s.run_batch(ct, feats, hi - lo))
        return self.s.torch.cat(outs)

    def run_alone(self, k: int):
        """Request k of the group by itself (the per-request path)."""
        n_in = self.s.n_inputs()
        R = len(self.rids)
        ct = self.ct[k * n_in:(k + 1) * n_in]
        feats = [None if f is None else f[k * (f.shape[0] // R):(k + 1) * (f.shape[0] // R)]
                 for f in self.features]
        return self.s.run_batch(ct, feats, 1)

    def capture(self, chunk: int | None = None):
        """Capture the batched pipeline into a hipGraph (after two eager warm-up runs)."""
        torch = self.s.torch
        self.run_batched(chunk)
        self.run_batched(chunk)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.graph_out = self.run_batched(chunk)
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
        return self.graph_out


class Mix:
    """A request mix over the three parameter sets, with both execution paths."""

    def __init__(self, n_requests: int, seed: int = 7, mix=MIX, autotune: bool = True):
        import torch
        self.torch = torch
        self.names = draw_mix(n_requests, seed, mix)
        self.sessions = {}
        self.groups = {}
        for name in mix:
            rids = [i for i, w in enumerate(self.names) if w == name]
            if not rids:
                continue
            s = GpuSession(name)
            if autotune:
                s.autotune()
            self.sessions[name] = s
            self.groups[name] = Group(s, rids)
        self.streams = {name: torch.cuda.Stream() for name in self.groups}
        torch.cuda.synchronize()

    def run_per_request(self):
        """Every request alone, in arrival order, on one stream."""
        order = {name: 0 for name in self.groups}
        outs = {}
        for rid, name in enumerate(self.names):
            k = order[name]
            order[name] += 1
            outs[rid] = self.groups[name].run_alone(k)
        self.torch.cuda.synchronize()
        return outs

    def run_batched(self, chunks=None, graphs: bool = False):
        """Each parameter set's requests in one stacked pipeline, groups on their own streams."""
        torch = self.torch
        outs = {}
        cur = torch.cuda.current_stream()
        for name, grp in self.groups.items():
            st = self.streams[name]
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                if graphs:
                    outs[name] = grp.replay()
                else:
                    outs[name] = grp.run_batched((chunks or {}).get(name))
        for st in self.streams.values():
            cur.wait_stream(st)
        torch.cuda.synchronize()
        return outs

    def capture(self, chunks=None):
        torch = self.torch
        for name, grp in self.groups.items():
            with torch.cuda.stream(self.streams[name]):
                grp.capture((chunks or {}).get(name))
        torch.cuda.synchronize()

    def transform_phase(self, multi: bool, reps: int = 5) -> float:
        """Forward then inverse transforms of every request's input ciphertexts (all limbs) across
        the parameter sets: one persistent launch per direction over the uneven (N, limbs) work
        list (multi), or each group's own launches on its stream.  Returns ms per phase."""
        torch = self.torch
        from . import bcn
        if not hasattr(self, "_tp"):
            self._tp = {name: grp.ct.clone().reshape(-1, grp.ct.shape[2], grp.ct.shape[3])
                        for name, grp in self.groups.items()}
        items = [(self.sessions[name].ctx, buf, 0) for name, buf in self._tp.items()]
        cur = torch.cuda.current_stream()

        def once():
            if multi:
                bcn.ntt_multi(items)
                bcn.ntt_multi(items, inverse=True)
                return
            for name, buf in self._tp.items():
                st = self.streams[name]
                st.wait_stream(cur)
                with torch.cuda.stream(st):
                    self.sessions[name].ctx.ntt(buf, 0)
                    self.sessions[name].ctx.ntt(buf, 0, inverse=True)
            for st in self.streams.values():
                cur.wait_stream(st)
        once()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    def request_output(self, outs_batched, rid: int):
        """Output ciphertexts of request rid from a batched result."""
        name = self.names[rid]
        grp = self.groups[name]
        k = grp.rids.index(rid)
        n_out = grp.s.n_outputs()
        return outs_batched[name][k * n_out:(k + 1) * n_out]
