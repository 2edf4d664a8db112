"""Continuous-batching server for encrypted-inference requests on one GPU.

Requests of the three parameter sets arrive by a Poisson process.  The server
keeps every model's evaluation keys resident, admits queued requests into a
batch of their parameter set when the batch's HBM footprint fits the budget
(keys plus ciphertext state), and launches the batch on that parameter set's
stream.  Requests that arrive while batches are on the GPU wait only until
their stream can take another batch (at most `depth` batches in flight per
stream), so their work overlaps on the device with the other parameter sets'.
Latency = completion (event observed) - arrival.  Results are exact: a request
returns the same ciphertexts alone or in any batch.
"""
from __future__ import annotations

import collections
import time

import numpy as np

import synthetic

from .batch import MIX, Group
from .workload import GpuSession


def poisson_arrivals(rate: float, n: int, seed: int = 11, mix=MIX):
    """(arrival time in s, workload name) of n requests: exponential gaps, uniform mix."""
    g = synthetic.rng(seed, "req", int(rate))
    gaps = g.exponential(1.0 / rate, size=n)
    names = g.integers(0, len(mix), size=n)
    return list(zip(np.cumsum(gaps).tolist(), [mix[i] for i in names]))


class Server:
    def __init__(self, mix=MIX, pool: int = 8, hbm_budget: float = 200e9, max_batch=None, depth: int = 2,
                 autotune: bool = True):
        import torch
        self.torch = torch
        self.mix = mix
        self.budget = hbm_budget
        self.depth = depth
        self.max_batch = dict(max_batch or {})
        self.sessions, self.pools, self.streams = {}, {}, {}
        self.req_bytes, self.key_bytes = {}, 0
        for name in mix:
            s = GpuSession(name)
            if autotune:
                s.autotune()
            self.sessions[name] = s
            # a pool of distinct pre-encrypted requests; arrivals reuse them cyclically
            self.pools[name] = Group(s, range(pool))
            self.streams[name] = torch.cuda.Stream()
            self.key_bytes += self._key_bytes(s)
        torch.cuda.synchronize()
        for name in mix:
            self.req_bytes[name] = self._measure_request_bytes(name)

    @staticmethod
    def _key_bytes(s: GpuSession) -> int:
        c = s.ctx
        per_key = c.dnum() * 2 * (c.L + c.K) * c.n * 8
        return per_key * (1 + len(s.steps))

    def _measure_request_bytes(self, name: str) -> int:
        """Upper bound of one request's device bytes: the largest layer working set
        (inputs, outputs, rotation taps and key-switching buffers, the square's
        extended / tensor / rounded / key-switching intermediates)."""
        s = self.sessions[name]
        c = s.ctx
        n, K, m = c.n, c.K, c.n_aux
        worst = 0
        for lay in s.layers:
            lv = lay.level
            ct = 2 * lv * n * 8
            dn = c.dnum(lv)
            b = (lay.n_in + lay.n_out) * ct
            conv_hw = lay.desc.packing == 1 and lay.desc.kind == 0
            if conv_hw:
                k2 = lay.desc.k * lay.desc.k
                b += lay.n_in * k2 * ct                                        # taps
                b += lay.n_in * (dn * (lv + K) + (k2 - 1) * 2 * (lv + K)) * n * 8   # digits + products
            if lay.desc.square:
                b += lay.n_out * (5 * (lv + m) + 3 * lv + (dn + 2) * (lv + K)) * n * 8
            if lay.steps:
                b += lay.n_out * (dn + 2) * (lv + K) * n * 8 + lay.n_out * ct       # rotate-and-sum
            worst = max(worst, b)
        return int(worst)

    def footprint(self, name: str, r: int) -> int:
        return self.req_bytes[name] * r

    def _stack(self, name: str, ks):
        torch = self.torch
        grp = self.pools[name]
        R = len(grp)
        n_in = grp.s.n_inputs()
        ct = torch.cat([grp.ct[k * n_in:(k + 1) * n_in] for k in ks])
        feats = []
        for f in grp.features:
            if f is None:
                feats.append(None)
            else:
                per = f.shape[0] // R
                feats.append(torch.cat([f[k * per:(k + 1) * per] for k in ks]))
        return ct, feats

    def serve(self, arrivals, keep_outputs: bool = False, max_batch=None):
        """Runs the trace in real time; returns per-request latencies (s) and summary numbers."""
        torch = self.torch
        max_batch = dict(self.max_batch, **(max_batch or {}))
        pending = collections.deque(sorted((t, i, name) for i, (t, name) in enumerate(arrivals)))
        queues = {name: collections.deque() for name in self.mix}
        inflight = {name: collections.deque() for name in self.mix}
        used = 0
        latency = {}
        outputs = {}
        batches = []
        n_total = len(arrivals)
        t0 = time.perf_counter()
        done = 0
        while done < n_total:
            now = time.perf_counter() - t0
            while pending and pending[0][0] <= now:
                t, i, name = pending.popleft()
                queues[name].append((t, i))
            progressed = False
            for name in self.mix:
                fl = inflight[name]
                while fl and fl[0]["event"].query():
                    b = fl.popleft()
                    fin = time.perf_counter() - t0
                    for (t, i) in b["reqs"]:
                        latency[i] = fin - t
                    if keep_outputs:
                        # copy on the batch's own stream: the output block returns to that
                        # stream's allocator pool when the batch is dropped, so a copy on another
                        # stream could race with the next batch reusing the block
                        n_out = self.sessions[name].n_outputs()
                        with torch.cuda.stream(self.streams[name]):
                            for j, (t, i) in enumerate(b["reqs"]):
                                outputs[i] = b["out"][j * n_out:(j + 1) * n_out].clone()
                    used -= b["bytes"]
                    done += len(b["reqs"])
                    progressed = True
            for name in self.mix:
                q = queues[name]
                if not q or len(inflight[name]) >= self.depth:
                    continue
                r = min(len(q), max_batch.get(name, 64))
                while r > 0 and used + self.key_bytes + self.footprint(name, r) > self.budget:
                    r -= 1
                if r == 0:
                    continue
                reqs = [q.popleft() for _ in range(r)]
                pool = len(self.pools[name])
                ks = [i % pool for (t, i) in reqs]
                st = self.streams[name]
                with torch.cuda.stream(st):
                    ct, feats = self._stack(name, ks)
                    out = self.sessions[name].run_batch(ct, feats, r)
                    ev = torch.cuda.Event()
                    ev.record(st)
                by = self.footprint(name, r)
                used += by
                inflight[name].append(dict(event=ev, reqs=reqs, out=out, bytes=by))
                batches.append((name, r))
                progressed = True
            if not progressed:
                time.sleep(0.0001)
        elapsed = time.perf_counter() - t0
        torch.cuda.synchronize()
        lat = np.array([latency[i] for i in range(n_total)])
        sizes = collections.Counter(n for n, _ in batches)
        mean_batch = {k: float(np.mean([r for n, r in batches if n == k])) for k in sizes}
        return dict(latency=lat, outputs=outputs, elapsed=elapsed, throughput=n_total / elapsed,
                    p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                    batches=len(batches), mean_batch=mean_batch)
