"""Continuous-batching server for encrypted-inference requests on one GPU.

Requests of the three parameter sets arrive by a Poisson process.  The server
keeps every model's evaluation keys resident, admits queued requests into a
batch of their parameter set when the device bytes of everything in flight fit
the budget (keys plus ciphertext state), and launches the batch on that
parameter set's stream.  A request that finds its stream idle is launched at
once; requests that arrive while a batch of their parameter set runs wait at
most `window` seconds (the latency budget) or until `max_batch` of them are
queued, then share one launch as the next batch (at most `depth` batches in
flight per stream), and their work overlaps on the device with the other
parameter sets'.  Per-request device bytes are measured, not modelled: the
scratch arena's high-water mark plus torch's peak allocation for batches of one
and two requests.  Latency = completion (event observed) - arrival.  Results
are exact: a request returns the same ciphertexts alone or in any batch.
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
                 autotune: bool = True, window: float = 0.002):
        import torch
        self.torch = torch
        self.mix = mix
        self.budget = hbm_budget
        self.depth = depth
        self.window = window
        self.max_batch = dict(max_batch or {})
        self.sessions, self.pools, self.streams = {}, {}, {}
        self.req_bytes, self.req_fixed, self.key_bytes = {}, {}, 0
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
            self.req_fixed[name], self.req_bytes[name] = self._measure_request_bytes(name)

    def close(self):
        self.torch.cuda.synchronize()
        self.sessions.clear()
        self.pools.clear()
        self.torch.cuda.empty_cache()

    @staticmethod
    def _key_bytes(s: GpuSession) -> int:
        c = s.ctx
        per_key = c.dnum() * 2 * (c.L + c.K) * c.n * 8
        return per_key * (1 + len(s.steps))

    def _measure_request_bytes(self, name: str):
        """(fixed, per-request) device bytes of a batch of this parameter set, measured: for
        batches of one and two requests, the largest scratch any library call used (the
        context's arena high-water mark) plus torch's peak allocation above the resident state
        (stacked inputs, every layer's outputs).  The two points give the slope and intercept."""
        torch = self.torch
        s = self.sessions[name]
        tot = {}
        for r in (1, 2, 1, 2):     # the first pair settles the arena and allocator
            torch.cuda.synchronize()
            torch.cuda.reset_peak_memory_stats()
            base = torch.cuda.memory_allocated()
            s.ctx.scratch_info()                     # restarts the per-call high-water mark
            ct, feats = self._stack(name, list(range(r)))
            s.run_batch(ct, feats, r)
            torch.cuda.synchronize()
            peak = torch.cuda.max_memory_allocated() - base
            tot[r] = peak + s.ctx.scratch_info()["high_bytes"]
            del ct, feats
        per = max(1, tot[2] - tot[1])
        return int(max(0, tot[1] - per)), int(per)

    def footprint(self, name: str, r: int) -> int:
        return self.req_fixed[name] + self.req_bytes[name] * r

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

    def serve(self, arrivals, keep_outputs: bool = False, max_batch=None, window=None):
        """Runs the trace in real time; returns per-request latencies (s) and summary numbers."""
        torch = self.torch
        max_batch = dict(self.max_batch, **(max_batch or {}))
        window = self.window if window is None else window
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
                mb = max_batch.get(name, 64)
                # an idle stream takes the queue at once; a busy one waits for a full batch or
                # until the oldest queued request has used up the window
                if inflight[name] and len(q) < mb and now - q[0][0] < window:
                    continue
                r = min(len(q), mb)
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
