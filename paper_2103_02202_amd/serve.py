"""Continuous-batching sampling server over the C ABI.

The server keeps a pool of compiled circuits resident on the GPU (programs and
reference samples uploaded once) and serves detection-event sampling requests
as they arrive:

* Admission by HBM footprint: a request's device memory -- its detection-event
  and observable outputs plus the scratch the library reports for the call
  (flip record, noise records of the pre-pass, and the frame scratch when the
  frame is too large for LDS) -- is reserved
  against a byte budget; requests that do not fit wait (a deferral) until
  earlier work completes and releases memory.
* Chunking: a request is split along the shot axis into chunks of at most
  ``max_chunk_shots`` shots and ``max_chunk_bytes`` of footprint (results are
  identical because random bits are keyed by absolute shot); the request
  completes with its last chunk.
* Continuous batching: whenever a launch slot (a HIP stream) is free, the
  admitted small chunks that have arrived are submitted together as one
  persistent batched launch (stim_batch_sample) on that slot.  Chunks that
  arrive while others run start on the next free slot, so their work overlaps
  on the device.  Big chunks (at least ``big_work`` shot-gates) take slot 0
  one at a time: a large circuit's frames fill the GPU and its last-level
  cache on their own, and two of them side by side only slow each other down.
* Sampling method per circuit: ``Server.calibrate`` times each large pool
  circuit's detection events through the frame path and through sparse
  detection sampling (identical results, Sec. 5.6) and keeps the faster.
  Chunks of a circuit served by sparse sampling launch one per slot; they
  need no flip record or frame scratch, so their footprint is the outputs.
* Latency: arrival (the request's scheduled Poisson time) to the completion of
  its last chunk, observed by polling HIP events; p50 / p99 reported beside
  throughput.

``Server.serve_one_at_a_time`` is the comparison point: one stream, requests in
arrival order, each launched alone and waited for.
"""
from __future__ import annotations

import math
import time
from concurrent.futures import ThreadPoolExecutor

from . import stim_gpu


class PoolCircuit:
    def __init__(self, text: str, name: str):
        self.name = name
        self.c = stim_gpu.Circuit(text)
        self.c.reference()              # host analysis happens once, at pool load
        self.method = "frame"           # or "sparse" (see Server.calibrate)

    def footprint(self, shots: int) -> int:
        """HBM one chunk holds while in flight: its outputs plus the scratch
        the library takes for it (flip table, noise records, global frame)."""
        W = (shots + 63) // 64
        c = self.c
        out = 8 * W * (c.num_detectors + max(c.num_observables, 1))
        return out + c.scratch_bytes(shots, "sparse" if self.method == "sparse" else "detector")

    def sample(self, seed, offset, shots, det, obs, stream):
        """Detection events of one chunk by this circuit's method."""
        fn = stim_gpu.stim_sparse_detector_sample if self.method == "sparse" else stim_gpu.stim_detector_sample
        fn(self.c.handle, seed, offset, shots, det, obs, stream)


def load_pool(texts, names=None, threads: int = 8):
    """Compiles circuits (and their reference samples) in parallel host threads."""
    names = names or [str(i) for i in range(len(texts))]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda tn: PoolCircuit(*tn), zip(texts, names)))


def percentile(values, q):
    """The q-th percentile (linear interpolation), or None for no values."""
    if not values:
        return None
    v = sorted(values)
    k = (len(v) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


class Server:
    def __init__(self, pool, hbm_budget_bytes: int = 48 << 30, num_slots: int = 4,
                 max_chunk_shots: int = 1 << 18, max_chunk_bytes: int | None = None, max_group: int = 64,
                 max_group_shot_gates: float = 4e10, keep_outputs: bool = False, big_work: float = 1e11):
        import torch
        self.torch = torch
        self.pool = pool
        self.budget = hbm_budget_bytes
        self.slots = [torch.cuda.Stream() for _ in range(num_slots)]      # default priority
        self.max_chunk = max(64, (max_chunk_shots // 64) * 64)
        self.max_chunk_bytes = max_chunk_bytes or max(hbm_budget_bytes // 8, 1)
        self.max_group = max_group
        self.max_group_work = max_group_shot_gates
        self.keep_outputs = keep_outputs
        self.big_work = big_work

    # -- method per circuit ---------------------------------------------------
    def calibrate(self, shots: int = 1 << 16, min_qubits: int = 1000, gain: float = 1.2):
        """Times frame and sparse detection sampling of `shots` shots for every
        pool circuit of at least `min_qubits` qubits and switches it to sparse
        sampling when that is at least `gain` times faster.  Returns
        {name: (frame_ms, sparse_ms or None, method)}."""
        torch = self.torch
        out = {}
        for pc in self.pool:
            c = pc.c
            if c.num_qubits < min_qubits:
                continue
            try:
                c.error_sets()                     # builds them, or refuses the circuit
            except stim_gpu.StimError:
                out[pc.name] = (None, None, pc.method)
                continue
            W = (shots + 63) // 64
            det = torch.empty((c.num_detectors, W), dtype=torch.int64, device="cuda")
            obs = torch.empty((max(c.num_observables, 1), W), dtype=torch.int64, device="cuda")
            times = {}
            for name, fn in (("frame", stim_gpu.stim_detector_sample),
                             ("sparse", stim_gpu.stim_sparse_detector_sample)):
                fn(c.handle, 0, 0, shots, det, obs)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(2):
                    fn(c.handle, 0, 0, shots, det, obs)
                torch.cuda.synchronize()
                times[name] = (time.perf_counter() - t0) / 2 * 1e3
            if times["frame"] >= gain * times["sparse"]:
                pc.method = "sparse"
            out[pc.name] = (times["frame"], times["sparse"], pc.method)
        return out

    def _is_big(self, ch):
        return ch["pc"].method == "frame" and ch["work"] >= self.big_work

    # -- chunks -------------------------------------------------------------
    def _chunks(self, req):
        pc = self.pool[req["circuit"]]
        words = (self.max_chunk + 63) // 64
        per_word = max(pc.footprint(words * 64) / words, 1.0)
        cap = max(64, min(self.max_chunk, int(self.max_chunk_bytes // per_word) * 64))
        out = []
        off = 0
        while off < req["shots"]:
            n = min(cap, req["shots"] - off)
            out.append({"req": req, "pc": pc, "offset": off, "shots": n, "bytes": pc.footprint(n),
                        "work": pc.c.num_gate_targets * n, "deferred": False})
            off += n
        return out

    def _alloc(self, ch):
        torch = self.torch
        c = ch["pc"].c
        W = (ch["shots"] + 63) // 64
        ch["det"] = torch.empty((c.num_detectors, W), dtype=torch.int64, device="cuda")
        ch["obs"] = torch.empty((max(c.num_observables, 1), W), dtype=torch.int64, device="cuda")

    def _request_dict(self, ch):
        return {"handle": ch["pc"].c.handle, "seed": ch["req"]["seed"], "shot_offset": ch["offset"],
                "num_shots": ch["shots"], "mode": 1, "out0": ch["det"], "out1": ch["obs"]}

    def _finish(self, ch, now, stats):
        req = ch["req"]
        req["_left"] -= 1
        if not self.keep_outputs:
            ch["det"] = ch["obs"] = None
        if req["_left"] == 0:
            req["completion"] = now
            stats["latencies"].append(now - req["arrival"])

    # -- continuous batching -----------------------------------------------
    def serve(self, requests, time_scale: float = 1.0):
        """Serves `requests` (dicts with arrival [s], circuit, shots, seed),
        replaying their arrival times in real time.  Returns statistics."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r["arrival"])
        for r in reqs:
            r["_left"] = 0
            r["chunks"] = []
        stats = {"latencies": [], "deferrals": 0, "launches": 0, "chunks": 0, "max_group": 0}
        pending = []                                   # arrived, not yet admitted (FIFO)
        inflight = []                                  # (slot index, event, chunks, bytes)
        free_slots = list(range(len(self.slots)))
        used = 0
        nxt = 0
        done = 0
        total = len(reqs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done < total:
            now = time.perf_counter() - t0
            while nxt < total and reqs[nxt]["arrival"] * time_scale <= now:
                chs = self._chunks(reqs[nxt])
                reqs[nxt]["_left"] = len(chs)
                reqs[nxt]["chunks"] = chs
                pending.extend(chs)
                nxt += 1
            # completions
            still = []
            for slot, ev, chs, nbytes in inflight:
                if ev.query():
                    t = time.perf_counter() - t0
                    for ch in chs:
                        if ch["req"]["_left"] == 1:
                            done += 1
                        self._finish(ch, t / time_scale if time_scale else t, stats)
                    used -= nbytes
                    free_slots.append(slot)
                else:
                    still.append((slot, ev, chs, nbytes))
            inflight = still
            # admissions: big chunks one at a time on slot 0; small chunks in
            # groups on the other slots, FIFO, bounded in work so that a
            # launch stays short and later arrivals start soon
            while free_slots and pending:
                bigs = [ch for ch in pending if self._is_big(ch)]
                smalls = [ch for ch in pending if not self._is_big(ch)]
                small_slots = [x for x in free_slots if x != 0]
                if 0 in free_slots and not bigs:
                    small_slots.append(0)            # no big chunk waiting: slot 0 takes small ones too
                if len(self.slots) == 1:
                    slot, queue = 0, list(pending)
                elif 0 in free_slots and bigs:
                    slot, queue = 0, bigs
                elif smalls and small_slots:
                    slot, queue = small_slots[0], smalls
                else:
                    break
                big_slot = self._is_big(queue[0])
                method = queue[0]["pc"].method
                if big_slot or method == "sparse":         # one chunk per launch
                    limit_n, limit_w = 1, float("inf")
                else:
                    limit_n, limit_w = self.max_group, self.max_group_work
                group, gbytes, gwork = [], 0, 0.0
                while (queue and len(group) < limit_n and used + gbytes + queue[0]["bytes"] <= self.budget
                       and (not group or gwork + queue[0]["work"] <= limit_w)
                       and self._is_big(queue[0]) == big_slot and queue[0]["pc"].method == method):
                    ch = queue.pop(0)
                    group.append(ch)
                    gbytes += ch["bytes"]
                    gwork += ch["work"]
                if not group:
                    if not inflight:         # a chunk larger than the whole budget: run it alone
                        group = [queue.pop(0)]
                        gbytes = group[0]["bytes"]
                    else:
                        if not queue[0]["deferred"]:
                            queue[0]["deferred"] = True
                            stats["deferrals"] += 1
                        break
                taken = {id(ch) for ch in group}
                pending = [ch for ch in pending if id(ch) not in taken]
                free_slots.remove(slot)
                stream = self.slots[slot]
                with torch.cuda.stream(stream):
                    for ch in group:
                        self._alloc(ch)
                if group[0]["pc"].method == "sparse":
                    ch = group[0]
                    ch["pc"].sample(ch["req"]["seed"], ch["offset"], ch["shots"], ch["det"], ch["obs"], stream)
                else:
                    stim_gpu.stim_batch_sample([self._request_dict(ch) for ch in group], stream=stream)
                ev = torch.cuda.Event()
                ev.record(stream)
                inflight.append((slot, ev, group, gbytes))
                used += gbytes
                stats["launches"] += 1
                stats["chunks"] += len(group)
                stats["max_group"] = max(stats["max_group"], len(group))
            if not inflight and not pending and nxt < total:
                wait = reqs[nxt]["arrival"] * time_scale - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.002))
        torch.cuda.synchronize()
        stats["makespan_s"] = time.perf_counter() - t0
        return self._summary(reqs, stats)

    # -- comparison: one request at a time ----------------------------------
    def serve_one_at_a_time(self, requests, time_scale: float = 1.0):
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r["arrival"])
        stats = {"latencies": [], "deferrals": 0, "launches": 0, "chunks": 0, "max_group": 1}
        stream = self.slots[0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in reqs:
            now = time.perf_counter() - t0
            if r["arrival"] * time_scale > now:
                time.sleep(r["arrival"] * time_scale - now)
            chs = self._chunks(r)
            r["_left"] = len(chs)
            r["chunks"] = chs
            for ch in chs:
                with torch.cuda.stream(stream):
                    self._alloc(ch)
                    ch["pc"].sample(r["seed"], ch["offset"], ch["shots"], ch["det"], ch["obs"], stream)
                stream.synchronize()
                stats["launches"] += 1
                stats["chunks"] += 1
                self._finish(ch, time.perf_counter() - t0, stats)
        stats["makespan_s"] = time.perf_counter() - t0
        return self._summary(reqs, stats)

    # Requests below this many shot-gates count as small in the latency split.
    SMALL_WORK = 1e10

    def _summary(self, reqs, stats):
        """Throughput and latency of one served stream.  Rates are equivalent
        shot-gates per second (gate targets x shots of the requests over the
        makespan): circuits served by sparse detection sampling produce the
        same events without walking the gates.  Latencies are also split
        between small requests (under SMALL_WORK shot-gates) and the rest."""
        work = {id(r): self.pool[r["circuit"]].c.num_gate_targets * r["shots"] for r in reqs}
        sg = sum(work.values())
        lat = [r["completion"] - r["arrival"] for r in reqs if "completion" in r]
        small = [r["completion"] - r["arrival"] for r in reqs if "completion" in r and work[id(r)] < self.SMALL_WORK]
        large = [r["completion"] - r["arrival"] for r in reqs if "completion" in r and work[id(r)] >= self.SMALL_WORK]
        frame_sg = sum(work[id(r)] for r in reqs if self.pool[r["circuit"]].method == "frame")

        def ms(values, q):       # None (JSON null) when there is no such request
            v = percentile(values, q)
            return None if v is None else 1e3 * v

        return {"requests": len(reqs), "shot_gates": sg, "makespan_s": stats["makespan_s"],
                "equivalent_shot_gates_per_s": sg / stats["makespan_s"],
                "frame_path_shot_gates": frame_sg,
                "requests_per_s": len(reqs) / stats["makespan_s"],
                "p50_latency_ms": ms(lat, 50), "p99_latency_ms": ms(lat, 99),
                "mean_latency_ms": 1e3 * sum(lat) / max(len(lat), 1),
                "small_requests": len(small), "small_p50_latency_ms": ms(small, 50),
                "small_p99_latency_ms": ms(small, 99),
                "large_p50_latency_ms": ms(large, 50),
                "large_p99_latency_ms": ms(large, 99),
                "deferrals": stats["deferrals"],
                "launches": stats["launches"], "chunks": stats["chunks"], "max_group": stats["max_group"]}
