"""Benchmark: batched Pauli-frame sampling of a distance-49 surface-code memory
experiment (49 rounds, p = 1e-3, 65,536 shots) on one MI355X.

One step = one pass of the whole sampling path over one batch of shots:
frame initialisation, Clifford propagation, Pauli noise, resets, measurements
(flip record written to HBM) and detection events + observable flips
(stim_detector_sample).  Inputs (the compiled program and reference sample)
are resident on the GPU before the timed region; compile and reference
("analysis") time is reported separately.

Prints one JSON line.  Fields beyond the driver's contract:
  roofline      -- for the step's frame kernel (k_frame, HIP events on its
                   stream): compulsory bytes (the flip record it writes)
                   against HBM peak, measured HBM traffic when the counters
                   match the sources
  cpu_baseline  -- the oracle (-O3 -march=native) timed on this host on a
                   bounded shot sample, at all usable CPUs and at one
  walk_events   -- the same step with the events formed inside the frame
                   walk (STIM_WALK_EVENTS=1) instead of the flip record
  configs       -- d=3 x 1,024, d=15 x 2^20 and d=49 x 262,144 shots:
                   detector- and measurement-mode call times
  analysis_s    -- host compile + reference-sample time
  meas_mode     -- measurement-record sampling (stim_frame_sample) rate
  host_copy     -- copying one step's events to pinned host memory, and the
                   PCIe-inclusive rate (outputs otherwise stay in HBM)
  formats       -- shot-major output formats (01, b8, hits, r8) of the run's
                   detection events and record: time and bytes per second
  feedback      -- the same workload with ancillas reset by classically
                   controlled X (M + CX rec[-k] a) instead of R
  sparse        -- sparse detection-event sampling (identical events) at
                   p = 1e-3 and 1e-4 beside the frame path
  reference     -- canonical reference sample at d = 49 and 101: host
                   inverse tableau vs the GPU tableau
  batch         -- the 64-circuit mix in one persistent graph-captured launch
                   vs the same requests one at a time
  serving       -- Poisson request streams over the resident d = 3..101 pool,
                   and over a pool of small codes (d = 3..15) at 3,000 and
                   10,000 requests/s: throughput and p50/p99 latency,
                   continuous batching vs a one-at-a-time server
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D, ROUNDS, P, SHOTS, SEED = 49, 49, 1e-3, 65536, 0
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of k_frame at this workload, from rocprofv3 --pmc
# FETCH_SIZE and --pmc WRITE_SIZE runs (KiB per dispatch), scaled by what the
# same counters read for a plain 2 GiB device copy (python bench.py
# --copy-probe): FETCH_SIZE reports half the bytes read, WRITE_SIZE all bytes
# written.  The counters hold for the library sources whose digest is
# PMC_SOURCES (those the detector step is built from); once any of them
# changes, `traffic` is reported as null.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
PMC_KIB = {"k_frame": (360467.1, 1005908.3)}    # FETCH_SIZE KiB, WRITE_SIZE KiB per dispatch
# SQ counters of the same kernel and workload (per dispatch): what bounds it.
PMC_SQ = {"SQ_INSTS_VALU": 8.619e8, "SQ_BUSY_CU_CYCLES": 1.529e9, "SQ_LDS_IDX_ACTIVE": 3.960e8,
          "SQ_LDS_BANK_CONFLICT": 1.825e8, "SQ_WAIT_ANY": 2.765e9, "SQ_WAVE_CYCLES": 6.115e9}
PMC_SOURCES = "69a43ed4c65997c2"                  # sources_digest() when the counters were taken
PMC_PROFILE = "profiles/k_frame_surface_d49_65536shots.md"
CUS, CLOCK_HZ = 256, 2.4e9


# Sources the counted kernels (the detector step's walk and event kernels)
# do not depend on: output formats, sparse sampling, the GPU reference.
DIGEST_EXCLUDED = ("format_kernels", "sparse_kernels", "reference_gpu")


def sources_digest() -> str:
    """Digest of the library sources the detector step is built from
    (kernels, compiler, C ABI)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2103_02202_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.split(".")[0] in DIGEST_EXCLUDED:
            continue
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def streaming_bytes(d: int, rounds: int, p: float, shots: int) -> float:
    """Bytes the paper's per-op method would move on the rotated surface code
    (each operation reads and writes its frame rows in memory, Sec. 5.1):
    bits per shot for R 2, H 4, CX 6, M 4 (x read, record write, z read and
    write), dense noise on the 64-shot words an error touches (DEPOLARIZE1 4,
    DEPOLARIZE2 8, X_ERROR 2).  Here the frame stays on chip, so this is an
    upper bound on useful traffic, not what the kernel moves."""
    A, data, cx = d * d - 1, d * d, d * (d - 1)
    hit = 1 - (1 - p) ** 64
    per_round = A * 2 + 2 * (A // 2) * 4 + 4 * cx * 6 + A * 4
    per_round += (2 * (A // 2) * 4 + 4 * cx * 8 + A * 2) * hit
    bits = data * 2 + rounds * per_round + data * 2 * hit + data * 2
    return bits * shots / 8


def host_cpu():
    """CPU model, logical CPUs, CPUs this process may run on and the cgroup
    CPU quota (None if unlimited)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, period = f.read().split()
            if q != "max":
                quota = max(1, int(int(q) / int(period)))
    except (OSError, ValueError):
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "cgroup_cpus": quota}


def cpu_baseline(text: str, num_gate_targets: int, budget_s: float = 10.0):
    """The oracle as it stands (g++ -O3 -march=native build of the same
    source, OpenMP over 64-shot words), timed on this host over a bounded
    sample of the same workload: the first shots of the run, doubling until
    about budget_s / 2 per measurement; at one thread and at every CPU this
    process may use.  Its single-threaded reference-sample time is reported
    beside it."""
    import tempfile
    import oracle
    cpu = host_cpu()
    cores = cpu["affinity"]
    if cpu["cgroup_cpus"]:
        cores = min(cores, cpu["cgroup_cpus"])
    oracle.use_native_build(os.path.join(tempfile.gettempdir(), f"liboracle_native_{os.getpid()}.so"))
    c = oracle.Circuit(text)
    t0 = time.perf_counter()
    ref = c.reference()
    ref_s = time.perf_counter() - t0

    def rate(threads):
        shots = 256
        while True:
            t0 = time.perf_counter()
            c.sample(SEED, 0, shots, ref=ref, meas=False, det=True, obs=True, threads=threads)
            dt = time.perf_counter() - t0
            if dt * 2 > budget_s / 2 or shots >= SHOTS:
                return shots, dt
            shots *= 2

    s1, t1 = rate(1)
    sn, tn = rate(cores)
    return {"value": num_gate_targets * sn / tn, "unit": "shot-gates/s", "cores": cores, "kind": "oracle",
            "sample": f"d={D} surface code, shots [0, {sn}) of the {SHOTS}-shot run, detector mode, "
                      f"{tn:.2f} s sampling on {cores} threads; reference sample {ref_s:.2f} s single-threaded",
            "one_core": {"value": num_gate_targets * s1 / t1, "shots": s1, "seconds": t1},
            "build": "g++ -std=c++17 -O3 -march=native -fopenmp", "host": cpu, "reference_s": ref_s}


def finite(x):
    """x with every non-finite float replaced by None: the result line is
    strict JSON (no NaN or Infinity)."""
    import math
    if isinstance(x, float):
        return x if math.isfinite(x) else None
    if isinstance(x, dict):
        return {k: finite(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [finite(v) for v in x]
    return x


def time_calls(fn, reps, stream):
    """Average milliseconds per call of fn() over `reps` calls, HIP events on
    the stream the calls enqueue on (after two warm-up calls)."""
    import torch
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_configs(stream):
    """The other single-circuit configurations: d=3 (3 rounds, 1,024 shots),
    d=15 (15 rounds, 2^20 shots) and d=49 at 262,144 shots (a 315 MB frame,
    larger than the last-level cache), p = 1e-3, seed 0: detector-mode and
    measurement-mode call times."""
    import torch
    from paper_2103_02202_amd import stim_gpu, workloads
    out = {}
    for d, rounds, shots, reps in ((3, 3, 1024, 200), (15, 15, 1 << 20, 5), (49, 49, 1 << 18, 3)):
        c = stim_gpu.Circuit(workloads.surface_code(d, rounds, P))
        c.reference()
        W = (shots + 63) // 64
        det = torch.empty((c.num_detectors, W), dtype=torch.int64, device="cuda")
        obs = torch.empty((max(c.num_observables, 1), W), dtype=torch.int64, device="cuda")
        det_ms = time_calls(lambda: stim_gpu.stim_detector_sample(c.handle, SEED, 0, shots, det, obs, stream),
                            reps, stream)
        del det, obs
        meas = torch.empty((c.num_measurements, W), dtype=torch.int64, device="cuda")
        meas_ms = time_calls(lambda: stim_gpu.stim_frame_sample(c.handle, SEED, 0, shots, meas, stream), reps,
                             stream)
        del meas
        torch.cuda.empty_cache()
        G = c.num_gate_targets
        out[f"d={d}"] = {"workload": f"rotated surface-code Z memory d={d}, {rounds} rounds, p={P}, {shots} shots",
                         "gate_targets": G, "shots": shots, "detector_ms": det_ms,
                         "detector_shot_gates_per_s": G * shots / (det_ms * 1e-3), "measurement_ms": meas_ms,
                         "measurement_shot_gates_per_s": G * shots / (meas_ms * 1e-3),
                         "record_bytes": c.num_measurements * W * 8,
                         "record_hbm_frac": c.num_measurements * W * 8 / (meas_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def bench_host_copy(det, obs, stream, ms_per_step, G):
    """The step's outputs stay in HBM (`value` has no PCIe part).  For a
    caller that wants them on the host: the time to copy one step's detection
    events and observables into pinned host memory, and the PCIe-inclusive
    rate of step + copy (not overlapped)."""
    import torch
    h_det = torch.empty(det.shape, dtype=det.dtype, pin_memory=True)
    h_obs = torch.empty(obs.shape, dtype=obs.dtype, pin_memory=True)
    for _ in range(2):
        h_det.copy_(det, non_blocking=True)
        h_obs.copy_(obs, non_blocking=True)
    torch.cuda.synchronize()
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        h_det.copy_(det, non_blocking=True)
        h_obs.copy_(obs, non_blocking=True)
    e1.record(stream)
    e1.synchronize()
    copy_ms = e0.elapsed_time(e1) / reps
    nbytes = det.numel() * 8 + obs.numel() * 8
    return {"bytes": nbytes, "d2h_ms": copy_ms, "d2h_GBps": nbytes / (copy_ms * 1e-3) / 1e9,
            "pcie_inclusive_shot_gates_per_s": G * SHOTS / ((ms_per_step + copy_ms) * 1e-3)}


def bench_batch(steps: int):
    import torch
    from paper_2103_02202_amd import serve, stim_gpu, workloads
    mix = workloads.batch_mix(seed=0)
    t0 = time.perf_counter()
    pool = serve.load_pool([m["text"] for m in mix], threads=16)
    analysis = time.perf_counter() - t0
    reqs = []
    sg_total = 0
    for m, pc in zip(mix, pool):
        c = pc.c
        W = (m["shots"] + 63) // 64
        if m["kind"] == "surface":
            out0 = torch.empty((c.num_detectors, W), dtype=torch.int64, device="cuda")
            out1 = torch.empty((max(c.num_observables, 1), W), dtype=torch.int64, device="cuda")
            mode = 1
        else:
            out0 = torch.empty((c.num_measurements, W), dtype=torch.int64, device="cuda")
            out1, mode = None, 0
        reqs.append({"handle": c.handle, "seed": m["seed"], "shot_offset": 0, "num_shots": m["shots"],
                     "mode": mode, "out0": out0, "out1": out1})
        sg_total += c.num_gate_targets * m["shots"]
    stream = torch.cuda.current_stream()
    for _ in range(3):      # one-shot launch, then tuned + captured plan, then a replay
        stim_gpu.stim_batch_sample(reqs, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        stim_gpu.stim_batch_sample(reqs, stream=stream)
    e1.record(stream)
    e1.synchronize()
    batched_ms = e0.elapsed_time(e1) / steps
    # One circuit at a time on the same GPU, each call waited for.
    def one_by_one():
        for r, pc in zip(reqs, pool):
            if r["mode"] == 1:
                stim_gpu.stim_detector_sample(r["handle"], r["seed"], 0, r["num_shots"], r["out0"], r["out1"], stream)
            else:
                stim_gpu.stim_frame_sample(r["handle"], r["seed"], 0, r["num_shots"], r["out0"], stream)
            stream.synchronize()
    one_by_one()
    t0 = time.perf_counter()
    one_by_one()
    single_ms = (time.perf_counter() - t0) * 1e3
    return {"circuits": len(reqs), "shot_gates": sg_total, "batched_ms": batched_ms,
            "batched_shot_gates_per_s": sg_total / (batched_ms * 1e-3), "one_at_a_time_ms": single_ms,
            "one_at_a_time_shot_gates_per_s": sg_total / (single_ms * 1e-3),
            "speedup_vs_one_at_a_time": single_ms / batched_ms, "analysis_s": analysis}


def bench_formats(det, meas, rows_det, rows_meas, shots, reps: int = 3):
    """Shot-major output formats of the d=49 run's detection events and
    measurement record: time per call (HIP events on the stream) and
    algorithmic bytes (table in + formatted bytes out) per second."""
    import torch
    from paper_2103_02202_amd import stim_gpu
    stream = torch.cuda.current_stream()
    out = {}
    for name, table, rows, fmts in (("detection_events", det, rows_det, ("b8", "r8", "hits", "01")),
                                    ("measurement_record", meas, rows_meas, ("b8",))):
        for fmt in fmts:
            n = stim_gpu.stim_format_shots(table, rows, shots, fmt, None, stream)
            buf = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
            stim_gpu.stim_format_shots(table, rows, shots, fmt, buf, stream)        # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                stim_gpu.stim_format_shots(table, rows, shots, fmt, buf, stream)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            moved = rows * ((shots + 63) // 64) * 8 + n
            out[f"{name}/{fmt}"] = {"ms": ms, "out_bytes": n, "GB_per_s": moved / (ms * 1e-3) / 1e9,
                                    "hbm_frac": moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
            del buf
    return out


def bench_feedback(steps: int, det, obs, stream):
    """The same d=49 workload with ancillas reset by classically controlled X
    (measurement + CX rec[-k] a) instead of R: detector-mode step time."""
    import torch
    from paper_2103_02202_amd import stim_gpu, workloads
    circ = stim_gpu.Circuit(workloads.surface_code(D, ROUNDS, P, feedback_reset=True))
    for _ in range(2):
        stim_gpu.stim_detector_sample(circ.handle, SEED, 0, SHOTS, det, obs, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stim_gpu.stim_detector_sample(circ.handle, SEED, 0, SHOTS, det, obs, stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return {"workload": f"d={D}, {ROUNDS} rounds, p={P}, {SHOTS} shots, feedback resets",
            "ms_per_step": dt * 1e3, "gate_targets": circ.num_gate_targets,
            "shot_gates_per_s": circ.num_gate_targets * SHOTS / dt}


def bench_sparse(steps: int, det, obs, stream):
    """Sparse detection-event sampling (identical events) on the d=49 workload
    at p = 1e-3 and 1e-4, beside the frame path at the same p."""
    import torch
    from paper_2103_02202_amd import stim_gpu, workloads
    out = {}
    for p in (P, P / 10):
        circ = stim_gpu.Circuit(workloads.surface_code(D, ROUNDS, p))
        t0 = time.perf_counter()
        circ.error_sets()
        sets_s = time.perf_counter() - t0
        entry = {"error_sets_s": sets_s}
        for name, fn in (("sparse", stim_gpu.stim_sparse_detector_sample), ("frame", stim_gpu.stim_detector_sample)):
            for _ in range(2):
                fn(circ.handle, SEED, 0, SHOTS, det, obs, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn(circ.handle, SEED, 0, SHOTS, det, obs, stream)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            entry[name + "_ms"] = dt * 1e3
            # Sparse sampling draws the same errors without walking the gates:
            # its rate is an equivalent one (gate targets x shots / time).
            key = "sparse_equivalent_shot_gates_per_s" if name == "sparse" else "frame_shot_gates_per_s"
            entry[key] = circ.num_gate_targets * SHOTS / dt
        entry["sparse_speedup"] = entry["frame_ms"] / entry["sparse_ms"]
        out[f"p={p:g}"] = entry
    return out


def bench_reference():
    """Canonical reference sample (Sec. 4) of the d=49 and d=101 surface codes:
    host inverse tableau (one core) vs the GPU tableau; both must agree."""
    import torch
    from paper_2103_02202_amd import stim_gpu, workloads
    out = {}
    for d in (D, 101):
        text = workloads.surface_code(d, d, P)
        g = stim_gpu.Circuit(text)
        g.reference_gpu()                       # warm-up (allocations, code load)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gpu_bits = g.reference_gpu()
        gpu_s = time.perf_counter() - t0
        h = stim_gpu.Circuit(text)
        t0 = time.perf_counter()
        host_bits = h.reference()
        host_s = time.perf_counter() - t0
        out[f"d={d}"] = {"qubits": g.num_qubits, "measurements": g.num_measurements, "host_s": host_s,
                         "gpu_s": gpu_s, "speedup": host_s / gpu_s, "identical": gpu_bits == host_bits}
    return out


def bench_serving(rates=(10, 30, 100, 300, 1000)):
    import torch
    from paper_2103_02202_amd import serve, workloads
    pool_spec = workloads.serving_pool(seed=0)
    t0 = time.perf_counter()
    pool = serve.load_pool([x["text"] for x in pool_spec], names=[f"d{x['d']}" for x in pool_spec], threads=16)
    analysis = time.perf_counter() - t0
    os.environ["STIM_TUNE"] = "0"         # launches of unseen request sets are never tuned
    # Outputs come from torch's caching allocator and the flip scratch from the
    # library's stream-ordered pool; each can grow to the budget, so the budget
    # is kept below half of the 288 GB of HBM.
    srv = serve.Server(pool, hbm_budget_bytes=96 << 30, num_slots=4, max_chunk_shots=1 << 18,
                       max_chunk_bytes=8 << 30)
    t0 = time.perf_counter()
    methods = srv.calibrate()              # frame or sparse sampling per large circuit
    calibrate_s = time.perf_counter() - t0
    srv.serve(workloads.serving_requests(8, rate=1000.0, pool_size=len(pool), seed=999, max_shots=4096))  # warm-up
    out = {"pool": f"rotated surface codes d=3..101 (odd), rounds=d, p log-uniform [1e-4, 1e-2]",
           "analysis_s": analysis, "calibrate_s": calibrate_s,
           "methods": {k: {"frame_ms": v[0], "sparse_ms": v[1], "method": v[2]} for k, v in methods.items()},
           "rates": {}}
    keys = ("p50_latency_ms", "p99_latency_ms", "small_p50_latency_ms", "small_p99_latency_ms",
            "equivalent_shot_gates_per_s", "requests_per_s", "deferrals")
    for rate in rates:
        n = 50 if rate <= 10 else 100
        reqs = workloads.serving_requests(n, rate=float(rate), pool_size=len(pool), seed=rate)
        torch.cuda.empty_cache()
        st = srv.serve(reqs)
        entry = {"continuous": st}
        if rate in (10, 30, 100, 300):
            entry["one_at_a_time"] = srv.serve_one_at_a_time(
                workloads.serving_requests(n, rate=float(rate), pool_size=len(pool), seed=rate))
        out["rates"][str(rate)] = entry
        print(json.dumps({"serving_rate": rate, "continuous": {k: st[k] for k in keys},
                          "one_at_a_time": {k: entry["one_at_a_time"][k] for k in keys}
                          if "one_at_a_time" in entry else None}), file=sys.stderr, flush=True)
    # Admission under a small HBM budget: requests wait for memory (deferrals).
    small = serve.Server(pool, hbm_budget_bytes=8 << 30, num_slots=4, max_chunk_shots=1 << 18,
                         max_chunk_bytes=2 << 30)
    torch.cuda.empty_cache()
    st = small.serve(workloads.serving_requests(60, rate=100.0, pool_size=len(pool), seed=100))
    out["budget_8GiB_rate_100"] = st
    print(json.dumps({"serving_budget_8GiB": {k: st[k] for k in keys}}), file=sys.stderr, flush=True)
    # Many small requests: a pool of small surface codes (d = 3..15) at high
    # rates, where one launch per request is bound by launch and wait
    # overheads and continuous batching groups the arrivals.
    spec = workloads.serving_pool(seed=1, d_max=15)
    small_pool = serve.load_pool([x["text"] for x in spec], names=[f"d{x['d']}" for x in spec], threads=16)
    small_srv = serve.Server(small_pool, hbm_budget_bytes=96 << 30, num_slots=4, max_chunk_shots=1 << 18,
                             max_chunk_bytes=8 << 30)
    small_srv.serve(workloads.serving_requests(16, rate=1000.0, pool_size=len(small_pool), seed=999,
                                               max_shots=4096))                    # warm-up
    out["small_pool"] = {"pool": "rotated surface codes d=3..15 (odd), rounds=d, p log-uniform [1e-4, 1e-2]",
                         "requests": 400, "rates": {}}
    for rate, max_shots in ((3000, 1 << 16), (10000, 1 << 12), (10000, 1 << 16)):
        def reqs():
            return workloads.serving_requests(400, rate=float(rate), pool_size=len(small_pool), seed=rate,
                                              max_shots=max_shots)
        a = small_srv.serve(reqs())
        b = small_srv.serve_one_at_a_time(reqs())
        out["small_pool"]["rates"][f"{rate}/shots<={max_shots}"] = {"continuous": a, "one_at_a_time": b}
        print(json.dumps({"serving_small_pool": rate, "max_shots": max_shots,
                          "continuous": {k: a[k] for k in keys}, "one_at_a_time": {k: b[k] for k in keys}}),
              file=sys.stderr, flush=True)
    del os.environ["STIM_TUNE"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-formats", action="store_true")
    ap.add_argument("--no-feedback", action="store_true")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--sparse-probe", type=float, default=None, metavar="P",
                    help="only run sparse detection sampling of the d=49 workload at noise P, 5 times "
                         "(for profiling)")
    ap.add_argument("--reference-probe", type=int, default=None, metavar="D",
                    help="only compute the GPU reference sample of the distance-D surface code twice "
                         "(for profiling)")
    ap.add_argument("--frame-probe", action="store_true",
                    help="only run the d=49 step (detection events) 3 times (for profiling k_noise_gen and "
                         "k_frame)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 2 GiB device-to-device three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the shot axis shards across GPUs "
              "without communication, so N-GPU throughput is N independent copies of this run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_02202_amd import stim_gpu, workloads

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 8, "copies": 3}), flush=True)
        return

    if args.frame_probe:
        circ = stim_gpu.Circuit(workloads.surface_code(D, ROUNDS, P))
        W = (SHOTS + 63) // 64
        det = torch.empty((circ.num_detectors, W), dtype=torch.int64, device="cuda")
        obs = torch.empty((max(circ.num_observables, 1), W), dtype=torch.int64, device="cuda")
        for _ in range(3):
            stim_gpu.stim_detector_sample(circ.handle, SEED, 0, SHOTS, det, obs)
        torch.cuda.synchronize()
        print(json.dumps({"frame_probe": f"d={D}", "calls": 3}), flush=True)
        return

    if args.reference_probe is not None:
        circ = stim_gpu.Circuit(workloads.surface_code(args.reference_probe, args.reference_probe, P))
        for _ in range(2):
            circ.reference_gpu()
        print(json.dumps({"reference_probe_d": args.reference_probe, "calls": 2}), flush=True)
        return

    if args.sparse_probe is not None:
        circ = stim_gpu.Circuit(workloads.surface_code(D, ROUNDS, args.sparse_probe))
        circ.error_sets()
        W = (SHOTS + 63) // 64
        det = torch.empty((circ.num_detectors, W), dtype=torch.int64, device="cuda")
        obs = torch.empty((max(circ.num_observables, 1), W), dtype=torch.int64, device="cuda")
        for _ in range(5):
            stim_gpu.stim_sparse_detector_sample(circ.handle, SEED, 0, SHOTS, det, obs)
        torch.cuda.synchronize()
        print(json.dumps({"sparse_probe_p": args.sparse_probe, "calls": 5}), flush=True)
        return

    text = workloads.surface_code(D, ROUNDS, P)
    t0 = time.perf_counter()
    circ = stim_gpu.Circuit(text)
    compile_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    circ.reference()
    ref_s = time.perf_counter() - t0
    G = circ.num_gate_targets
    M, Dn, L = circ.num_measurements, circ.num_detectors, circ.num_observables
    W = (SHOTS + 63) // 64
    dev = torch.device("cuda:0")
    det = torch.empty((Dn, W), dtype=torch.int64, device=dev)
    obs = torch.empty((max(L, 1), W), dtype=torch.int64, device=dev)
    meas = torch.empty((M, W), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        stim_gpu.stim_detector_sample(circ.handle, SEED, 0, SHOTS, det, obs, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = G * SHOTS / (dt / args.steps)

    # The step's kernels: the noise pre-pass and the frame kernel, which
    # writes the flip record the event kernel then reads (HIP events recorded
    # by the library on the stream the kernels run on).
    reps = max(5, args.steps)
    stim_gpu.stim_kernel_timing(True)
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    det_gen_ms, det_frame_ms, det_passes = stim_gpu.stim_kernel_times()
    stim_gpu.stim_kernel_timing(False)
    det_gen_ms, det_frame_ms = det_gen_ms / det_passes, det_frame_ms / det_passes

    # One sampling pass in measurement mode = the noise pre-pass kernel plus
    # the frame kernel.  The pass is timed with HIP events on the stream it
    # runs on; the library's own events split it per kernel.
    for _ in range(2):
        stim_gpu.stim_frame_sample(circ.handle, SEED, 0, SHOTS, meas, stream)
    torch.cuda.synchronize()
    stim_gpu.stim_kernel_timing(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        stim_gpu.stim_frame_sample(circ.handle, SEED, 0, SHOTS, meas, stream)
    ev1.record(stream)
    ev1.synchronize()
    gen_ms, kframe_ms, passes = stim_gpu.stim_kernel_times()
    stim_gpu.stim_kernel_timing(False)
    pass_ms = ev0.elapsed_time(ev1) / reps
    gen_ms, kframe_ms = gen_ms / passes, kframe_ms / passes
    # Dominant kernel: k_frame of the step.  Its algorithmic bytes are the
    # compulsory ones, the flip record it writes (M S / 8 bytes: one bit per
    # measurement and shot; the frame stays on chip).
    event_bytes = (Dn + L) * SHOTS / 8
    record_bytes = M * SHOTS / 8
    per_op_bytes = streaming_bytes(D, ROUNDS, P, SHOTS)
    achieved = record_bytes / (det_frame_ms * 1e-3) / 1e9
    digest = sources_digest()
    fresh = PMC_KIB is not None and PMC_SOURCES == digest
    traffic = None
    if fresh:
        f, w = PMC_KIB["k_frame"]
        traffic = 1024 * (f * FETCH_SCALE + w * WRITE_SCALE)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_frame (the step's walk: flip record for the event kernel)",
                "launch_ms": det_frame_ms, "algorithmic_bytes": record_bytes,
                "algorithmic_bytes_basis": "compulsory: the flip record, M*S/8 bytes (frame kept in LDS)",
                "measured_hbm_frac": (traffic / (det_frame_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
                "traffic_over_algorithmic": (traffic / record_bytes) if traffic else None,
                "per_op_streaming_bytes": per_op_bytes,
                "traffic_over_per_op_streaming": (traffic / per_op_bytes) if traffic else None,
                "k_noise_gen_ms": det_gen_ms,
                "counters": PMC_PROFILE if fresh else f"none for library sources {digest}"}
    if fresh:
        # The resource that binds the kernel, from its counters against this
        # run's launch time: VALU issue (one wave64 instruction per CU and
        # cycle), the LDS pipe's active cycles (and the share of them lost to
        # bank conflicts), and the waves' waiting time.  None is saturated:
        # the walk is bound by issue and barrier latency.
        cu_cycles = CUS * CLOCK_HZ * det_frame_ms * 1e-3
        roofline["binding_resource"] = {
            "name": "VALU issue and barrier latency (no unit saturated)",
            "valu_issue_frac": PMC_SQ["SQ_INSTS_VALU"] / cu_cycles,
            "lds_active_frac": PMC_SQ["SQ_LDS_IDX_ACTIVE"] / cu_cycles,
            "lds_bank_conflict_share": PMC_SQ["SQ_LDS_BANK_CONFLICT"] / PMC_SQ["SQ_LDS_IDX_ACTIVE"],
            "wave_wait_frac": PMC_SQ["SQ_WAIT_ANY"] / PMC_SQ["SQ_WAVE_CYCLES"],
            "hbm_measured_frac": roofline["measured_hbm_frac"]}

    out = {
        "metric": "shot-gates/s + HBM GB/s frac of peak; batched/served vs single; p99 latency",
        "value": value,
        "unit": "shot-gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"rotated surface-code Z memory d={D}, {ROUNDS} rounds, p={P}, {SHOTS} shots, "
                               "detection events + observables", "d": D, "rounds": ROUNDS, "p": P,
                   "shots": SHOTS, "seed": SEED, "num_qubits": circ.num_qubits, "gate_targets": G,
                   "measurements": M, "detectors": Dn},
        "roofline": roofline,
        "meas_mode": {"ms": pass_ms, "shot_gates_per_s": G * SHOTS / (pass_ms * 1e-3),
                      "k_noise_gen_ms": gen_ms, "k_frame_ms": kframe_ms, "record_bytes": record_bytes,
                      "k_frame_record_GBs": record_bytes / (kframe_ms * 1e-3) / 1e9},
        "analysis_s": {"compile": compile_s, "reference": ref_s},
    }
    # The alternative detector path: events formed inside the walk from flip
    # rings (STIM_WALK_EVENTS=1), the same bits without the flip record.
    os.environ["STIM_WALK_EVENTS"] = "1"
    walk_ms = time_calls(step, max(3, args.steps // 2), stream)
    del os.environ["STIM_WALK_EVENTS"]
    out["walk_events"] = {"ms": walk_ms, "flip_record_ms": ms_per_step,
                          "event_bytes": event_bytes, "note": "STIM_WALK_EVENTS=1 path, not the default"}
    def leg(name, fn):
        # One progress line per leg on stderr; the result line stays on stdout.
        t = time.perf_counter()
        out[name] = fn()
        print(json.dumps({"bench_leg": name, "s": round(time.perf_counter() - t, 1)}), file=sys.stderr, flush=True)

    leg("host_copy", lambda: bench_host_copy(det, obs, stream, ms_per_step, G))
    if not args.no_formats:
        leg("formats", lambda: bench_formats(det, meas, Dn, M, SHOTS))
    if not args.no_feedback:
        leg("feedback", lambda: bench_feedback(max(3, args.steps // 2), det, obs, stream))
    if not args.no_sparse:
        leg("sparse", lambda: bench_sparse(max(3, args.steps // 2), det, obs, stream))
    if not args.no_configs:
        leg("configs", lambda: bench_configs(stream))
    if not args.no_reference:
        leg("reference", bench_reference)
    if not args.no_batch:
        leg("batch", lambda: bench_batch(max(3, args.steps // 2)))
    if not args.no_serving:
        leg("serving", bench_serving)
    if not args.no_cpu_baseline:
        leg("cpu_baseline", lambda: cpu_baseline(text, G))
    print(json.dumps(finite(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
