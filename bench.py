"""Benchmark: batched Pauli-frame sampling of a distance-49 surface-code memory
experiment (49 rounds, p = 1e-3, 65,536 shots) on one MI355X.

One step = one pass of the whole sampling path over one batch of shots:
frame initialisation, Clifford propagation, Pauli noise, resets, measurements
(flip record written to HBM) and detection events + observable flips
(stim_detector_sample).  Inputs (the compiled program and reference sample)
are resident on the GPU before the timed region; compile and reference
("analysis") time is reported separately.

Prints one JSON line.  Fields beyond the driver's contract:
  roofline      -- for the frame kernel, from HIP events on its stream
  cpu_baseline  -- the oracle timed on this host on a bounded shot sample
  analysis_s    -- host compile + reference-sample time
  meas_mode     -- measurement-record sampling (stim_frame_sample) rate
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


def cpu_baseline(text: str, num_gate_targets: int, budget_s: float = 12.0, threads: int | None = None):
    """The oracle as it stands, timed on the host cores over a bounded sample
    of the same workload (first shots of the run, doubling until ~budget)."""
    import oracle
    threads = threads or min(16, os.cpu_count() or 1)
    c = oracle.Circuit(text)
    t0 = time.perf_counter()
    ref = c.reference()
    ref_s = time.perf_counter() - t0
    shots = 256
    while True:
        t0 = time.perf_counter()
        c.sample(SEED, 0, shots, ref=ref, meas=False, det=True, obs=True, threads=threads)
        dt = time.perf_counter() - t0
        if dt * 2 > budget_s / 2 or shots >= SHOTS:
            break
        shots *= 2
    return {"value": num_gate_targets * shots / dt, "unit": "shot-gates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"d={D} surface code, shots [0, {shots}) of the {SHOTS}-shot run, detector mode, "
                      f"{dt:.2f} s sampling; reference sample {ref_s:.2f} s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the shot axis shards across GPUs "
              "without communication, so N-GPU throughput is N independent copies of this run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_02202_amd import stim_gpu, workloads

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

    # Frame kernel alone (measurement mode is exactly one launch of it), timed
    # with HIP events recorded on the stream the kernel runs on.
    for _ in range(2):
        stim_gpu.stim_frame_sample(circ.handle, SEED, 0, SHOTS, meas, stream)
    reps = max(5, args.steps)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        stim_gpu.stim_frame_sample(circ.handle, SEED, 0, SHOTS, meas, stream)
    ev1.record(stream)
    ev1.synchronize()
    frame_ms = ev0.elapsed_time(ev1) / reps
    record_bytes = M * SHOTS / 8
    achieved = record_bytes / (frame_ms * 1e-3) / 1e9

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
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_frame (measurement mode)", "kernel_ms": frame_ms,
                     "algorithmic_bytes": record_bytes},
        "meas_mode": {"ms": frame_ms, "shot_gates_per_s": G * SHOTS / (frame_ms * 1e-3)},
        "analysis_s": {"compile": compile_s, "reference": ref_s},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(text, G)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
