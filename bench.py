#!/usr/bin/env python3
"""Benchmark of the state-vector hot path on one MI355X.

Default workload (one "step"): a 28-qubit random brickwork circuit, 20 layers
(U3 on every qubit, then CNOTs on alternating neighbour pairs; 830 gates), from
|0...0>, followed by 4096 shots; then the 28-qubit QFT (420 gates) applied to a
seeded random basis state, followed by 4096 shots. complex128 state, one kernel
per gate. `value` = gates per second over the timed steps (state resident in HBM
before timing starts; sampling included in the step).

The JSON line also carries:
  roofline     -- the dominant kernel's algorithmic bytes per launch divided by
                  its average launch time (HIP events around every launch on the
                  launch stream, during the timed steps), against 8 TB/s;
  cpu_baseline -- the plain complex128 CPU oracle timed on a bounded prefix of the
                  same brickwork circuit (single thread).

--gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
SEED = 20251205      # seed of the 28-qubit workload


def workload_28q(dtype):
    import workloads as W

    n = 28
    brick = W.brickwork(n, 20, seed=SEED)
    x = W.random_basis_state(n, SEED)
    qft = W.qft(n)
    return n, brick, x, qft


def gate_bytes(ops, n, s):
    """Algorithmic bytes of a per-gate run: read + write of every amplitude a
    gate changes (2 * s * 2^n * touched fraction)."""
    frac = {"u3": 1.0, "h": 1.0, "rx": 1.0, "ry": 1.0, "rz": 1.0, "x": 1.0, "y": 1.0, "sx": 1.0,
            "s": 0.5, "sdg": 0.5, "t": 0.5, "tdg": 0.5, "z": 0.5, "p": 0.5,
            "cx": 0.5, "cy": 0.5, "swap": 0.5, "cz": 0.25, "cp": 0.25, "rzz": 1.0, "ccx": 0.25}
    return sum(2.0 * s * (1 << n) * frac[o[0]] for o in ops)


def source_digest():
    h = hashlib.sha256()
    for f in ("k_gate.hip", "sv_device.h"):
        with open(os.path.join(ROOT, "paper_2512_04216_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, launches_bytes):
    """HBM traffic of `kernel` per launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_28q_brickwork_qft.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except OSError:
        return None
    if d.get("source_digest") != source_digest():
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k:
        return None
    return k.get("hbm_bytes_per_launch")


def cpu_baseline(budget_s=15.0):
    """The oracle as it stands, on a bounded prefix of the 28-qubit brickwork."""
    from oracle import oracle as O

    n, brick, _, _ = workload_28q("c128")
    psi = O.basis_state(n, 0)
    t0 = time.perf_counter()
    done = 0
    for op in brick:
        O.apply_op(psi, op)
        done += 1
        if time.perf_counter() - t0 > budget_s and done >= 2:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "gates/s", "cores": 1, "kind": "oracle",
            "sample": "first %d gates of the 28-qubit brickwork, complex128, from |0>, one thread "
                      "(%.1f s)" % (done, dt)}


def run_28q(S, ctx, dtype, steps, warmup, shots=4096, trace=True):
    import torch

    n, brick, x, qft = workload_28q(dtype)
    st = S.State(ctx, n, dtype)
    s = 8 if dtype == "c64" else 16
    ngates = len(brick) + len(qft)

    def step(i):
        st.reset(0)
        st.run(brick)
        st.sample(shots, SEED + 2 * i)
        st.reset(x)
        st.run(qft)
        st.sample(shots, SEED + 2 * i + 1)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    if trace:
        ctx.trace_read()
        ctx.trace(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(warmup + i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tr = {}
    if trace:
        ctx.trace(False)
        tr = ctx.trace_read()
    st.close()
    algo = (gate_bytes(brick, n, s) + gate_bytes(qft, n, s)) * steps
    return {"seconds": dt, "gates": ngates * steps, "algo_bytes": algo, "trace": tr}


def stream_copy_gbps(nbytes=4 << 30, reps=5):
    """Achievable HBM bandwidth of a plain device copy (torch), for context."""
    import torch

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c64", action="store_true", help="skip the complex64 side measurement")
    ap.add_argument("--no-trace", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no sharding or collectives); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2512_04216_amd as S

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    print("bench: 28-qubit brickwork + QFT, %s, %d warmup + %d timed steps" % (args.dtype, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    copy_gbps = stream_copy_gbps()
    print("bench: device copy %.0f GB/s" % copy_gbps, file=sys.stderr, flush=True)
    ctx = S.Context(arena_bytes=24 << 30)
    r = run_28q(S, ctx, args.dtype, args.steps, args.warmup, trace=not args.no_trace)
    print("bench: %s done in %.3f s" % (args.dtype, r["seconds"]), file=sys.stderr, flush=True)
    side = None
    if not args.no_c64 and args.dtype == "c128":
        r64 = run_28q(S, ctx, "c64", args.steps, args.warmup, trace=False)
        side = {"gates_per_s": r64["gates"] / r64["seconds"], "ms_per_step": 1e3 * r64["seconds"] / args.steps,
                "hbm_GBps": r64["algo_bytes"] / r64["seconds"] / 1e9}
        print("bench: c64 done in %.3f s" % r64["seconds"], file=sys.stderr, flush=True)
    ctx.close()

    roof = None
    if r["trace"]:
        dom = max(r["trace"].items(), key=lambda kv: kv[1]["seconds"])
        name, rec = dom
        per_launch_bytes = rec["bytes"] / rec["launches"]
        avg_s = rec["seconds"] / rec["launches"]
        ach = per_launch_bytes / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(name, per_launch_bytes),
                "launches": rec["launches"], "avg_launch_us": round(avg_s * 1e6, 2),
                "bytes_per_launch": per_launch_bytes,
                "share_of_kernel_time": round(rec["seconds"] / sum(v["seconds"] for v in r["trace"].values()), 4)}
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    value = r["gates"] / r["seconds"]
    out = {
        "metric": "gates/sec (28-qubit brickwork + QFT, per-gate kernels, 4096 shots each)",
        "value": round(value, 2), "unit": "gates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["seconds"] / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.dtype == "c128" else "f32", "data": "synthetic",
        "config": {"workload": "28-qubit random brickwork (20 layers, 830 gates) + 28-qubit QFT on a seeded "
                               "basis state (420 gates), %s state, 4096 shots each" % args.dtype,
                   "qubits": 28, "gates_per_step": r["gates"] // args.steps, "shots_per_step": 8192,
                   "fuse_k": 0, "parallelism": "none (1 GPU)"},
        "hbm_GBps": round(r["algo_bytes"] / r["seconds"] / 1e9, 1),
        "device_copy_GBps": round(copy_gbps, 1),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if side:
        out["c64"] = {k: round(v, 2) for k, v in side.items()}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
