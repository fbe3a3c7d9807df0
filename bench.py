#!/usr/bin/env python3
"""Throughput of shot-parallel p-BP decoding of the 3D toric code on one MI355X.

A step is one complete decoding experiment (tc3d_run_cycles) over a fresh
batch of shots: every noisy cycle plus the perfect-measurement cycle (noise,
syndrome, 20 FP32 BP iterations, the P F F P F F sweep schedule, carry-over)
and the majority-vote readout. Inputs are synthetic by construction: the
workload is the phenomenological noise the library draws from its Philox
counters, so nothing but the seed is loaded.

Prints one JSON line with the throughput in decoded qubit-cycles/s (one
qubit-cycle = one edge x one cycle x one shot), the roofline of the dominant
kernel, measured live with HIP events, and the oracle timed on the host.

    python bench.py [--workload c5|c2|c1] [--steps K] [--warmup W]
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# name -> workload. Shots per step x steps covers the configuration's shots.
WORKLOADS = {
    # L = 48 (331,776 qubits), p = q = 0.05, 48 noisy cycles + 1 perfect,
    # BP 20 iterations + P F F P F F, 2x10^4 shots (10 steps of 2048)
    "c5": dict(L=48, ps=[0.05], noisy=48, bp=20, sweeps=6, mask=0b001001,
               sched="PFFPFF", shots=2048, steps=10, warmup=1),
    # L = 12 (5,184 qubits), p = q in {0.04, 0.05, 0.055, 0.06}, 12 + 1 cycles,
    # BP 20 + P F F P F F, 10^5 shots per p (one step per p value)
    "c2": dict(L=12, ps=[0.04, 0.05, 0.055, 0.06], noisy=12, bp=20, sweeps=6, mask=0b001001,
               sched="PFFPFF", shots=100_032, steps=4, warmup=1),
    # L = 6 (648 qubits), p = q = 0.02, 6 + 1 cycles, flip + p-flip F F P F F,
    # no BP, 10^4 shots
    "c1": dict(L=6, ps=[0.02], noisy=6, bp=0, sweeps=5, mask=0b00100, sched="FFPFF",
               shots=10_048, steps=10, warmup=2),
}

# algorithmic HBM bytes per launch unit of each kernel class:
# (bytes, unit) with unit "edge-shot" (one qubit of one shot) or "edge-word"
# (one qubit row of a 64-shot word)
ALGO_BYTES = {
    "bp_iter": (32.0, "edge-shot"),   # read + write the 4 FP32 messages per qubit
    "bp_first": (16.0, "edge-shot"),  # write only: its inputs come from the syndrome
    "bp_post": (16.0, "edge-shot"),   # read the messages once
    "noise": (16.0, "edge-word"),     # read + write the error plane
    "syndrome": (16.0, "edge-word"),  # read one plane, write the check plane
    "sweep": (32.0, "edge-word"),     # read checks, read+write correction, write flips
    "apply": (24.0, "edge-word"),
    "readout": (8.0, "edge-word"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2212_06985_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(cfg, target_s: float):
    """The oracle, as it is, on a bounded sample of the same workload: a few
    shots for the first cycle(s), one shot per thread."""
    import concurrent.futures as cf

    from oracle.oracle import Oracle, make_params

    cores = min(os.cpu_count() or 1, 16)
    o = Oracle(cfg["L"])
    n = 3 * cfg["L"] ** 3
    p = cfg["ps"][0]

    def one(shot, cycles):
        prm = make_params(p, p, cycles, cfg["bp"], cfg["sweeps"], cfg["mask"], seed=1,
                          perfect_final=0)
        o.run_cycles(prm, 1, shot0=shot)

    # calibrate on one shot-cycle, then size the sample to ~target_s of wall
    t0 = time.perf_counter()
    one(0, 1)
    t1 = time.perf_counter() - t0
    cycles = max(1, min(cfg["noisy"], int(target_s / max(t1, 1e-6))))
    shots = cores
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        list(ex.map(lambda s: one(s, cycles), range(shots)))
    wall = time.perf_counter() - t0
    qc = n * cycles * shots
    return {
        "value": qc / wall,
        "unit": "qubit-cycles/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{shots} shots x first {cycles} noisy cycle(s) of the workload, one shot "
                  f"per thread, {wall:.1f} s wall",
    }


def copy_calibration(nbytes: int, reps: int):
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--shots", type=int, default=None, help="shots per step")
    ap.add_argument("--batch-shots", type=int, default=0)
    ap.add_argument("--bp-tile", type=int, default=0, help="BP traversal tile (0: auto)")
    ap.add_argument("--noisy-cycles", type=int, default=None,
                    help="override the workload's noisy cycles (short counter runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibrate", type=int, default=0,
                    help="only run a plain copy of this many bytes (counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(shots shard across GPUs with no exchange but a final 8-counter sum; "
              "see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibrate:
        copy_calibration(args.copy_calibrate, 5)
        return

    import paper_2212_06985_amd as tc

    if not os.path.exists(tc.LIB_PATH):
        from paper_2212_06985_amd import build as hip_build
        hip_build.build()

    cfg = dict(WORKLOADS[args.workload])
    if args.shots:
        cfg["shots"] = args.shots
    if args.noisy_cycles is not None:
        cfg["noisy"] = args.noisy_cycles
    steps = cfg["steps"] if args.steps is None else args.steps
    warmup = cfg["warmup"] if args.warmup is None else args.warmup
    L, S = cfg["L"], cfg["shots"]
    lat = tc.make_lattice(L)
    cycles = cfg["noisy"] + 1
    W = tc.n_words(S)

    # shots decoded together: the whole step unless a smaller batch is asked for
    batch = min(64 * W, args.batch_shots) if args.batch_shots else 64 * W

    def params(step):
        p = cfg["ps"][step % len(cfg["ps"])]
        return tc.make_run_params(p, p, cfg["noisy"], cfg["bp"], cfg["sweeps"], cfg["mask"],
                                  n_shots=S, seed=1, shot0=64 * W * step, batch_shots=batch,
                                  bp_tile=args.bp_tile)

    need = max(tc.run_workspace_bytes(lat, params(k)) for k in range(len(cfg["ps"])))
    ws = tc.alloc_workspace(need)
    err = torch.zeros((lat.n_edges, W), dtype=torch.int64, device="cuda")
    mask = torch.zeros(S, dtype=torch.uint8, device="cuda")
    odd = torch.zeros((S, 3), dtype=torch.int32, device="cuda")
    log(f"[bench] workload {args.workload}: L={L} shots/step={S} cycles={cycles} "
        f"batch={batch} workspace {need / 2**30:.2f} GiB; warmup {warmup}, steps {steps}")

    for k in range(warmup):
        err.zero_()
        tc.run_cycles(lat, params(k), err, mask, odd, ws)
        torch.cuda.synchronize()
        log(f"[bench] warmup step {k} done")

    per_class = {k: {"ms": 0.0, "launches": 0} for k in tc.KERNEL_CLASSES}
    fails_x = fails_any = 0
    hist = [0] * 8  # mask histogram: bit d = logical X error on qubit d
    ties = 0        # majority-vote ties (an axis with exactly L^2/2 odd strings)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        err.zero_()
        t = tc.run_cycles_timed(lat, params(k), err, mask, odd, ws)
        for name, v in t.as_dict().items():
            per_class[name]["ms"] += v["ms"]
            per_class[name]["launches"] += v["launches"]
        m = mask.cpu()
        fails_x += int((m & 1).ne(0).sum())
        fails_any += int(m.ne(0).sum())
        hb = torch.bincount(m.long(), minlength=8)
        hist = [h + int(v) for h, v in zip(hist, hb.tolist())]
        ties += int((2 * odd == L * L).any(dim=1).sum())
        log(f"[bench] step {k}: {t.total_ms:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    n = lat.n_edges
    qubit_cycles = n * cycles * S * steps
    value = qubit_cycles / wall

    # roofline of the dominant kernel class
    dom = max(per_class, key=lambda k: per_class[k]["ms"])
    d = per_class[dom]
    avg_ms = d["ms"] / max(d["launches"], 1)
    per_unit, unit = ALGO_BYTES[dom]
    # one launch covers one batch (the last batch of a step may be smaller;
    # with batch = the whole step every launch is a full batch)
    units = n * batch if unit == "edge-shot" else n * (batch // 64)
    algo_bytes = per_unit * units
    achieved = algo_bytes / (avg_ms * 1e-3) / 1e9
    traffic = stored_traffic(dom, args.workload)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": dom, "avg_launch_ms": round(avg_ms, 4),
            "launches": d["launches"], "algo_bytes_per_launch": algo_bytes,
            "algo_bytes_per_unit": per_unit, "unit_of_work": unit}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        cpu = cpu_baseline(cfg, args.cpu_seconds)

    N = S * steps
    ler = {"axis_x": fails_x / N, "axis_x_sigma": (fails_x / N * (1 - fails_x / N) / N) ** 0.5,
           "any_axis": fails_any / N, "shots": N,
           "mask_histogram": {format(k, "03b")[::-1]: hist[k] for k in range(8)},
           "majority_ties": ties}
    out = {
        "metric": "decoded qubit-cycles/s at fixed logical error rate; CNN-prior vs plain "
                  "BP+p-flip",
        "value": value,
        "unit": "qubit-cycles/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg["bp"] else "u64",
        "data": "synthetic (phenomenological noise drawn from Philox counters, seed 1)",
        "config": {"workload": f"L={L} p=q={'/'.join(str(p) for p in cfg['ps'])} "
                               f"{cfg['noisy']}+1 cycles "
                               f"{'BP' + str(cfg['bp']) + ' + ' if cfg['bp'] else ''}"
                               f"{cfg['sched']}",
                   "L": L, "shots_per_step": S, "batch_shots": batch, "shots_total": N, "cycles": cycles,
                   "bp_iters": cfg["bp"], "schedule": cfg["sched"], "decoder": "plain p-BP",
                   "parallelism": "shots (bit-sliced 64 per word; one lane per shot in BP)"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "ler": ler,
        "kernel_ms": {k: round(v["ms"], 3) for k, v in per_class.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
