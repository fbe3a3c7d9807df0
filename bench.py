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
kernel, measured live with HIP events (HBM-bound for the streaming BP
iteration; ALU-bound where a lattice of at most 3072 sites decodes each shot
inside one workgroup's LDS), the whole path against the HBM peak, and the
oracle timed on the host.

    python bench.py [--workload c5|c4|c3|c2|c1] [--decoder plain|cnn] [--steps K] [--warmup W]

With --decoder cnn the BP prior comes from the committed CNN (blended with
the channel prior); with --compare the other decoder also decodes the same
shots and its throughput and logical error rate are reported beside it.
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
    # BP 20 iterations + P F F P F F, 2x10^4 shots (10 steps of 2048), with and
    # without the CNN prior: the comparison decodes the shots of the first
    # compare_steps steps again with the CNN prior at its matched-throughput
    # point (6 BP iterations, prior blended at 0.5)
    "c5": dict(L=48, ps=[0.05], noisy=48, bp=20, cnn_bp=6, beta=0.5, sweeps=6, mask=0b001001,
               sched="PFFPFF", shots=2048, steps=10, warmup=1, compare=True, compare_steps=5),
    # L = 12 (5,184 qubits), p = q in {0.04, 0.05, 0.055, 0.06}, 12 + 1 cycles,
    # BP 20 + P F F P F F, 10^5 shots per p (one step per p value)
    "c2": dict(L=12, ps=[0.04, 0.05, 0.055, 0.06], noisy=12, bp=20, sweeps=6, mask=0b001001,
               sched="PFFPFF", shots=100_032, steps=4, warmup=1),
    # batched mixed jobs: L in {8, 12, 16, 20, 24} x p = q in {0.045 .. 0.065},
    # L noisy cycles + 1 perfect each, BP 20 + P F F P F F, all 25 jobs in one
    # captured graph per step (2x10^4 shots per job per step; --shots changes it)
    "c3": dict(Ls=[8, 12, 16, 20, 24], ps=[0.045, 0.05, 0.055, 0.06, 0.065], bp=20, sweeps=6,
               mask=0b001001, sched="PFFPFF", shots=20_032, steps=2, warmup=1, L=24, noisy=24),
    # CNN prior vs plain: L = 24 (41,472 qubits), p = q = 0.05, 24 + 1 cycles,
    # P F F P F F, 10^5 shots (5 steps of 20,032), both decoders on the same shots.
    # Plain p-BP runs its 20 BP iterations; the CNN decoder runs at its
    # matched-throughput point, 6 iterations with the prior blended at 0.5
    "c4": dict(L=24, ps=[0.05], noisy=24, bp=20, cnn_bp=6, beta=0.5, sweeps=6, mask=0b001001,
               sched="PFFPFF", shots=20_032, steps=5, warmup=1, decoder="cnn", compare=True),
    # L = 6 (648 qubits), p = q = 0.02, 6 + 1 cycles, flip + p-flip F F P F F,
    # no BP, 10^4 shots
    "c1": dict(L=6, ps=[0.02], noisy=6, bp=0, sweeps=5, mask=0b00100, sched="FFPFF",
               shots=10_048, steps=10, warmup=2, graph=True),
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

# The CNN prior's forward pass: 4 periodic 3x3x3 convolutions 8 -> 32 -> 32 -> 32
# -> 3 channels, 27 (8*32 + 32*32 + 32*32 + 32*3) multiply-adds per site of a shot.
# A forward runs as passes over a few shot groups, 5 launches each (input
# assembly + 4 layers); the class average launch carries the forward's FLOP
# divided by its launches.
CNN_FLOP_PER_SITE = 2 * 27 * (8 * 32 + 32 * 32 + 32 * 32 + 32 * 3)
# BP with each shot's state in LDS (lattices of at most 3072 sites, scalar
# prior) is bound by the vector ALU. Its FP32 work per site and iteration, in
# VALU issue cycles of one lane: per check 4 clamps (one min-max-median op
# each), 8 (a -+ 1), 10 products forming N and D, and for each of the 4
# outputs D +- N (two fused multiply-adds), a reciprocal and a product; a
# reciprocal holds the VALU for two issue cycles (rocprofv3's
# SQ_ACTIVE_INST_VALU), every other op for one: 42 cycles per check; per site
# 3 checks plus 30 products forming the incoming e^mu. The posterior adds 12
# products per site.
RESIDENT_MAX_SITES = 3072
RESIDENT_SLOTS_PER_SITE_ITER = 3 * (4 + 8 + 10 + 4 * (2 + 2 + 1)) + 30
RESIDENT_SLOTS_PER_SITE_POST = 12
# one non-packed FP32 operation per lane per clock: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz (the 157.3 TFLOP/s vector peak counts packed FMAs, 4 FLOP
# per lane per clock, which the library does not use)
VALU_SLOTS_PEAK_T = 256 * 64 * 2.4e9 / 1e12
MFMA_BF16_PEAK_TFLOPS = 2500.0
DEFAULT_WEIGHTS = os.path.join(ROOT, "paper_2212_06985_amd", "weights", "cnn_L12_long.npy")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# source files each kernel class is built from (its counters stay valid while
# these are unchanged)
KERNEL_SOURCES = {
    "bp_iter": ["tc3d_bp.hip", "tc3d_device.hpp", "tc3d_internal.hpp"],
    "bp_iter_prior": ["tc3d_bp.hip", "tc3d_device.hpp", "tc3d_internal.hpp"],
    "bp_resident": ["tc3d_bp.hip", "tc3d_device.hpp", "tc3d_internal.hpp"],
    "cnn": ["tc3d_cnn.hip", "tc3d_device.hpp", "tc3d_internal.hpp"],
}


def kernel_source_hash(kernel: str = "bp_iter") -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2212_06985_amd", "csrc")
    for name in sorted(KERNEL_SOURCES.get(kernel, os.listdir(csrc))):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def stored_ceiling(kernel: str, workload: str):
    """The measured streaming ceiling (GB/s, the library's plain copy) kept
    beside the kernel's counters, or None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("stream_ceiling_GBps:"):
                try:
                    return float(line.split(":", 1)[1])
                except ValueError:
                    return None
    return None


def profile_key(workload: str, L=None, shots=None, batch_shots=0) -> str:
    """The name the stored counter summaries of a run are looked up under: they
    describe the workload's own launches, so with a lattice, shot count or
    batch of its own no summary applies."""
    base = WORKLOADS[workload]
    if (L and L != base["L"]) or (shots and shots != base["shots"]) or batch_shots:
        return workload + "_custom"
    return workload


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
    if vals.get("source_sha256") != kernel_source_hash(kernel):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """The host's CPU model, core count and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return model, os.cpu_count() or 1, allowed


# worker threads of the oracle: the host cores this process may use, at most
# 16 (a one-GPU share of the GPU hosts)
CPU_SHARE = 16


def cpu_baseline(cfg, target_s: float, tc=None):
    """The oracle, as it is, on a bounded sample of the same workload: a few
    shots for the first cycle(s), one shot per thread. With the library given,
    the GPU decodes the same sample and the shots that came out differently
    are counted (FP32 against FP64 BP near a tie)."""
    import concurrent.futures as cf

    import numpy as np

    from oracle.oracle import Oracle, make_params

    model, nproc, allowed = host_cpu()
    cores = min(allowed, CPU_SHARE)
    o = Oracle(cfg["L"])
    n = 3 * cfg["L"] ** 3
    p = cfg["ps"][0]

    def prm_of(cycles):
        return make_params(p, p, cycles, cfg["bp"], cfg["sweeps"], cfg["mask"], seed=1,
                           perfect_final=0)

    def one(shot, cycles):
        return o.run_cycles(prm_of(cycles), 1, shot0=shot)

    # calibrate on one shot-cycle, then size the sample to ~target_s of wall
    t0 = time.perf_counter()
    one(0, 1)
    t1 = time.perf_counter() - t0
    cycles = max(1, min(cfg["noisy"], int(target_s / max(t1, 1e-6))))
    shots = cores
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        res = list(ex.map(lambda s: one(s, cycles), range(shots)))
    wall = time.perf_counter() - t0
    qc = n * cycles * shots
    out = {
        "value": qc / wall,
        "unit": "qubit-cycles/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{shots} shots x first {cycles} noisy cycle(s) of the workload, one shot "
                  f"per thread, {wall:.1f} s wall",
        "host": {"cpu_model": model, "nproc": nproc, "cores_allowed": allowed,
                 "threads_used": cores},
    }
    if tc is not None:
        import torch
        lat = tc.make_lattice(cfg["L"])
        prm = tc.make_run_params(p, p, cycles, cfg["bp"], cfg["sweeps"], cfg["mask"],
                                 n_shots=shots, seed=1, perfect_final=0)
        err = torch.zeros((lat.n_edges, tc.n_words(shots)), dtype=torch.int64, device="cuda")
        mask = torch.zeros(shots, dtype=torch.uint8, device="cuda")
        ws = tc.alloc_workspace(tc.run_workspace_bytes(lat, prm))
        tc.run_cycles(lat, prm, err, mask, None, ws)
        torch.cuda.synchronize()
        w = err.cpu().numpy().view(np.uint64)
        g = np.unpackbits(w.view(np.uint8).reshape(w.shape[0], -1), axis=1,
                          bitorder="little")[:, :shots].T
        same = sum(int(np.array_equal(g[s], r[2][0])) for s, r in enumerate(res))
        out["parity_vs_gpu"] = {"shots": shots, "identical": same, "diverged": shots - same}
    return out


def copy_calibration(nbytes: int, reps: int):
    """The library's plain streaming copy of known size: scales rocprofv3 byte
    counters, and its rate (read + write, HIP events) is the practical
    streaming ceiling beside the 8 TB/s peak."""
    import torch

    import paper_2212_06985_amd as tc
    n = nbytes // 16 * 16
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {"copy_bytes_read": n, "copy_bytes_written": n, "reps": reps}
    for nt in (1, 0):
        tc.stream_copy(dst, src, nontemporal=bool(nt))  # warm-up
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            tc.stream_copy(dst, src, nontemporal=bool(nt))
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out["nontemporal" if nt else "temporal"] = {"ms": ms, "GB_per_s": 2 * n / ms / 1e6}
    assert torch.equal(dst, src)
    print(json.dumps(out))


def cnn_packed(p: float, beta: float, weights: str):
    """Device copy of the committed network, blended with the channel prior at
    strength beta, in the library's packed BF16 layout."""
    import numpy as np
    import torch

    from paper_2212_06985_amd.train_cnn import packed_prior
    packed = packed_prior(np.load(weights, allow_pickle=False), beta, p)
    torch.cuda.synchronize()
    return packed


def run_decoder(tc, lat, cfg, decoder, steps, warmup, S, batch, bp_tile, beta, weights, tag,
                graph=False):
    """Warm up, then time `steps` complete experiments of one decoder. Returns
    the wall time of the timed steps, per-class kernel times and statistics.
    graph: every step is one HIP graph of all its launches (plain decoder);
    the per-class kernel times then come from one more step run eagerly."""
    import torch
    W = tc.n_words(S)
    L = cfg["L"]
    cnn = decoder == "cnn"

    def params(step):
        p = cfg["ps"][step % len(cfg["ps"])]
        return tc.make_run_params(p, p, cfg["noisy"], cfg["bp"], cfg["sweeps"], cfg["mask"],
                                  n_shots=S, seed=1, shot0=64 * W * step, batch_shots=batch,
                                  bp_tile=bp_tile, flags=tc.RUN_GRAPH if graph else 0,
                                  **RUN_KNOBS)

    nps = len(cfg["ps"])
    packs = [cnn_packed(p, beta, weights) for p in cfg["ps"]] if cnn else [None] * nps
    ws_of = tc.run_cnn_workspace_bytes if cnn else tc.run_workspace_bytes
    need = max(ws_of(lat, params(k)) for k in range(nps))
    ws = tc.alloc_workspace(need)
    err = torch.zeros((lat.n_edges, W), dtype=torch.int64, device="cuda")
    mask = torch.zeros(S, dtype=torch.uint8, device="cuda")
    odd = torch.zeros((S, 3), dtype=torch.int32, device="cuda")
    log(f"[bench] {tag} decoder {decoder}: L={L} shots/step={S} cycles={cfg['noisy'] + 1} "
        f"batch={batch} workspace {need / 2**30:.2f} GiB; warmup {warmup}, steps {steps}")

    def one(k, timed):
        err.zero_()
        pk = packs[k % nps]
        if cnn:
            f = tc.run_cycles_cnn_timed if timed else tc.run_cycles_cnn
            return f(lat, params(k), pk, err, mask, odd, ws)
        if graph and timed:  # the graph's launches, without per-class events
            tc.run_cycles(lat, params(k), err, mask, odd, ws)
            return None
        if graph:
            prm = params(k)
            prm.flags = 0
            return tc.run_cycles_timed(lat, prm, err, mask, odd, ws)
        f = tc.run_cycles_timed if timed else tc.run_cycles
        return f(lat, params(k), err, mask, odd, ws)

    for k in range(warmup):
        one(k, False)
        # the statistics' torch kernels load on first use: not inside the timed steps
        torch.bincount(mask.long(), minlength=8)
        (2 * odd == L * L).any(dim=1).sum()
        torch.cuda.synchronize()
        log(f"[bench] {tag} warmup step {k} done")

    per_class = {k: {"ms": 0.0, "launches": 0} for k in tc.KERNEL_CLASSES}
    decisions = near_ties = 0
    # statistics stay on the device during the timed steps (no copy, no sync)
    hist_d = torch.zeros(8, dtype=torch.int64, device="cuda")  # mask histogram
    ties_d = torch.zeros((), dtype=torch.int64, device="cuda")  # majority-vote ties
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        t0k = time.perf_counter()
        t = one(k, True)
        if t is not None:
            for name, v in t.as_dict().items():
                per_class[name]["ms"] += v["ms"]
                per_class[name]["launches"] += v["launches"]
            decisions += t.bp_decisions
            near_ties += t.bp_near_ties
        hist_d += torch.bincount(mask.long(), minlength=8)
        ties_d += (2 * odd == L * L).any(dim=1).sum()
        if k < 3 or k == steps - 1:
            log(f"[bench] {tag} step {k}: "
                f"{t.total_ms if t is not None else (time.perf_counter() - t0k) * 1e3:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hist = hist_d.tolist()  # bit d of the index: logical X error on qubit d
    ties = int(ties_d)
    fails_x = sum(hist[i] for i in range(8) if i & 1)
    fails_any = sum(hist[1:])
    if graph:  # kernel times of one eager step (the same work)
        t = one(0, False)
        for name, v in t.as_dict().items():
            per_class[name]["ms"] += v["ms"] * steps
            per_class[name]["launches"] += v["launches"] * steps
    N = S * steps
    ler = {"axis_x": fails_x / N, "axis_x_sigma": (fails_x / N * (1 - fails_x / N) / N) ** 0.5,
           "any_axis": fails_any / N,
           "any_axis_sigma": (fails_any / N * (1 - fails_any / N) / N) ** 0.5, "shots": N,
           "mask_histogram": {format(k, "03b")[::-1]: hist[k] for k in range(8)},
           "majority_ties": ties,
           # BP decisions whose posterior was within 1e-3 nats of 0, where FP32
           # and the FP64 oracle may decide apart
           "bp_near_ties": {"count": near_ties, "decisions": decisions,
                            "fraction": near_ties / decisions if decisions else None}}
    # residual syndrome weight of the last step's final state (what the
    # decoder left behind; stabiliser-equivalent residue is invisible to it)
    syn = torch.zeros_like(err)
    tc.syndrome(lat, err, syn, W)
    import numpy as np
    resid = int(np.unpackbits(syn.cpu().numpy().view(np.uint8)).sum()) / (64 * W)
    del ws
    return wall, per_class, ler, resid


def bp_message_bytes(bp_iters, per_edge_prior=False, fused=True):
    """HBM bytes of BP messages per qubit and decode (4 FP32 messages = 16 B
    per pass). Scalar prior: iteration 1 is implied by the syndrome, so
    iteration 2 only writes, iterations 3..T read and write and the posterior
    reads; fused, iteration T and the posterior are one pass that reads once.
    Per-edge prior: the first iteration writes, every later one reads and
    writes, the posterior reads, and every iteration reads the 4-byte prior;
    fused (T >= 2), iteration T and the posterior read the state and the
    prior once."""
    T = bp_iters
    if T <= 0:
        return 0.0
    if per_edge_prior:
        if fused and T >= 2:
            return 20.0 + 36.0 * (T - 2) + 20.0
        return 20.0 + 36.0 * (T - 1) + 16.0
    if T == 1:
        return 0.0
    split = 16.0 + 32.0 * (T - 2) + 16.0
    return split - 32.0 if fused else split


def path_roofline(bp_iters, value, per_edge_prior=False, n_sites=None, fused=True):
    """Whole-path HBM model: algorithmic bytes per decoded qubit-cycle times the
    qubit-cycles/s, against the HBM peak. Per qubit and cycle: BP's message
    passes (bp_message_bytes), one syndrome bit per iteration and about 32 bits
    of bit planes (noise, syndrome, correction, sweeps, apply). None without
    BP, where the path is bound by integer ALU work and launches, and where the
    decode runs resident in LDS (at most RESIDENT_MAX_SITES sites, scalar
    prior): its messages never reach HBM, and the BP roofline (ALU) is the one
    that applies."""
    if not bp_iters:
        return None
    if n_sites is not None and n_sites <= RESIDENT_MAX_SITES and not per_edge_prior:
        return None
    per_unit = bp_message_bytes(bp_iters, per_edge_prior, fused) + bp_iters / 8.0 + 4.0
    achieved = value * per_unit / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_unit": per_unit,
            "unit_of_work": "decoded qubit-cycle"}


def roofline(per_class, n, batch, n_sites, workload, forwards=0, shots_padded=0,
             per_edge_prior=False, bp_iters=0):
    """Roofline of the dominant kernel class, from the HIP-event launch times.
    For the CNN class, `forwards` forward passes over `shots_padded` shots
    (whole 64-shot words) were timed. With a per-edge prior, the BP iterations
    also read each edge's FP32 prior (4 more bytes per edge-shot); the
    posterior reads none, as a decode keeps the priors folded into its state."""
    dom = max(per_class, key=lambda k: per_class[k]["ms"])
    d = per_class[dom]
    avg_ms = d["ms"] / max(d["launches"], 1)
    if dom == "cnn":
        # MFMA-bound: algorithmic FLOP of all forwards, per launch on average
        flop = CNN_FLOP_PER_SITE * n_sites * shots_padded * forwards / max(d["launches"], 1)
        achieved = flop / (avg_ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": round(achieved, 1), "peak": MFMA_BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / MFMA_BF16_PEAK_TFLOPS, 4),
                "traffic": stored_traffic("cnn", workload),
                "kernel": "cnn (forward: input + 4 BF16 conv launches)",
                "avg_launch_ms": round(avg_ms, 4), "launches": d["launches"],
                "algo_flop_per_launch": flop, "algo_flop_per_unit": CNN_FLOP_PER_SITE,
                "unit_of_work": "site-shot forward (passes of 5 launches)"}
    shots = shots_padded if shots_padded else batch
    n_batches = -(-shots // batch)
    if (dom == "bp_iter" and not per_edge_prior and bp_iters >= 1
            and n_sites <= RESIDENT_MAX_SITES):
        # one launch decodes a batch with each shot's state in LDS: ALU-bound
        per_site = RESIDENT_SLOTS_PER_SITE_ITER * (bp_iters - 1) + RESIDENT_SLOTS_PER_SITE_POST
        ops = per_site * n_sites * shots / n_batches
        achieved = ops / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(VALU_SLOTS_PEAK_T, 2),
                "unit": "T VALU slots/s (FP32 lane-ops; a reciprocal takes 2 slots)",
                "frac": round(achieved / VALU_SLOTS_PEAK_T, 4),
                "traffic": stored_traffic("bp_resident", workload),
                "kernel": "bp_resident (whole decode of a shot in one workgroup's LDS)",
                "avg_launch_ms": round(avg_ms, 4), "launches": d["launches"],
                "algo_ops_per_launch": ops, "algo_ops_per_unit": per_site,
                "unit_of_work": "site-shot decode"}
    per_unit, unit = ALGO_BYTES[dom]
    # counters are kept per kernel variant: the per-edge-prior BP iteration's
    # under the name bp_iter_prior
    key = dom
    if per_edge_prior and dom in ("bp_iter", "bp_first"):
        per_unit += 4.0
        key = dom + "_prior"
    # a launch covers one batch of shots; with uneven batches (the last one of
    # a step may be smaller) the average launch carries shots / batches
    units = n * shots / n_batches if unit == "edge-shot" else n * (shots // 64) / n_batches
    algo_bytes = per_unit * units
    achieved = algo_bytes / (avg_ms * 1e-3) / 1e9
    ceiling = stored_ceiling(key, workload)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(key, workload), "kernel": dom,
            "stream_ceiling": ceiling,
            "frac_of_stream_ceiling": round(achieved / ceiling, 4) if ceiling else None,
            "avg_launch_ms": round(avg_ms, 4), "launches": d["launches"],
            "algo_bytes_per_launch": algo_bytes, "algo_bytes_per_unit": per_unit,
            "unit_of_work": unit}


def run_c3(args, cfg, tc):
    """The batched workload: every (L, p) job of a step in one tc3d_run_jobs
    call (concurrent job streams captured in one graph), after autotuning the
    traversal tile and batch size per L. The same jobs run sequentially (one
    stream, no graph) for comparison."""
    import torch
    S = cfg["shots"]
    W = tc.n_words(S)
    steps = cfg["steps"] if args.steps is None else args.steps
    warmup = cfg["warmup"] if args.warmup is None else args.warmup
    tuned = {}
    for L in cfg["Ls"]:
        lat = tc.make_lattice(L)
        prm = tc.make_run_params(0.055, 0.055, L, cfg["bp"], cfg["sweeps"], cfg["mask"],
                                 n_shots=S, seed=1, batch_shots=min(64 * W, 32768))
        ws = tc.alloc_workspace(tc.autotune_workspace_bytes(lat, prm))
        tried = tc.autotune(lat, prm, ws, probe_cycles=1)
        tuned[L] = dict(bp_tile=prm.bp_tile, batch_shots=prm.batch_shots, bp_path=prm.bp_path,
                        bp_occupancy=prm.bp_occupancy, candidates=len(tried))
        del ws
        log(f"[bench] c3 autotune L={L}: path {prm.bp_path} tile {prm.bp_tile} occupancy "
            f"{prm.bp_occupancy} batch {prm.batch_shots} ({len(tried)} candidates)")
    specs = [(L, p) for L in cfg["Ls"] for p in cfg["ps"]]
    bufs = []
    for L, p in specs:
        n = 3 * L ** 3
        bufs.append((torch.zeros((n, W), dtype=torch.int64, device="cuda"),
                     torch.zeros(S, dtype=torch.uint8, device="cuda"),
                     torch.zeros((S, 3), dtype=torch.int32, device="cuda")))

    def jobs_of(step):
        out = []
        for (L, p), (e, m, o) in zip(specs, bufs):
            prm = tc.make_run_params(p, p, L, cfg["bp"], cfg["sweeps"], cfg["mask"], n_shots=S,
                                     seed=1, shot0=64 * W * step,
                                     **{k: v for k, v in tuned[L].items() if k != "candidates"})
            out.append(tc.make_job(L, prm, e, m, o))
        return out

    ws = tc.alloc_workspace(tc.run_jobs_workspace_bytes(jobs_of(0)))
    qc = sum(3 * L ** 3 * (L + 1) * S for L, _ in specs)
    hist = {f"L={L} p={p}": [0] * 8 for L, p in specs}

    def timed(flags, tag, count):
        t_all = 0.0
        for k in range(warmup + steps):
            for e, _, _ in bufs:
                e.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tc.run_jobs(jobs_of(k), ws, flags)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if k >= warmup:
                t_all += dt
                if count:
                    for (L, p), (_, m, _) in zip(specs, bufs):
                        hb = torch.bincount(m.long(), minlength=8).tolist()
                        h = hist[f"L={L} p={p}"]
                        for i in range(8):
                            h[i] += hb[i]
            log(f"[bench] c3 {tag} step {k}: {dt * 1e3:.1f} ms")
        return t_all

    wall = timed(tc.JOBS_CONCURRENT | tc.JOBS_GRAPH, "graph", True)
    wall_seq = timed(0, "sequential", False)
    # roofline of the dominant kernel from one timed run of the largest job
    L = max(cfg["Ls"])
    lat = tc.make_lattice(L)
    prm = tc.make_run_params(0.055, 0.055, L, cfg["bp"], cfg["sweeps"], cfg["mask"], n_shots=S,
                             seed=1, **{k: v for k, v in tuned[L].items() if k != "candidates"})
    w1 = tc.alloc_workspace(tc.run_workspace_bytes(lat, prm))
    e, m, o = bufs[-1]
    e.zero_()
    t = tc.run_cycles_timed(lat, prm, e, m, o, w1)
    per_class = t.as_dict()
    batch = tuned[L]["batch_shots"] if tuned[L]["batch_shots"] else 64 * W
    roof = roofline(per_class, lat.n_edges, min(batch, 64 * W), lat.n_sites, "c3",
                    shots_padded=64 * W)
    roof["measured_on"] = f"L={L} job, p=0.055, {S} shots, timed separately"
    N = S * steps
    ler = {k: {"axis_x": sum(h[i] for i in range(8) if i & 1) / N,
               "any_axis": sum(h[1:]) / N} for k, h in hist.items()}
    return {
        "metric": "decoded qubit-cycles/s at fixed logical error rate; CNN-prior vs plain "
                  "BP+p-flip",
        "value": qc * steps / wall,
        "unit": "qubit-cycles/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (phenomenological noise drawn from Philox counters, seed 1)",
        "config": {"workload": f"batched: L in {cfg['Ls']} x p=q in {cfg['ps']}, L+1 cycles, "
                               f"BP{cfg['bp']} + {cfg['sched']}, one graph per step",
                   "jobs": len(specs), "shots_per_job_per_step": S, "shots_per_job": N,
                   "decoder": "plain p-BP",
                   "autotuned": {str(L): v
                                 for L, v in tuned.items()},
                   "parallelism": "jobs on 8 concurrent streams inside one HIP graph; shots "
                                  "bit-sliced 64 per word"},
        "roofline": roof,
        "cpu_baseline": None,
        # jobs of every size: those up to L = 14 decode resident in LDS, so no
        # single HBM model covers the mix
        "path_roofline": None,
        "comparison": {"decoder": "same jobs, one stream, no graph",
                       "value": qc * steps / wall_seq, "unit": "qubit-cycles/s",
                       "ms_per_step": wall_seq / steps * 1e3},
        "ler": ler,
    }


# kernel choices that never change a result (--bp-path, --bp-occupancy)
RUN_KNOBS = {}
BP_PATHS = {"auto": 0, "streaming": 1, "resident": 2, "split": 3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--L", type=int, default=None, help="override the workload's lattice size")
    ap.add_argument("--shots", type=int, default=None, help="shots per step")
    ap.add_argument("--batch-shots", type=int, default=0)
    ap.add_argument("--bp-tile", type=int, default=0, help="BP traversal tile (0: auto)")
    ap.add_argument("--bp-path", choices=sorted(BP_PATHS), default="auto",
                    help="BP kernels: resident where it fits (auto), streaming with the last "
                         "iteration fused into the posterior, resident, or split (the last "
                         "iteration and the posterior launched separately)")
    ap.add_argument("--bp-occupancy", type=int, default=0,
                    help="workgroups per CU of the streaming BP iterations (0: default)")
    ap.add_argument("--noisy-cycles", type=int, default=None,
                    help="override the workload's noisy cycles (short counter runs)")
    ap.add_argument("--decoder", choices=["plain", "cnn"], default=None,
                    help="plain p-BP or BP with the CNN prior (default: the workload's)")
    ap.add_argument("--compare", action=argparse.BooleanOptionalAction, default=None,
                    help="also decode the same shots with the other decoder")
    ap.add_argument("--bp-iters", type=int, default=None,
                    help="BP iterations of the main decoder (the comparison keeps the "
                         "workload's)")
    ap.add_argument("--beta", type=float, default=None,
                    help="CNN prior strength: llr0 = l0 + beta (llr_cnn - l0) "
                         "(default: the workload's, else 0.3)")
    ap.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--graph", action=argparse.BooleanOptionalAction, default=None,
                    help="run each step as one HIP graph (default: the workload's)")
    ap.add_argument("--copy-calibrate", type=int, default=0,
                    help="only run a plain copy of this many bytes (counter scaling)")
    args = ap.parse_args()
    RUN_KNOBS.update(bp_path=BP_PATHS[args.bp_path], bp_occupancy=args.bp_occupancy)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (shots "
              "would shard across GPUs with no exchange but a final sum of 8 mask "
              "counters). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibrate:
        copy_calibration(args.copy_calibrate, 5)
        return

    import paper_2212_06985_amd as tc

    from paper_2212_06985_amd import build as hip_build
    if tc.built_id() != hip_build.source_id():  # missing, or older than its sources
        log("[bench] building libtc3d.so")
        hip_build.build()

    cfg = dict(WORKLOADS[args.workload])
    if args.shots:
        cfg["shots"] = args.shots
    if args.workload == "c3":
        out = run_c3(args, cfg, tc)
        if not args.no_cpu_baseline:
            log("[bench] timing the oracle on the host")
            out["cpu_baseline"] = cpu_baseline(dict(cfg, L=12, ps=[0.055], noisy=12),
                                               args.cpu_seconds, tc)
        print(json.dumps(out), flush=True)
        return
    prof_key = profile_key(args.workload, args.L, args.shots, args.batch_shots)
    if args.L:
        cfg["L"] = args.L
        if args.noisy_cycles is None:
            cfg["noisy"] = args.L
    if args.noisy_cycles is not None:
        cfg["noisy"] = args.noisy_cycles
    decoder = args.decoder or cfg.get("decoder", "plain")
    compare = cfg.get("compare", False) if args.compare is None else args.compare
    steps = cfg["steps"] if args.steps is None else args.steps
    warmup = cfg["warmup"] if args.warmup is None else args.warmup
    L, S = cfg["L"], cfg["shots"]
    lat = tc.make_lattice(L)
    cycles = cfg["noisy"] + 1
    W = tc.n_words(S)
    n = lat.n_edges
    if decoder == "cnn" and not cfg["bp"]:
        sys.exit("the CNN prior feeds BP: pick a workload with BP iterations")

    # shots decoded together: the whole step unless a smaller batch is asked for
    batch = min(64 * W, args.batch_shots) if args.batch_shots else 64 * W

    beta = args.beta if args.beta is not None else cfg.get("beta", 0.3)

    def cfg_for(dec, main):
        """BP iterations of a decoder: the CNN decoder may run fewer than
        plain p-BP; --bp-iters sets the main decoder's."""
        bp = cfg.get("cnn_bp", cfg["bp"]) if dec == "cnn" else cfg["bp"]
        if main and args.bp_iters:
            bp = args.bp_iters
        return dict(cfg, bp=bp)

    main_cfg = cfg_for(decoder, True)
    graph = cfg.get("graph", False) if args.graph is None else args.graph
    graph = graph and decoder == "plain"
    wall, per_class, ler, resid = run_decoder(tc, lat, main_cfg, decoder, steps, warmup, S,
                                              batch, args.bp_tile, beta, args.weights,
                                              "main", graph=graph)
    qubit_cycles = n * cycles * S * steps
    value = qubit_cycles / wall
    roof = roofline(per_class, n, batch, lat.n_sites, prof_key, forwards=cycles * steps,
                    shots_padded=64 * W, per_edge_prior=decoder == "cnn",
                    bp_iters=main_cfg["bp"])
    # with the CNN prior, the conv launches' own (MFMA) roofline as well
    cnn_roof = None
    if decoder == "cnn" and per_class["cnn"]["launches"]:
        only = {k: (v if k == "cnn" else {"ms": 0.0, "launches": 0}) for k, v in per_class.items()}
        cnn_roof = roofline(only, n, batch, lat.n_sites, prof_key, forwards=cycles * steps,
                            shots_padded=64 * W)

    comparison = None
    if compare:
        other = "plain" if decoder == "cnn" else "cnn"
        other_cfg = cfg_for(other, False)
        c_steps = min(steps, cfg.get("compare_steps", steps))
        c_warm = min(warmup, 1)
        w2, pc2, ler2, resid2 = run_decoder(tc, lat, other_cfg, other, c_steps, c_warm, S, batch,
                                            args.bp_tile, beta, args.weights, "compare")
        dec2 = "plain p-BP" if other == "plain" else f"CNN prior (beta={beta}) + p-BP"
        comparison = {"decoder": dec2, "bp_iters": other_cfg["bp"], "steps": c_steps,
                      "shots": S * c_steps, "same_shots_as_main": "the first "
                      f"{S * c_steps} of the main run's {S * steps}",
                      "value": n * cycles * S * c_steps / w2, "unit": "qubit-cycles/s",
                      "ms_per_step": w2 / c_steps * 1e3, "ler": ler2,
                      "mean_residual_syndrome": resid2,
                      "roofline": roofline(pc2, n, batch, lat.n_sites, prof_key,
                                           forwards=cycles * c_steps, shots_padded=64 * W,
                                           per_edge_prior=other == "cnn",
                                           bp_iters=other_cfg["bp"]),
                      "kernel_ms": {k: round(v["ms"], 3) for k, v in pc2.items()}}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        cpu = cpu_baseline(cfg, args.cpu_seconds, tc)

    dec_name = "plain p-BP" if decoder == "plain" else f"CNN prior (beta={beta}) + p-BP"
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
        "dtype": ("bf16+f32" if decoder == "cnn" else "f32") if cfg["bp"] else "u64",
        "data": "synthetic (phenomenological noise drawn from Philox counters, seed 1)",
        "config": {"workload": f"L={L} p=q={'/'.join(str(p) for p in cfg['ps'])} "
                               f"{cfg['noisy']}+1 cycles "
                               f"{'BP' + str(main_cfg['bp']) + ' + ' if main_cfg['bp'] else ''}"
                               f"{cfg['sched']}"
                               f"{' with the CNN prior' if decoder == 'cnn' else ''}",
                   "L": L, "shots_per_step": S, "batch_shots": batch, "shots_total": S * steps,
                   "cycles": cycles, "bp_iters": main_cfg["bp"], "schedule": cfg["sched"],
                   "decoder": dec_name, "graph": graph, "bp_path": args.bp_path,
                   "parallelism": "shots (bit-sliced 64 per word; one lane per shot in BP)"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "path_roofline": path_roofline(main_cfg["bp"], value, per_edge_prior=decoder == "cnn",
                                       n_sites=lat.n_sites, fused=args.bp_path != "split"),
        "ler": ler,
        "mean_residual_syndrome": resid,
        "kernel_ms": {k: round(v["ms"], 3) for k, v in per_class.items()},
    }
    if cnn_roof is not None:
        out["cnn_roofline"] = cnn_roof
    if comparison is not None:
        out["comparison"] = comparison
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
