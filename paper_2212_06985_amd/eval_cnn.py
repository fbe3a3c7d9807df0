"""Logical error rate and throughput of the CNN-prior decoder next to the
paper's p-BP, on the same shots (same seed, so the same noise).

    python -m paper_2212_06985_amd.eval_cnn --weights w.npy --L 12 --p 0.065 --cycles 40
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import paper_2212_06985_amd as tc  # noqa: E402
from paper_2212_06985_amd.train_cnn import packed_prior  # noqa: E402


def run(L, shots, p, cycles, params=None, seed=777, bp_iters=20, batch_shots=0, beta=1.0):
    """One experiment; params None: the paper's prior, else the network's
    prior blended at strength beta. Returns a dict."""
    import torch
    lat = tc.make_lattice(L)
    prm = tc.make_run_params(p, p, cycles, bp_iters, 6, 0b001001, n_shots=shots, seed=seed,
                             batch_shots=batch_shots)
    err = torch.zeros((lat.n_edges, tc.n_words(shots)), dtype=torch.int64, device="cuda")
    mask = torch.zeros(shots, dtype=torch.uint8, device="cuda")
    odd = torch.zeros((shots, 3), dtype=torch.int32, device="cuda")
    if params is None:
        ws = tc.alloc_workspace(tc.run_workspace_bytes(lat, prm))
        t = tc.run_cycles_timed(lat, prm, err, mask, odd, ws)
    else:
        packed = packed_prior(params, beta, p)
        ws = tc.alloc_workspace(tc.run_cnn_workspace_bytes(lat, prm))
        t = tc.run_cycles_cnn_timed(lat, prm, packed, err, mask, odd, ws)
    m = mask.cpu().numpy()
    fx = float((m & 1).mean())
    fa = float((m != 0).mean())
    # residual syndrome weight (stabiliser parts of the residual are invisible
    # to it, as they are to the logical readout)
    syn = torch.zeros_like(err)
    tc.syndrome(lat, err, syn, tc.n_words(shots))
    sw = int(np.unpackbits(syn.cpu().numpy().view(np.uint8)).sum())
    return {"L": L, "p": p, "cycles": cycles + 1, "shots": shots, "bp_iters": bp_iters,
            "ler_x": fx, "ler_x_sigma": math.sqrt(fx * (1 - fx) / shots),
            "ler_any": fa, "ler_any_sigma": math.sqrt(fa * (1 - fa) / shots),
            "mean_residual_syndrome": sw / (64 * tc.n_words(shots)),
            "qubit_cycles_per_s": 3 * L ** 3 * (cycles + 1) * shots / (t.total_ms / 1e3),
            "ms": t.total_ms}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--weights", required=True)
    ap.add_argument("--L", type=int, nargs="+", default=[12])
    ap.add_argument("--p", type=float, default=0.05)
    ap.add_argument("--cycles", type=int, default=0, help="noisy cycles (0: L)")
    ap.add_argument("--shots", type=int, default=32768)
    ap.add_argument("--betas", type=float, nargs="+", default=[1.0])
    ap.add_argument("--bp-iters", type=int, nargs="+", default=[20])
    ap.add_argument("--seed", type=int, default=777)
    args = ap.parse_args()
    w = np.load(args.weights, allow_pickle=False)
    for L in args.L:
        cycles = args.cycles or L
        base = run(L, args.shots, args.p, cycles, None, args.seed)
        base["decoder"] = "plain p-BP"
        print(json.dumps(base), flush=True)
        for it in args.bp_iters:
            for beta in args.betas:
                r = run(L, args.shots, args.p, cycles, w, args.seed, bp_iters=it, beta=beta)
                r["decoder"] = f"CNN prior beta={beta}"
                print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
