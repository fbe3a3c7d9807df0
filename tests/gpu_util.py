"""Helpers of the GPU parity tests: device transfer of bit planes, the
tolerance of BP messages, and running the oracle over shot chunks in threads
(ctypes releases the GIL inside the oracle's C calls)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import sys

import numpy as np

import inputs

# BP message tolerance: |gpu - oracle| <= REL * max(|oracle|, FLOOR), one step
# from the same (GPU) state, FP32 against FP64. Below FLOOR the bound becomes
# absolute because mu = l - nu cancels there.
BP_REL = 1e-4
BP_FLOOR = 0.1
# hard decisions may differ only where the oracle's posterior is this close to 0
LLR_TIE = 1e-3


def announce(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray):
    import torch
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def plane_from_dev(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def dev_plane_of_bits(bits: np.ndarray):
    return to_dev(inputs.pack(bits))


def bits_of_dev(t, n_shots) -> np.ndarray:
    return inputs.unpack(plane_from_dev(t), n_shots)


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def oracle_run_parallel(o, params, n_shots, shot0=0, chunk=None):
    """Oracle run_cycles over [shot0, shot0+n_shots) split into chunks."""
    chunk = chunk or max(1, (n_shots + workers() - 1) // workers())
    starts = list(range(0, n_shots, chunk))

    def job(s):
        k = min(chunk, n_shots - s)
        return o.run_cycles(params, k, shot0=shot0 + s)

    with cf.ThreadPoolExecutor(workers()) as ex:
        parts = list(ex.map(job, starts))
    mask = np.concatenate([p[0] for p in parts])
    odd = np.concatenate([p[1] for p in parts])
    err = np.concatenate([p[2] for p in parts])
    return mask, odd, err


def within_bp_tol(g: np.ndarray, o: np.ndarray):
    bound = BP_REL * np.maximum(np.abs(o), BP_FLOOR)
    dev = np.abs(g - o)
    return bool((dev <= bound).all()), float((dev / np.maximum(np.abs(o), 1e-30)).max()), \
        float(dev.max())
