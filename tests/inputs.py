"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module holds no arithmetic of the decoding method: it draws random bit
patterns and message arrays with numpy's seeded generators, converts between
the oracle's unpacked [shot][site] uint8 layout and the GPU's bit-sliced
[site][word] uint64 planes (bit i of word w is shot 64*w + i), and names
lattice sites by their coordinates.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------- naming
def site(L, x, y, z):
    return (x % L) + L * ((y % L) + L * (z % L))


def edge(L, x, y, z, a):
    """Index of the edge from (x,y,z) to (x,y,z)+unit(a)."""
    return a * L ** 3 + site(L, x, y, z)


def face(L, x, y, z, n):
    """Index of the unit square at corner (x,y,z) with normal axis n."""
    return n * L ** 3 + site(L, x, y, z)


# ------------------------------------------------------------ random data
def random_bits(seed: int, n_shots: int, n_sites: int, density: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.random((n_shots, n_sites)) < density).astype(np.uint8)


def random_messages(seed: int, n_shots: int, n_faces: int, scale: float = 3.0) -> np.ndarray:
    """Factor-to-variable message arrays [shot][face][4] in FP64."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=(n_shots, n_faces, 4))


def random_llr(seed: int, n_shots: int, n_edges: int, lo: float = -2.0, hi: float = 6.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n_shots, n_edges))


# ------------------------------------------------------------ bit layout
def n_words(n_shots: int) -> int:
    return (n_shots + 63) // 64


def pack(bits: np.ndarray) -> np.ndarray:
    """[S][sites] uint8 -> [sites][W] uint64 (padding shots are zero)."""
    S, n = bits.shape
    W = n_words(S)
    padded = np.zeros((n, W * 64), np.uint8)
    padded[:, :S] = bits.T
    # little bit order: shot 64w+i -> bit i of word w (little-endian words)
    by = np.packbits(padded, axis=1, bitorder="little")  # [n][W*8] bytes
    return np.ascontiguousarray(by).view(np.uint64).reshape(n, W)


def unpack(words: np.ndarray, n_shots: int) -> np.ndarray:
    """[sites][W] uint64 -> [S][sites] uint8."""
    n, W = words.shape
    by = np.ascontiguousarray(words).view(np.uint8).reshape(n, W * 8)
    b = np.unpackbits(by, axis=1, bitorder="little")  # [n][W*64]
    return np.ascontiguousarray(b[:, :n_shots].T)


def nu_to_gpu(nu: np.ndarray, L: int, s_pad: int) -> np.ndarray:
    """Oracle messages [S][face][4] -> GPU layout [word][site][normal*4+k][64]."""
    S = nu.shape[0]
    N = L ** 3
    full = np.zeros((s_pad, N, 12), np.float32)
    full[:S] = nu.reshape(S, 3, N, 4).transpose(0, 2, 1, 3).reshape(S, N, 12)
    W = s_pad // 64
    return np.ascontiguousarray(full.reshape(W, 64, N, 12).transpose(0, 2, 3, 1))


def nu_from_gpu(g: np.ndarray, L: int, n_shots: int) -> np.ndarray:
    """GPU layout [word][site][12][64] -> oracle [S][face][4] (FP64)."""
    N = L ** 3
    a = np.asarray(g, np.float64).reshape(-1, N, 12, 64)
    W = a.shape[0]
    per_shot = a.transpose(0, 3, 1, 2).reshape(W * 64, N, 12)[:n_shots]  # [S][site][12]
    return np.ascontiguousarray(
        per_shot.reshape(n_shots, N, 3, 4).transpose(0, 2, 1, 3).reshape(n_shots, 3 * N, 4))


def rows_to_gpu(x: np.ndarray) -> np.ndarray:
    """Per-shot rows [S_pad][rows] -> word-blocked [W][rows][64] (float32)."""
    S, R = x.shape
    return np.ascontiguousarray(x.reshape(S // 64, 64, R).transpose(0, 2, 1).astype(np.float32))


def rows_from_gpu(g: np.ndarray, n_rows: int) -> np.ndarray:
    """Word-blocked [W][rows][64] -> per-shot rows [S_pad][rows]."""
    a = np.asarray(g).reshape(-1, n_rows, 64)
    return np.ascontiguousarray(a.transpose(0, 2, 1).reshape(-1, n_rows))
