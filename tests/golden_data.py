"""Readers of the paper's worked examples and printed tables under
tests/golden/ (plain text; each file states its source in the paper)."""
from __future__ import annotations

import os

from inputs import edge

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
AXES = {"x": 0, "y": 1, "z": 2}

# the flip examples sit around this site of an L = 6 lattice
EXAMPLE_L = 6
EXAMPLE_SITE = (2, 2, 2)


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if line:
                yield line


def edge_of_token(tok: str, L: int = EXAMPLE_L, at=EXAMPLE_SITE) -> int:
    """'a@dx,dy,dz' -> index of the edge along axis a from at + (dx,dy,dz)."""
    a, off = tok.split("@")
    d = [int(v) for v in off.split(",")]
    if a not in AXES or len(d) != 3:
        raise ValueError(f"bad edge token {tok!r}")
    return edge(L, at[0] + d[0], at[1] + d[1], at[2] + d[2], AXES[a])


def flip_examples():
    """name -> fields; edge-set fields become sets of edge indices,
    'unsat' an int, 'cleared' a bool, 'cite' a string."""
    out, cur = {}, None
    for line in _lines("flip_examples.txt"):
        if line.startswith("["):
            cur = out.setdefault(line.strip("[]"), {})
            continue
        key, _, rest = line.partition(" ")
        rest = rest.strip()
        if key == "cite":
            cur[key] = rest
        elif key == "unsat":
            cur[key] = int(rest)
        elif key == "cleared":
            cur[key] = rest == "yes"
        elif key in ("support", "flips", "ties", "after1", "after2"):
            cur[key] = set() if rest == "-" else {edge_of_token(t) for t in rest.split()}
        else:
            raise ValueError(f"unknown field {key!r}")
    return out


def table1():
    """[(n_A, lambda_p, threshold as a fraction, shaded)]"""
    rows = []
    for line in _lines("table1_thresholds.txt"):
        n_a, lam, th, shaded = line.split()
        rows.append((int(n_a), int(lam), float(th) / 100.0, shaded == "yes"))
    return rows


def table2():
    """configuration string 'xyz' -> occurrences out of 1000"""
    return {k: int(v) for k, v in (line.split() for line in _lines("table2_correlations.txt"))}
