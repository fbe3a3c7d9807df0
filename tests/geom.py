"""Independent coordinate geometry of the periodic cubic lattice (test helper).

Built only from points: an edge is the unordered pair of its two endpoints, a
face is the set of its four corners, and an edge lies on a face's boundary
exactly when both endpoints are corners of the face and they differ in one
coordinate. Used to pin the oracle's index tables, never by the oracle.
"""
from __future__ import annotations

import itertools

from inputs import edge as edge_index
from inputs import face as face_index

UNIT = ((1, 0, 0), (0, 1, 0), (0, 0, 1))


def add(L, p, d, k=1):
    return tuple((p[i] + k * d[i]) % L for i in range(3))


def edge_points(L, x, y, z, a):
    p = (x % L, y % L, z % L)
    return frozenset({p, add(L, p, UNIT[a])})


def face_corners(L, x, y, z, n):
    a, b = [ax for ax in range(3) if ax != n]
    p = (x % L, y % L, z % L)
    return frozenset({p, add(L, p, UNIT[a]), add(L, p, UNIT[b]),
                      add(L, add(L, p, UNIT[a]), UNIT[b])})


def all_edges(L):
    for z, y, x, a in itertools.product(range(L), range(L), range(L), range(3)):
        yield (x, y, z, a), edge_index(L, x, y, z, a), edge_points(L, x, y, z, a)


def face_members_by_points(L):
    """face index -> set of member edge indices, from corner sets alone."""
    by_pts = {}
    for _, idx, pts in all_edges(L):
        by_pts.setdefault(pts, []).append(idx)
    out = {}
    for z, y, x, n in itertools.product(range(L), range(L), range(L), range(3)):
        corners = face_corners(L, x, y, z, n)
        members = set()
        for c1, c2 in itertools.combinations(sorted(corners), 2):
            diff = sum(1 for i in range(3) if c1[i] != c2[i])
            if diff == 1:
                members.update(by_pts[frozenset({c1, c2})])
        out[face_index(L, x, y, z, n)] = members
    return out


def star(L, x, y, z):
    """The six edges meeting at a vertex: the support of an X stabiliser."""
    out = []
    for a in range(3):
        out.append(edge_index(L, x, y, z, a))
        d = [0, 0, 0]
        d[a] = -1
        out.append(edge_index(L, x + d[0], y + d[1], z + d[2], a))
    return out


def membrane(L, a, c):
    """All a-edges whose a-coordinate equals c: a logical X operator."""
    out = []
    for i, j in itertools.product(range(L), range(L)):
        p = [0, 0, 0]
        p[a] = c
        p[(a + 1) % 3] = i
        p[(a + 2) % 3] = j
        out.append(edge_index(L, p[0], p[1], p[2], a))
    return out


def string(L, d, i, j):
    """The L d-edges through fixed other coordinates: a logical Z operator."""
    out = []
    for t in range(L):
        p = [0, 0, 0]
        p[d] = t
        p[(d + 1) % 3] = i
        p[(d + 2) % 3] = j
        out.append(edge_index(L, p[0], p[1], p[2], d))
    return out


def cube_faces(L, x, y, z):
    """The six faces of the unit cube with lower corner (x,y,z)."""
    out = []
    for n in range(3):
        d = [0, 0, 0]
        d[n] = 1
        out.append(face_index(L, x, y, z, n))
        out.append(face_index(L, x + d[0], y + d[1], z + d[2], n))
    return out


def bits_of(n, idx):
    import numpy as np
    v = np.zeros(n, np.uint8)
    for i in idx:
        v[i] ^= 1
    return v
