"""Pins of the oracle's lattice and syndrome (Section 2) against facts that hold
by construction: incidence from coordinates, stabilisers and logical operators
in the kernel of the check matrix, even cube parities, linearity."""
import itertools

import numpy as np
import pytest

import geom
from inputs import face, random_bits
from oracle.oracle import Oracle


@pytest.mark.parametrize("L", [3, 4, 5])
def test_counts_and_degrees(L):
    o = Oracle(L)
    fe, ef, es = o.incidence()
    assert o.n_edges == o.n_faces == 3 * L ** 3
    # every face has 4 distinct edges, every edge lies in exactly 4 faces
    assert all(len(set(r)) == 4 for r in fe.tolist())
    counts = np.bincount(fe.ravel(), minlength=o.n_edges)
    assert (counts == 4).all()
    # the reverse table points back at the same member slot
    for e in range(o.n_edges):
        for j in range(4):
            assert fe[ef[e, j], es[e, j]] == e


@pytest.mark.parametrize("L", [3, 4])
def test_face_members_match_coordinates(L):
    o = Oracle(L)
    fe, _, _ = o.incidence()
    ref = geom.face_members_by_points(L)
    for f in range(o.n_faces):
        assert set(fe[f].tolist()) == ref[f], f


@pytest.mark.parametrize("L", [3, 4, 6])
def test_member_order_convention(L):
    """Members k=0..3 of f(v,n) with axes a<b: e(v,a), e(v+b,a), e(v,b), e(v+a,b)."""
    o = Oracle(L)
    fe, _, _ = o.incidence()
    from inputs import edge
    for x, y, z, n in itertools.product(range(L), range(L), range(L), range(3)):
        a, b = [ax for ax in range(3) if ax != n]
        ua = [0, 0, 0]
        ua[a] = 1
        ub = [0, 0, 0]
        ub[b] = 1
        want = [edge(L, x, y, z, a), edge(L, x + ub[0], y + ub[1], z + ub[2], a),
                edge(L, x, y, z, b), edge(L, x + ua[0], y + ua[1], z + ua[2], b)]
        assert fe[face(L, x, y, z, n)].tolist() == want


@pytest.mark.parametrize("L", [3, 4, 5])
def test_stabilisers_and_membranes_have_no_syndrome(L):
    o = Oracle(L)
    for x, y, z in itertools.product(range(L), repeat=3):
        e = geom.bits_of(o.n_edges, geom.star(L, x, y, z))
        assert o.syndrome(e[None]).sum() == 0
    for a in range(3):
        for c in range(L):
            e = geom.bits_of(o.n_edges, geom.membrane(L, a, c))
            assert o.syndrome(e[None]).sum() == 0
            # a membrane meets every parallel logical Z string once
            for i, j in itertools.product(range(L), repeat=2):
                assert e[geom.string(L, a, i, j)].sum() == 1
            # and no string of another axis
            for d in range(3):
                if d != a:
                    assert e[geom.string(L, d, 0, 0)].sum() % 2 == 0


@pytest.mark.parametrize("L", [3, 4, 6])
def test_single_error_syndrome_is_its_four_faces(L):
    o = Oracle(L)
    ref = geom.face_members_by_points(L)
    rng = np.random.default_rng(L)
    for e_idx in rng.choice(o.n_edges, size=20, replace=False):
        e = np.zeros((1, o.n_edges), np.uint8)
        e[0, e_idx] = 1
        s = o.syndrome(e)[0]
        assert set(np.flatnonzero(s).tolist()) == {f for f, m in ref.items() if e_idx in m}


@pytest.mark.parametrize("L", [3, 5, 6])
def test_cube_parity_is_even_for_perfect_syndromes(L):
    """Every valid X syndrome is a union of closed loops: each cube has an even
    number of unsatisfied faces (the meta-checks of Section 4.1)."""
    o = Oracle(L)
    err = random_bits(7 + L, 4, o.n_edges, 0.1)
    syn = o.syndrome(err)
    for x, y, z in itertools.product(range(L), repeat=3):
        cf = geom.cube_faces(L, x, y, z)
        assert len(set(cf)) == 6
        assert (syn[:, cf].sum(axis=1) % 2 == 0).all()


def test_syndrome_is_linear():
    o = Oracle(4)
    a = random_bits(1, 3, o.n_edges, 0.2)
    b = random_bits(2, 3, o.n_edges, 0.2)
    assert np.array_equal(o.syndrome(a ^ b), o.syndrome(a) ^ o.syndrome(b))
    s = o.syndrome(a)
    o.syndrome(b, s, xor_into=True)
    assert np.array_equal(s, o.syndrome(a ^ b))
