"""Pins of the oracle's belief propagation (Section 4.1, E1-E4 with
measurement-error variables) against closed forms and symmetries.

Closed forms used (derived from E1-E4, not retyped from the oracle):
  * tanh(l0/2) = 1 - 2p for l0 = ln((1-p)/p), and the measurement variable of
    degree 1 contributes tanh(ln((1-q)/q)/2) = 1 - 2q to every check product;
  * first iteration: every incoming message equals l0, so each check sends
    (-1)^s nu1 with nu1 = 2 atanh((1-2q)(1-2p)^3) and the posterior of bit i
    is l0 + (4 - 2 u_i) nu1, u_i = number of its unsatisfied checks;
  * zero syndrome: by translation symmetry every message is one scalar,
    nu_t = 2 atanh((1-2q) tanh((l0 + 3 nu_{t-1})/2)^3), nu_0 = 0, and every
    posterior is l0 + 4 nu_T (the "3" is the exclusion of the receiving
    check in E3, the "4" the full sum of E4).
"""
import itertools
import math

import numpy as np
import pytest

import geom
from inputs import edge, face, random_bits, random_llr, random_messages, site
from oracle.oracle import Oracle


def nu1(p, q):
    return 2 * math.atanh((1 - 2 * q) * (1 - 2 * p) ** 3)


@pytest.mark.parametrize("p,q", [(0.05, 0.05), (0.02, 0.04), (0.1, 0.01)])
def test_first_iteration_closed_form(p, q):
    o = Oracle(4)
    err = random_bits(3, 3, o.n_edges, 0.1)
    syn = o.syndrome(err)
    syn ^= random_bits(4, 3, o.n_faces, 0.05)
    _, ef, _ = o.incidence()
    l0 = math.log((1 - p) / p)
    for s in range(3):
        nu, post = o.bp_step(syn[s], p, q)
        u = syn[s][ef].sum(axis=1).astype(np.int64)
        np.testing.assert_allclose(post, l0 + (4 - 2 * u) * nu1(p, q), rtol=0, atol=1e-12)
        sign = np.where(syn[s] == 1, -1.0, 1.0)
        np.testing.assert_allclose(nu, np.repeat(sign[:, None] * nu1(p, q), 4, axis=1), rtol=0, atol=1e-12)


def test_measurement_factor_identity():
    for q in (0.001, 0.02, 0.05, 0.3):
        assert abs(math.tanh(0.5 * math.log((1 - q) / q)) - (1 - 2 * q)) < 1e-15


def scalar_recursion(p, q, T):
    l0 = math.log((1 - p) / p)
    nu = 0.0
    out = []
    for _ in range(T):
        nu = 2 * math.atanh((1 - 2 * q) * math.tanh((l0 + 3 * nu) / 2) ** 3)
        out.append(nu)
    return l0, out


@pytest.mark.parametrize("L", [3, 4])
def test_zero_syndrome_scalar_recursion(L):
    p = q = 0.05
    o = Oracle(L)
    syn = np.zeros(o.n_faces, np.uint8)
    l0, ref = scalar_recursion(p, q, 20)
    nu = None
    for t in range(20):
        nu, post = o.bp_step(syn, p, q, nu_in=nu)
        np.testing.assert_allclose(nu, ref[t], rtol=1e-13)
        np.testing.assert_allclose(post, l0 + 4 * ref[t], rtol=1e-13)
    # decode helper agrees with the chained steps
    _, post20 = o.bp_decode(syn[None], p, q, 20)
    np.testing.assert_allclose(post20[0], l0 + 4 * ref[-1], rtol=1e-13)
    # values at p = q = 0.05
    assert abs(ref[0] - 1.571869802157) < 1e-11
    assert abs(ref[1] - 2.918004664640) < 1e-11
    assert abs(ref[19] - 2.944002333351) < 1e-11
    assert abs(l0 + 4 * ref[19] - 14.720448312570) < 1e-10


@pytest.mark.parametrize("pq", [0.02, 0.04, 0.05, 0.055, 0.06])
def test_one_iteration_equals_flip_rule_below_crossover(pq):
    """With l0 < 2 nu1, BP(T=1) flips exactly the bits with >= 3 unsatisfied
    checks, i.e. the flip rule of Section 3.1."""
    l0 = math.log((1 - pq) / pq)
    assert l0 < 2 * nu1(pq, pq)
    o = Oracle(5)
    err = random_bits(11, 4, o.n_edges, 0.08)
    syn = o.syndrome(err) ^ random_bits(12, 4, o.n_faces, 0.05)
    corr, _ = o.bp_decode(syn, pq, pq, 1)
    _, ef, _ = o.incidence()
    for s in range(4):
        u = syn[s][ef].sum(axis=1).astype(np.int64)
        assert np.array_equal(corr[s], (u >= 3).astype(np.uint8))


def test_one_iteration_differs_from_flip_above_crossover():
    pq = 0.065
    assert math.log((1 - pq) / pq) > 2 * nu1(pq, pq)
    o = Oracle(4)
    e = geom.bits_of(o.n_edges, [edge(4, 1, 1, 1, 0), edge(4, 1, 1, 1, 1)])  # share one face
    syn = o.syndrome(e[None])
    _, ef, _ = o.incidence()
    u = syn[0][ef].sum(axis=1).astype(np.int64)
    assert (u == 3).any()
    corr, post = o.bp_decode(syn, pq, pq, 1)
    assert (post[0][u == 3] > 0).all()  # u = 3 bits are no longer flipped


def translate(L, arr, dx, dy, dz, per_site_axes=3):
    """Move per-(axis, site) data by a lattice translation."""
    N = L ** 3
    out = np.empty_like(arr)
    for a in range(per_site_axes):
        for z, y, x in itertools.product(range(L), repeat=3):
            out[..., a * N + site(L, x + dx, y + dy, z + dz)] = arr[..., a * N + site(L, x, y, z)]
    return out


def rotate(L, arr_edge_or_face):
    """Cyclic axis permutation (x,y,z) -> (y,z,x): the point (x,y,z) goes to
    (z,x,y) and axis a goes to a+1. Faces keep their corner and member set, so
    the same map applies to face normals."""
    N = L ** 3
    out = np.empty_like(arr_edge_or_face)
    for a in range(3):
        for z, y, x in itertools.product(range(L), repeat=3):
            out[..., ((a + 1) % 3) * N + site(L, z, x, y)] = \
                arr_edge_or_face[..., a * N + site(L, x, y, z)]
    return out


def test_bp_commutes_with_translations_and_axis_rotation():
    L = 4
    o = Oracle(L)
    err = random_bits(21, 1, o.n_edges, 0.1)
    syn = (o.syndrome(err) ^ random_bits(22, 1, o.n_faces, 0.04))[0]
    _, post = o.bp_decode(syn[None], 0.05, 0.05, 7)
    syn_t = translate(L, syn, 1, 2, 3)
    _, post_t = o.bp_decode(syn_t[None], 0.05, 0.05, 7)
    np.testing.assert_allclose(post_t[0], translate(L, post[0], 1, 2, 3), rtol=1e-12, atol=1e-12)
    syn_r = rotate(L, syn)
    _, post_r = o.bp_decode(syn_r[None], 0.05, 0.05, 7)
    np.testing.assert_allclose(post_r[0], rotate(L, post[0]), rtol=1e-12, atol=1e-12)


def test_step_from_messages_uses_other_checks_only():
    """E3 excludes the receiving check: a message change on check g reaches the
    outgoing messages of g itself only through its other members."""
    L = 3
    o = Oracle(L)
    syn = random_bits(5, 1, o.n_faces, 0.3)[0]
    nu = random_messages(6, 1, o.n_faces)[0]
    fe, ef, es = o.incidence()
    out0, _ = o.bp_step(syn, 0.05, 0.05, nu_in=nu)
    g = 17
    nu2 = nu.copy()
    nu2[g, :] += 5.0
    out1, _ = o.bp_step(syn, 0.05, 0.05, nu_in=nu2)
    np.testing.assert_array_equal(out0[g], out1[g])
    # but checks sharing a bit with g do change
    neigh = {f for i in fe[g] for f in ef[i]} - {g}
    for f in neigh:
        assert not np.allclose(out0[f], out1[f])


def test_per_edge_priors_match_scalar_prior():
    o = Oracle(3)
    syn = random_bits(8, 2, o.n_faces, 0.2)
    p = 0.07
    llr0 = np.full((2, o.n_edges), math.log((1 - p) / p))
    c1, p1 = o.bp_decode(syn, p, 0.05, 9, llr0=llr0)
    c2, p2 = o.bp_decode(syn, p, 0.05, 9)
    np.testing.assert_allclose(p1, p2, rtol=1e-14)
    llr = random_llr(9, 2, o.n_edges)
    _, p3 = o.bp_decode(syn, p, 0.05, 1, llr0=llr)
    assert not np.allclose(p3, p2)


def test_half_cube_posteriors_are_symmetric():
    """The corner half-star and its complement have the same syndrome, so BP
    cannot prefer either: all six star edges get one posterior and the
    correction takes all of them or none (Section 4.1)."""
    L = 6
    o = Oracle(L)
    st = geom.star(L, 2, 2, 2)
    e = geom.bits_of(o.n_edges, [st[0], st[2], st[4]])
    syn = o.syndrome(e[None])
    for T in (2, 3, 10, 20, 30):
        corr, post = o.bp_decode(syn, 0.05, 0.05, T)
        vals = post[0][st]
        assert np.ptp(vals) < 1e-9
        c = set(np.flatnonzero(corr[0]))
        assert c in (set(), set(st))
        # residual is equivalent to the original error (differs by a stabiliser)
        assert o.syndrome((e ^ corr[0])[None]).tolist() == syn.tolist()


def test_bp_corrects_planar_two_by_two():
    # Section 4.1: BP does not struggle with planar errors
    L = 6
    o = Oracle(L)
    idx = [edge(L, 2 + i, 2 + j, 2, 2) for i in (0, 1) for j in (0, 1)]
    e = geom.bits_of(o.n_edges, idx)
    corr, _ = o.bp_decode(o.syndrome(e[None]), 0.05, 0.05, 20)
    assert np.array_equal(corr[0], e)


@pytest.mark.slow
def test_L3_bp_returns_weight_one_and_two_errors():
    o = Oracle(3)
    n = o.n_edges
    errs = [geom.bits_of(n, [i]) for i in range(n)]
    errs += [geom.bits_of(n, [i, j]) for i, j in itertools.combinations(range(n), 2)]
    err = np.array(errs)
    corr, _ = o.bp_decode(o.syndrome(err), 0.05, 0.05, 20)
    assert np.array_equal(corr, err)


def test_L3_bp_returns_weight_one_errors():
    o = Oracle(3)
    n = o.n_edges
    err = np.eye(n, dtype=np.uint8)
    corr, _ = o.bp_decode(o.syndrome(err), 0.05, 0.05, 20)
    assert np.array_equal(corr, err)


def reflection_maps(L, axis):
    """Index maps of the reflection p -> p with coordinate `axis` negated
    (mod L), built from point sets alone (tests/geom.py): edge i goes to
    edge emap[i], face f to face fmap[f]."""
    import geom

    def refl(p):
        q = list(p)
        q[axis] = (-q[axis]) % L
        return tuple(q)

    e_of = {pts: idx for _, idx, pts in geom.all_edges(L)}
    emap = np.empty(3 * L ** 3, np.int64)
    for _, idx, pts in geom.all_edges(L):
        emap[idx] = e_of[frozenset(refl(p) for p in pts)]
    f_of = {}
    for z, y, x, n in itertools.product(range(L), range(L), range(L), range(3)):
        f_of[geom.face_corners(L, x, y, z, n)] = n * L ** 3 + site(L, x, y, z)
    fmap = np.empty(3 * L ** 3, np.int64)
    for corners, idx in f_of.items():
        fmap[idx] = f_of[frozenset(refl(p) for p in corners)]
    return emap, fmap


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_bp_commutes_with_reflections(axis):
    """Reflections are symmetries of the lattice and of the Tanner graph, and
    the flooding schedule treats every check alike, so reflecting the
    syndrome reflects every posterior (to 1e-12 in FP64). A mistake in which
    members a check excludes, or in an edge's neighbourhood on one side only,
    breaks it where translations and rotations cannot."""
    L = 5
    o = Oracle(L)
    emap, fmap = reflection_maps(L, axis)
    assert sorted(emap) == list(range(3 * L ** 3)) and sorted(fmap) == list(range(3 * L ** 3))
    err = random_bits(31 + axis, 1, o.n_edges, 0.08)
    syn = (o.syndrome(err) ^ random_bits(41 + axis, 1, o.n_faces, 0.03))[0]
    # the syndrome of a reflected error is the reflected syndrome
    err_r = np.zeros_like(err[0])
    err_r[emap] = err[0]
    syn_r_of_err = o.syndrome(err_r[None])[0]
    syn_plain = o.syndrome(err)[0]
    expect = np.zeros_like(syn_plain)
    expect[fmap] = syn_plain
    assert np.array_equal(syn_r_of_err, expect)
    syn_r = np.zeros_like(syn)
    syn_r[fmap] = syn
    for T in (1, 2, 9):
        _, post = o.bp_decode(syn[None], 0.05, 0.05, T)
        _, post_r = o.bp_decode(syn_r[None], 0.05, 0.05, T)
        np.testing.assert_allclose(post_r[0][emap], post[0], rtol=1e-12, atol=1e-12)


# ------------------------------------------- readings: damped and warm BP
def test_damped_step_reduces_to_the_plain_step():
    L = 4
    o = Oracle(L)
    syn = random_bits(61, 1, o.n_faces, 0.2)[0]
    nu = random_messages(62, 1, o.n_faces)[0]
    a, pa = o.bp_step(syn, 0.05, 0.05, nu_in=nu)
    b, pb = o.bp_step_damped(syn, 0.05, 0.05, 0.0, nu_in=nu)
    assert np.array_equal(a, b) and np.array_equal(pa, pb)


@pytest.mark.parametrize("damp", [0.3, 0.7])
def test_damped_zero_syndrome_scalar_recursion(damp):
    """On the zero syndrome every message is one scalar, and damping mixes it
    with the previous one: nu_t = (1 - g) F(nu_{t-1}) + g nu_{t-1}, nu_0 = 0,
    F(nu) = 2 atanh(K tanh((l0 + 3 nu)/2)^3); posterior l0 + 4 nu_T."""
    L, p, q, T = 4, 0.05, 0.05, 9
    o = Oracle(L)
    syn = np.zeros(o.n_faces, np.uint8)
    l0 = math.log((1 - p) / p)
    K = 1 - 2 * q
    nu, post = None, None
    s = 0.0
    for _ in range(T):
        nu, post = o.bp_step_damped(syn, p, q, damp, nu_in=nu)
        s = (1 - damp) * 2 * math.atanh(K * math.tanh((l0 + 3 * s) / 2) ** 3) + damp * s
        np.testing.assert_allclose(nu, s, rtol=1e-13)
    np.testing.assert_allclose(post, l0 + 4 * s, rtol=1e-13)


def test_warm_and_damped_runs():
    """run_cycles with the readings: damping 0 and a cold start are the
    paper's BP bit for bit; a warm start's first cycle is the cold one; its
    later cycles start from the previous cycle's final messages (checked by
    composing the damped step, the only BP in these runs)."""
    from oracle.oracle import make_params
    L, S = 4, 6
    o = Oracle(L)
    base = make_params(0.05, 0.05, 3, 6, 6, 0b001001, seed=13)
    m0, _, e0 = o.run_cycles(base, S)
    m1, _, e1 = o.run_cycles(make_params(0.05, 0.05, 3, 6, 6, 0b001001, seed=13, bp_damp=0.0),
                             S)
    assert np.array_equal(e0, e1) and np.array_equal(m0, m1)
    warm = make_params(0.05, 0.05, 1, 6, 6, 0b001001, seed=13, bp_warm=1, perfect_final=0)
    cold = make_params(0.05, 0.05, 1, 6, 6, 0b001001, seed=13, perfect_final=0)
    assert np.array_equal(o.run_cycles(warm, S)[2], o.run_cycles(cold, S)[2])
    # two warm cycles with damping by hand, one shot
    prm = make_params(0.06, 0.05, 2, 5, 0, 0, seed=21, bp_warm=1, bp_damp=0.4,
                      perfect_final=0)
    _, _, e_run = o.run_cycles(prm, 1, shot0=3)
    e = np.zeros((1, o.n_edges), np.uint8)
    nu = None
    for t in range(2):
        o.sample_noise(e, 0, 0.06, 21, t, 3)
        syn = o.syndrome(e)
        o.sample_noise(syn, 1, 0.05, 21, t, 3)
        for it in range(5):
            nu, post = o.bp_step_damped(syn[0], 0.06, 0.05, 0.4, nu_in=nu)
        e ^= (post < 0).astype(np.uint8)[None]
    assert np.array_equal(e, e_run)
