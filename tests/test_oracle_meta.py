"""Pins of the oracle's BP with meta-check factors (the extension Section 4.1
describes and does not use): closed forms of its first two iterations, whose
values depend on which faces make up each cube and which cubes hold each
face; the zero-syndrome scalar recursion with the message clamp; lattice
symmetry; and its effect on syndromes made of measurement errors only."""
import math

import numpy as np
import pytest

import geom
from inputs import random_bits
from oracle.oracle import Oracle

CLAMP = 30.0


def clamp(x):
    return max(-CLAMP, min(CLAMP, x))


def cube_parities(L, syn):
    """Parity of the measured outcomes of the six faces of every cube."""
    N = L ** 3
    par = np.zeros(N, np.uint8)
    for c in range(N):
        x, y, z = c % L, (c // L) % L, c // (L * L)
        par[c] = syn[geom.cube_faces(L, x, y, z)].sum() & 1
    return par


@pytest.mark.parametrize("L", [3, 4])
def test_first_two_iterations_closed_forms(L):
    p = q = 0.05
    l0 = math.log((1 - p) / p)
    lm = math.log((1 - q) / q)
    K = math.tanh(lm / 2)
    o = Oracle(L)
    N = L ** 3
    syn = random_bits(40 + L, 1, o.n_faces, 0.3)[0]
    # iteration 1: no factor messages yet; the qubit part is the paper's BP
    (nu1, lam1, kap1), _ = o.bp_meta_step(syn, p, q)
    nu_plain, _ = o.bp_step(syn, p, q)
    np.testing.assert_allclose(nu1, nu_plain, rtol=1e-14, atol=1e-14)
    s = np.where(syn == 1, -1.0, 1.0)
    np.testing.assert_allclose(lam1, s * 2 * math.atanh(math.tanh(l0 / 2) ** 4), rtol=1e-14)
    par = cube_parities(L, syn)
    want_k = np.where(par == 1, -1.0, 1.0) * 2 * math.atanh(K ** 5)
    np.testing.assert_allclose(kap1, np.repeat(want_k[:, None], 6, axis=1), rtol=1e-14)
    # iteration 2: the measurement message of face f is lm plus the kappa of
    # the two cubes that contain f
    (nu2, _, _), _ = o.bp_meta_step(syn, p, q, (nu1, lam1, kap1))
    fe, ef, es = o.incidence()
    holders = [[] for _ in range(o.n_faces)]
    for c in range(N):
        x, y, z = c % L, (c // L) % L, c // (L * L)
        for f in geom.cube_faces(L, x, y, z):
            holders[f].append(c)
    for f in range(o.n_faces):
        assert len(holders[f]) == 2
        M = clamp(lm + sum(want_k[c] for c in holders[f]))
        Q = []
        for k in range(4):
            e = fe[f, k]
            Q.append(clamp(l0 + sum(nu1[ef[e, j], es[e, j]] for j in range(4) if ef[e, j] != f)))
        for k in range(4):
            prod = math.tanh(M / 2)
            for kk in range(4):
                if kk != k:
                    prod *= math.tanh(Q[kk] / 2)
            want = s[f] * 2 * math.atanh(prod)
            assert abs(nu2[f, k] - want) <= 1e-12 * max(1.0, abs(want)), (f, k)


@pytest.mark.parametrize("L", [3, 4])
def test_zero_syndrome_scalar_recursion_with_clamp(L):
    p = q = 0.05
    l0 = math.log((1 - p) / p)
    lm = math.log((1 - q) / q)
    o = Oracle(L)
    syn = np.zeros(o.n_faces, np.uint8)
    nu = lam = kap = 0.0
    state = None
    for t in range(1, 9):
        Q, M, R = clamp(l0 + 3 * nu), clamp(lm + 2 * kap), clamp(lm + lam + kap)
        nu, lam, kap = (2 * math.atanh(math.tanh(M / 2) * math.tanh(Q / 2) ** 3),
                        2 * math.atanh(math.tanh(Q / 2) ** 4),
                        2 * math.atanh(math.tanh(R / 2) ** 5))
        state, post = o.bp_meta_step(syn, p, q, state)
        np.testing.assert_allclose(post, l0 + 4 * nu, rtol=1e-12)
        np.testing.assert_allclose(state[2], kap, rtol=1e-12)
    # the loops feed back: the messages saturate at the clamp instead of
    # converging as without meta-checks
    assert post.min() > 50


def test_translation_and_axis_symmetry():
    L, p, q = 4, 0.05, 0.05
    o = Oracle(L)
    N = L ** 3
    syn = random_bits(77, 1, o.n_faces, 0.25)[0]
    _, post = o.bp_meta_decode(syn[None], p, q, 6)

    def site(x, y, z):
        return (x % L) + L * ((y % L) + L * (z % L))

    # translate by (1, 2, 3)
    syn_t = np.zeros_like(syn)
    for n in range(3):
        for v in range(N):
            x, y, z = v % L, (v // L) % L, v // (L * L)
            syn_t[n * N + site(x + 1, y + 2, z + 3)] = syn[n * N + v]
    _, post_t = o.bp_meta_decode(syn_t[None], p, q, 6)
    for a in range(3):
        for v in range(N):
            x, y, z = v % L, (v // L) % L, v // (L * L)
            assert abs(post_t[0, a * N + site(x + 1, y + 2, z + 3)] - post[0, a * N + v]) < 1e-9
    # swap the x and y axes: faces of normal 0 <-> 1, edges of axis 0 <-> 1
    syn_s = np.zeros_like(syn)
    perm = [1, 0, 2]
    for n in range(3):
        for v in range(N):
            x, y, z = v % L, (v // L) % L, v // (L * L)
            syn_s[perm[n] * N + site(y, x, z)] = syn[n * N + v]
    _, post_s = o.bp_meta_decode(syn_s[None], p, q, 6)
    for a in range(3):
        for v in range(N):
            x, y, z = v % L, (v // L) % L, v // (L * L)
            assert abs(post_s[0, perm[a] * N + site(y, x, z)] - post[0, a * N + v]) < 1e-9


def test_meta_checks_explain_measurement_errors():
    """Syndromes made of measurement errors alone: every qubit flip is a
    mistake. The meta-checks see the open strings such errors leave and make
    BP flip fewer qubits than without them."""
    L, p, q = 6, 0.05, 0.05
    o = Oracle(L)
    S = 200
    syn = random_bits(5, S, o.n_faces, q)
    c_plain, _ = o.bp_decode(syn, p, q, 20)
    c_meta, _ = o.bp_meta_decode(syn, p, q, 20)
    # 120 against 59 wrong flips on these 200 syndromes; the bar leaves room
    # for the count's own spread (a few times its square root)
    assert c_meta.sum() < c_plain.sum() - 4 * math.sqrt(c_plain.sum()), \
        (c_meta.sum(), c_plain.sum())
