"""Pins of the oracle's majority-vote readout and multi-cycle loop."""
import itertools

import numpy as np
import pytest

import geom
from inputs import random_bits
from oracle.oracle import Oracle, make_params


@pytest.mark.parametrize("L", [3, 4, 6])
def test_membrane_sets_only_its_axis(L):
    o = Oracle(L)
    for a in range(3):
        e = geom.bits_of(o.n_edges, geom.membrane(L, a, 1))
        mask, odd = o.logical_check(e[None])
        assert mask[0] == 1 << a
        assert odd[0, a] == L * L
        assert odd[0].sum() == L * L


@pytest.mark.parametrize("L", [3, 4])
def test_readout_ignores_stabilisers(L):
    o = Oracle(L)
    rng = np.random.default_rng(L)
    err = random_bits(40 + L, 6, o.n_edges, 0.05)
    m0, odd0 = o.logical_check(err)
    for _ in range(4):
        x, y, z = rng.integers(0, L, size=3)
        st = geom.bits_of(o.n_edges, geom.star(L, x, y, z))
        m1, _ = o.logical_check(err ^ st)
        assert np.array_equal(m0, m1)
    zero = np.zeros((1, o.n_edges), np.uint8)
    assert o.logical_check(zero)[0][0] == 0


def test_majority_counts_lines_and_ties_fail():
    L = 4
    o = Oracle(L)
    # k disjoint logical Z strings along x each hit once
    for k in range(L * L + 1):
        e = np.zeros(o.n_edges, np.uint8)
        lines = list(itertools.product(range(L), range(L)))[:k]
        for i, j in lines:
            e[geom.string(L, 0, i, j)[0]] ^= 1
        mask, odd = o.logical_check(e[None])
        assert odd[0, 0] == k
        assert bool(mask[0] & 1) == (2 * k >= L * L)


def test_noiseless_run_stays_clean():
    o = Oracle(4)
    prm = make_params(0.0, 0.0, noisy_cycles=3, bp_iters=5, n_sweeps=6, pflip_mask=0b001001)
    mask, odd, err = o.run_cycles(prm, 5)
    assert mask.sum() == 0 and err.sum() == 0


def test_run_matches_composed_stages():
    """One cycle of the multi-cycle run equals noise, syndrome, measurement noise, BP,
    working-syndrome update, the sweep schedule and the final correction."""
    L = 4
    o = Oracle(L)
    prm = make_params(0.04, 0.03, noisy_cycles=2, bp_iters=4, n_sweeps=6,
                      pflip_mask=0b001001, seed=77)
    S, shot0 = 5, 128
    mask, odd, err, tr = o.run_cycles(prm, S, shot0=shot0, trace=True)
    e = np.zeros((S, o.n_edges), np.uint8)
    for t in range(3):
        qt = 0.03 if t < 2 else 0.0
        o.sample_noise(e, 0, 0.04, 77, t, shot0)
        syn = o.syndrome(e)
        o.sample_noise(syn, 1, qt, 77, t, shot0)
        corr, _ = o.bp_decode(syn, 0.04, 0.03, 4)
        o.syndrome(corr, syn, xor_into=True)
        for k in range(6):
            if (0b001001 >> k) & 1:
                o.pflip_sweep(syn, corr, 77, t, k, shot0)
            else:
                o.flip_sweep(syn, corr)
        e ^= corr
        assert np.array_equal(e, tr[t])
    assert np.array_equal(e, err)
    m2, odd2 = o.logical_check(e)
    assert np.array_equal(m2, mask) and np.array_equal(odd2, odd)


def test_perfect_final_round_leaves_valid_syndrome_region():
    """After the perfect round of a flip-only decoder every shot's residual
    syndrome is a valid (cube-even) one, and residuals stay small at low p."""
    L = 6
    o = Oracle(L)
    prm = make_params(0.02, 0.02, noisy_cycles=6, bp_iters=0, n_sweeps=5, pflip_mask=0b00100)
    mask, odd, err = o.run_cycles(prm, 64)
    assert err.sum(axis=1).mean() < 0.05 * o.n_edges
    syn = o.syndrome(err)
    for x, y, z in itertools.product(range(L), repeat=3):
        assert (syn[:, geom.cube_faces(L, x, y, z)].sum(axis=1) % 2 == 0).all()


def test_shots_are_independent_and_reproducible():
    o = Oracle(4)
    prm = make_params(0.05, 0.05, noisy_cycles=3, bp_iters=3, n_sweeps=6, pflip_mask=0b001001)
    m_all, odd_all, e_all = o.run_cycles(prm, 8, shot0=0)
    m_sub, odd_sub, e_sub = o.run_cycles(prm, 3, shot0=5)
    assert np.array_equal(e_all[5:8], e_sub)
    assert np.array_equal(odd_all[5:8], odd_sub)


def test_run_prefix_equals_shorter_run():
    """The residual after cycle 2 of a longer run equals a 2-cycle run: a
    shot's trajectory depends only on (seed, shot, cycle)."""
    o = Oracle(4)
    full = make_params(0.05, 0.05, noisy_cycles=4, bp_iters=3, n_sweeps=6, pflip_mask=0b001001,
                       perfect_final=0)
    _, _, e_full, tr = o.run_cycles(full, 4, trace=True)
    assert np.array_equal(tr[1], o.run_cycles(
        make_params(0.05, 0.05, noisy_cycles=2, bp_iters=3, n_sweeps=6, pflip_mask=0b001001,
                    perfect_final=0), 4)[2])


def test_logical_error_rate_grows_with_p():
    o = Oracle(4)
    rates = []
    for p in (0.01, 0.08):
        prm = make_params(p, p, noisy_cycles=4, bp_iters=0, n_sweeps=5, pflip_mask=0b00100)
        mask, _, _ = o.run_cycles(prm, 200)
        rates.append((mask != 0).mean())
    assert rates[0] < rates[1]


# ----------------------------------------------------- checkpoint / resume
@pytest.mark.parametrize("kind", ["flip", "pbp", "subset"])
def test_resumed_run_equals_unsplit_run(kind):
    """A run split after cycle k and resumed from its residual with cycle0 = k
    equals the unsplit run: noise and coins are keyed by the experiment's cycle
    index, so the residual and the next cycle index are the whole state."""
    L, S = 4, 6
    o = Oracle(L)
    kw = dict(flip=dict(bp_iters=0, n_sweeps=5, pflip_mask=0b00100),
              pbp=dict(bp_iters=5, n_sweeps=6, pflip_mask=0b001001),
              subset=dict(bp_iters=0, n_sweeps=5, pflip_mask=0, subset_mask=0b00100))[kind]
    full = make_params(0.06, 0.05, noisy_cycles=5, seed=9, **kw)
    m_full, odd_full, e_full = o.run_cycles(full, S, shot0=64)
    for k in (1, 3):
        head = make_params(0.06, 0.05, noisy_cycles=k, perfect_final=0, seed=9, **kw)
        _, _, e_k = o.run_cycles(head, S, shot0=64)
        tail = make_params(0.06, 0.05, noisy_cycles=5 - k, seed=9, cycle0=k, **kw)
        m, odd, e = o.run_cycles(tail, S, shot0=64, err=e_k.copy())
        assert np.array_equal(e, e_full) and np.array_equal(m, m_full), k
        assert np.array_equal(odd, odd_full)
    # a resumed call that starts from the wrong cycle draws other noise
    wrong = make_params(0.06, 0.05, noisy_cycles=4, seed=9, **kw)
    _, _, e_1 = o.run_cycles(make_params(0.06, 0.05, noisy_cycles=1, perfect_final=0, seed=9,
                                         **kw), S, shot0=64)
    _, _, e_w = o.run_cycles(wrong, S, shot0=64, err=e_1.copy())
    assert not np.array_equal(e_w, e_full)


# ------------------------------------- planted errors through the whole cycle
# With p = q = 0 a cycle adds no noise, so run_cycles decodes exactly the
# planted error. The expected residuals below come from the paper's examples
# and from the geometry of a vertex star, not from the oracle's stages.
def star_edges(L, x, y, z):
    """The six edges at vertex v as {(axis, sign): edge}: +a = e(v,a),
    -a = e(v - unit(a), a)."""
    from inputs import edge
    out = {}
    for a in range(3):
        d = [0, 0, 0]
        d[a] = -1
        out[(a, +1)] = edge(L, x, y, z, a)
        out[(a, -1)] = edge(L, x + d[0], y + d[1], z + d[2], a)
    return out


def star_automaton(L, v, A, schedule, coin):
    """Parallel flip / p-flip sweeps on an error inside the star of v.

    Each face at v holds exactly two star edges, one of each of two different
    axes, and each pair of perpendicular star edges shares exactly one face;
    every other edge touches at most one face at v. So for A inside the star,
    the unsatisfied checks of a star edge e are the faces it shares with the
    perpendicular star edges e' with [e' in A] != [e in A], other edges see at
    most one unsatisfied check and never flip, and the sweeps stay inside the
    star. schedule: 'P' or 'F' per sweep; coin(edge, sweep) -> 0/1."""
    st = star_edges(L, *v)
    A = set(A)
    for k, kind in enumerate(schedule):
        flips = set()
        for (a, sg), e in st.items():
            u = sum(1 for (b, _), f in st.items() if b != a and ((f in A) != (e in A)))
            if u >= 3 or (kind == "P" and u == 2 and coin(e, k)):
                flips.add(e)
        A ^= flips
    return A


@pytest.mark.parametrize("L", [4, 6])
def test_planted_corner_half_star_through_one_pffpff_cycle(L):
    """Section 3.2: the corner half-star (Fig. 3a) is stuck under flip (every
    star edge has exactly 2 unsatisfied checks) and p-flip's coin flips decide
    its fate. One P F F P F F cycle of run_cycles over 64 shots (64 coin
    streams) ends on the residual the star automaton predicts for each shot;
    some shots clear it (residual 0 or the whole star, a stabiliser) and some
    keep a half-star."""
    from oracle.oracle import coin
    o = Oracle(L)
    v = (1, 2, 1)
    st = star_edges(L, *v)
    A0 = {st[(0, 1)], st[(1, 1)], st[(2, 1)]}
    S, shot0, seed = 64, 128, 5
    err = np.zeros((S, o.n_edges), np.uint8)
    err[:, sorted(A0)] = 1
    prm = make_params(0.0, 0.0, noisy_cycles=1, bp_iters=0, n_sweeps=6, pflip_mask=0b001001,
                      perfect_final=0, seed=seed)
    _, _, res = o.run_cycles(prm, S, shot0=shot0, err=err)
    outcomes = {"cleared": 0, "stuck": 0}
    for s in range(S):
        want = star_automaton(L, v, A0, "PFFPFF",
                              lambda e, k: coin(seed, e, 0, k, shot0 + s))
        assert set(np.flatnonzero(res[s])) == want, s
        outcomes["cleared" if len(want) in (0, 6) else "stuck"] += 1
    assert outcomes["cleared"] > 0 and outcomes["stuck"] > 0, outcomes


@pytest.mark.parametrize("L", [4, 6])
def test_planted_errors_decoded_by_bp_inside_run_cycles(L):
    """The BP family's cycle: BP (T = 20, p_dec = q_dec = 5%) then P F F P F F.
    * the planar 2 x 2 error of Fig. 3b, which flip cannot correct, is
      corrected by BP (Section 4.1), so the residual is zero;
    * single qubit errors are corrected (the lowest-weight case);
    * a logical X membrane has zero syndrome: nothing flips and the readout
      reports its axis;
    * the corner half-star: BP gives its six star edges one posterior (the
      star's symmetry) and flips all or none, then the sweeps act as the star
      automaton, so the residual is the automaton's, possibly times the star."""
    from inputs import edge
    from oracle.oracle import coin
    o = Oracle(L)
    cases = {
        "planar": [edge(L, i, j, 0, 2) for i in (0, 1) for j in (0, 1)],
        "single_x": [edge(L, 2, 1, 3, 0)],
        "single_z": [edge(L, 0, 0, 0, 2)],
        "membrane_y": geom.membrane(L, 1, 2),
    }
    S, seed = len(cases), 3
    err = np.zeros((S, o.n_edges), np.uint8)
    for s, sup in enumerate(cases.values()):
        err[s, sup] = 1
    prm = make_params(0.0, 0.0, noisy_cycles=1, bp_iters=20, n_sweeps=6, pflip_mask=0b001001,
                      perfect_final=0, seed=seed, p_dec=0.05, q_dec=0.05)
    mask, odd, res = o.run_cycles(prm, S, err=err)
    for s, name in enumerate(cases):
        if name == "membrane_y":
            assert set(np.flatnonzero(res[s])) == set(cases[name])
            assert mask[s] == 0b010 and odd[s, 1] == L * L
        else:
            assert res[s].sum() == 0 and mask[s] == 0, name
    v = (2, 2, 2)
    st = star_edges(L, *v)
    A0 = {st[(0, 1)], st[(1, 1)], st[(2, 1)]}
    S = 16
    err = np.zeros((S, o.n_edges), np.uint8)
    err[:, sorted(A0)] = 1
    _, _, res = o.run_cycles(prm, S, err=err)
    whole = set(st.values())
    for s in range(S):
        want = star_automaton(L, v, A0, "PFFPFF", lambda e, k: coin(seed, e, 0, k, s))
        got = set(np.flatnonzero(res[s]))
        assert got in (want, want ^ whole), s
