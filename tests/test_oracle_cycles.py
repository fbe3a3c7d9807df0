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
