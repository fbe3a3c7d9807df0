"""Pins of the oracle's subset p-flip, the recovery rule of Dennis et al. that
the footnote of Section 3.2 contrasts with p-flip: it acts only on a set of
qubits no two of which are in the same check. The oracle's 12 edge classes
must each be such a set, together cover every qubit once, and a parallel
sweep on one class must equal the same rule applied one qubit at a time in
any order (which is what the independence buys)."""
import numpy as np
import pytest

from inputs import random_bits
from oracle.oracle import Oracle, coin, make_params, subset_class


@pytest.mark.parametrize("L", [4, 6])
def test_classes_are_independent_sets_covering_every_qubit(L):
    o = Oracle(L)
    fe, _, _ = o.incidence()
    cls = np.array([o.edge_class(e) for e in range(o.n_edges)])
    assert set(cls.tolist()) == set(range(12))
    assert np.all(np.bincount(cls, minlength=12) == o.n_sites // 4)
    # no check holds two qubits of one class
    for f in range(o.n_faces):
        assert len(set(cls[fe[f]].tolist())) == 4, f
    # a class is one axis and one parity pattern of the two other coordinates
    N = o.n_sites
    for e in range(o.n_edges):
        a, v = divmod(e, N)
        x, y, z = v % L, (v // L) % L, v // (L * L)
        others = [c for i, c in enumerate((x, y, z)) if i != a]
        assert cls[e] // 4 == a
        assert cls[e] % 4 == 2 * (others[0] % 2) + (others[1] % 2)


def test_odd_lattices_have_no_such_colouring_with_two_parities():
    """With L odd the wrap joins coordinates L-1 and 0, both even: some check
    then holds two qubits of one class, so the subset rule needs L even."""
    o = Oracle(5)
    fe, _, _ = o.incidence()
    cls = np.array([o.edge_class(e) for e in range(o.n_edges)])
    assert any(len(set(cls[fe[f]].tolist())) < 4 for f in range(o.n_faces))


def _sequential(o, syn, corr, members, coins, order):
    ef = o.incidence()[1]
    for b in order:
        if b not in members:
            continue
        u = int(syn[ef[b]].sum())
        if u >= 3 or (u == 2 and coins[b]):
            corr[b] ^= 1
            syn[ef[b]] ^= 1


@pytest.mark.parametrize("cls", [0, 5, 11])
def test_parallel_subset_sweep_equals_any_sequential_order(cls):
    L, seed, cycle, sweep = 4, 7, 3, 2
    o = Oracle(L)
    members = {e for e in range(o.n_edges) if o.edge_class(e) == cls}
    rng = np.random.default_rng(cls)
    for trial in range(20):
        syn = random_bits(100 + trial, 1, o.n_faces, 0.4)[0]
        corr = random_bits(200 + trial, 1, o.n_edges, 0.1)[0]
        s_par, c_par = syn.copy(), corr.copy()
        o.subset_pflip_sweep(s_par, c_par, seed, cycle, sweep, cls, shot0=trial)
        coins = np.array([coin(seed, e, cycle, sweep, trial) for e in range(o.n_edges)])
        for _ in range(3):
            s_seq, c_seq = syn.copy(), corr.copy()
            _sequential(o, s_seq, c_seq, members, coins, rng.permutation(o.n_edges))
            assert np.array_equal(s_par, s_seq) and np.array_equal(c_par, c_seq)
        # only the class's qubits ever move
        moved = np.flatnonzero(c_par != corr)
        assert all(e in members for e in moved)


def test_full_pflip_is_not_order_free():
    """Contrast: the ordinary parallel p-flip acts on neighbouring qubits at
    once and differs from a sequential pass, so the test above can fail."""
    L, seed = 4, 7
    o = Oracle(L)
    everyone = set(range(o.n_edges))
    rng = np.random.default_rng(1)
    differs = False
    for trial in range(20):
        syn = random_bits(300 + trial, 1, o.n_faces, 0.4)[0]
        corr = np.zeros(o.n_edges, np.uint8)
        s_par, c_par = syn.copy(), corr.copy()
        o.pflip_sweep(s_par, c_par, seed, 0, 0, shot0=trial)
        coins = np.array([coin(seed, e, 0, 0, trial) for e in range(o.n_edges)])
        s_seq, c_seq = syn.copy(), corr.copy()
        _sequential(o, s_seq, c_seq, everyone, coins, rng.permutation(o.n_edges))
        differs |= not np.array_equal(c_par, c_seq)
    assert differs


def test_class_schedule_visits_every_class():
    # m subset sweeps per cycle walk the 12 classes in order, wrapping
    for m in (1, 2, 3, 5):
        seen = [subset_class(j, m, t) for t in range(12) for j in range(m)]
        assert seen[:12] == [k % 12 for k in range(12)]
        assert set(seen) == set(range(12))


def test_run_cycles_with_subset_sweeps_is_deterministic_and_differs_from_pflip():
    L, S = 4, 8
    o = Oracle(L)
    a = make_params(0.05, 0.05, 4, 0, 5, 0b00100, seed=3)
    b = make_params(0.05, 0.05, 4, 0, 5, 0b00100, seed=3, subset_mask=0b00100)
    ma, ea = o.run_cycles(a, S)[:2]
    mb, eb = o.run_cycles(b, S)[:2]
    mb2, eb2 = o.run_cycles(b, S)[:2]
    assert np.array_equal(eb, eb2) and np.array_equal(mb, mb2)
    assert not np.array_equal(ea, eb)
