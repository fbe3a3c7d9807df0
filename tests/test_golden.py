"""Pins against the paper's worked examples and printed tables, read from the
text fixtures under tests/golden/.

* flip_examples.txt: the low-weight errors of Figs. 3-5 and Section 3.2. The
  oracle's parallel flip sweep, and an independent count of unsatisfied checks
  from lattice coordinates, must show what the paper states for each.
* table1_thresholds.txt: the schedule of every cell of Table 1 (shaded cells
  hold no p-flip sweep).
* table2_correlations.txt: the counts the experiment code carries, and the
  correlation the paper reads from them (Appendix A.2: several logical qubits
  fail together more often than independent failures would give, single ones
  less often)."""
import math

import numpy as np
import pytest

import geom
import golden_data as gd
from oracle.oracle import Oracle
from paper_2212_06985_amd import experiments as ex

L = gd.EXAMPLE_L
N_EDGES = 3 * L ** 3
EXAMPLES = gd.flip_examples()
_MEMBERS = []


def members():
    if not _MEMBERS:
        _MEMBERS.append(geom.face_members_by_points(L))
    return _MEMBERS[0]


def unsat_counts(err):
    """u_i and the number of unsatisfied checks, from face corner sets alone."""
    u = np.zeros(err.size, int)
    n_unsat = 0
    for f, m in members().items():
        if sum(int(err[i]) for i in m) % 2:
            n_unsat += 1
            for i in m:
                u[i] += 1
    return u, n_unsat


def test_fixture_is_complete():
    assert len(EXAMPLES) == 10
    for name, ex_ in EXAMPLES.items():
        assert ex_.get("cite") and ex_.get("support"), name
        assert "after1" in ex_, name


@pytest.mark.parametrize("name", sorted(EXAMPLES))
def test_flip_example(name):
    g = EXAMPLES[name]
    err = geom.bits_of(N_EDGES, sorted(g["support"]))
    u, n_unsat = unsat_counts(err)
    if "unsat" in g:
        assert n_unsat == g["unsat"]
    if "flips" in g:
        assert set(np.flatnonzero(u >= 3)) == g["flips"]
    if "ties" in g:
        assert set(np.flatnonzero(u == 2)) == g["ties"]
    o = Oracle(L)
    syn = o.syndrome(err[None])
    assert int(syn.sum()) == n_unsat
    corr = np.zeros_like(err[None])
    for k, key in enumerate(("after1", "after2")):
        o.flip_sweep(syn, corr)
        if key in g:
            assert set(np.flatnonzero(err ^ corr[0])) == g[key], key
        if k == 0 and g.get("cleared"):
            res = (err ^ corr[0])[None]
            _, odd = o.logical_check(res)
            assert o.syndrome(res).sum() == 0 and odd.sum() == 0
        if "after2" not in g:
            break


def test_table1_schedules():
    rows = gd.table1()
    assert len(rows) == 19
    for n_a, lam, th, shaded in rows:
        assert 0.02 < th < 0.05
        mask = ex.flip_mask(n_a, lam)
        # shaded exactly when lambda_p > n_A, and then the schedule is n_A flips
        assert shaded == (lam > n_a)
        assert (mask == 0) == shaded, (n_a, lam)
        assert mask == sum(1 << k for k in range(n_a) if (k + 1) % lam == 0)
        assert ex.decoder_params("flip", n_a, lam) == (0, n_a, mask)
    # the Fig. 2 decoder: one flip sweep per cycle
    assert [(n, lam) for n, lam, _, _ in rows if n == 1] == [(1, 2)]
    assert ex.decoder_params("flip", 1, 0) == (0, 1, 0)


def test_table2_counts_match_the_paper():
    paper = gd.table2()
    assert ex.TABLE2_COUNTS == paper
    assert sum(paper.values()) == 1000


def test_table2_correlations():
    c = ex.correlations(gd.table2())
    assert c["n"] == 1000
    # per-qubit failures: 128, 125 and 143 of 1000
    assert c["rate"] == pytest.approx([0.128, 0.125, 0.143], abs=1e-15)
    px, py, pz = 0.128, 0.125, 0.143
    assert c["expected"]["111"] == pytest.approx(1000 * px * py * pz, rel=1e-12)
    assert c["expected"]["000"] == pytest.approx(1000 * (1 - px) * (1 - py) * (1 - pz),
                                                 rel=1e-12)
    assert c["expected"]["101"] == pytest.approx(1000 * px * (1 - py) * pz, rel=1e-12)
    assert sum(c["expected"].values()) == pytest.approx(1000, rel=1e-12)
    # the paper's reading: joint failures above independence, single ones below
    for k, r in c["ratio"].items():
        weight = k.count("1")
        if weight >= 2:
            assert r > 1.5, k
        elif weight == 1:
            assert r < 0.8, k
    assert c["ratio"]["111"] > 10


def test_correlations_of_no_failure():
    c = ex.correlations({"000": 16384, **{format(k, "03b"): 0 for k in range(1, 8)}})
    assert c["rate"] == [0.0, 0.0, 0.0]
    assert c["ratio"]["000"] == 1.0
    assert all(c["ratio"][k] is None for k in c["ratio"] if k != "000")
    assert not any(math.isnan(v) for v in c["expected"].values())
    with pytest.raises(ValueError):
        ex.correlations({format(k, "03b"): 0 for k in range(8)})
