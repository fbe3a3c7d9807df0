"""GPU parity of the whole experiment (tc3d_run_cycles) against the oracle.

* flip + p-flip without BP (L = 6, p = q = 0.02, 6 noisy cycles + 1 perfect,
  schedule F F P F F, 10^4 shots, seed 1): every shot's residual error, mask
  and odd-string counts bit for bit, and the residual after every cycle.
* with BP (FP32 against FP64): shots whose BP decisions never met a
  near-tie agree bit for bit; the rest are counted and the logical error
  rates agree within 3 sigma.
* the full-size configuration (L = 48, p = q = 0.05, BP 20 + P F F P F F,
  2048 shots per batch): sampled shots against the oracle after one cycle,
  plus properties that hold at any size (valid residual syndromes,
  reproducibility, independence of the batch split).
"""
import math

import numpy as np
import pytest

import inputs
import paper_2212_06985_amd as tc
from gpu_util import announce, bits_of_dev, oracle_run_parallel, plane_from_dev
from oracle.oracle import Oracle, make_params

pytestmark = pytest.mark.gpu

FFPFF = 0b00100
PFFPFF = 0b001001


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    tc.lib()
    yield
    torch.cuda.synchronize()


def gpu_run(L, prm, err=None, timed=False):
    import torch
    lat = tc.make_lattice(L)
    S = prm.n_shots
    W = tc.n_words(S)
    if err is None:
        err = torch.zeros((lat.n_edges, W), dtype=torch.int64, device="cuda")
    mask = torch.zeros(S, dtype=torch.uint8, device="cuda")
    odd = torch.zeros((S, 3), dtype=torch.int32, device="cuda")
    ws = tc.alloc_workspace(tc.run_workspace_bytes(lat, prm))
    if timed:
        t = tc.run_cycles_timed(lat, prm, err, mask, odd, ws)
    else:
        tc.run_cycles(lat, prm, err, mask, odd, ws)
        t = None
    torch.cuda.synchronize()
    return (mask.cpu().numpy(), odd.cpu().numpy(), bits_of_dev(err, S), t)


def oracle_params(p, q, noisy, bp, sweeps, mask, seed=1, perfect_final=1):
    return make_params(p, q, noisy_cycles=noisy, bp_iters=bp, n_sweeps=sweeps,
                       pflip_mask=mask, seed=seed, perfect_final=perfect_final)


def test_flip_pflip_config_bit_exact():
    L, S = 6, 10_000
    announce(f"run_cycles flip+p-flip L={L} S={S}")
    prm = tc.make_run_params(0.02, 0.02, 6, 0, 5, FFPFF, n_shots=S, seed=1)
    m_g, odd_g, e_g, _ = gpu_run(L, prm)
    o = Oracle(L)
    m_o, odd_o, e_o = oracle_run_parallel(o, oracle_params(0.02, 0.02, 6, 0, 5, FFPFF), S)
    assert np.array_equal(e_g, e_o)
    assert np.array_equal(odd_g, odd_o)
    assert np.array_equal(m_g, m_o)
    announce(f"  logical failures (any axis) {int((m_g != 0).sum())} / {S}")
    # a different batch split gives identical results
    prm.batch_shots = 1024
    m_b, odd_b, e_b, _ = gpu_run(L, prm)
    assert np.array_equal(e_b, e_g) and np.array_equal(m_b, m_g)


def test_flip_pflip_every_cycle_bit_exact():
    """Residual after every cycle: the run truncated after t cycles equals the
    oracle's trace at cycle t (trajectories depend only on seed, shot, cycle)."""
    L, S = 6, 640
    o = Oracle(L)
    full = oracle_params(0.02, 0.02, 6, 0, 5, FFPFF)
    _, _, _, tr = o.run_cycles(full, S, trace=True)
    for t in range(1, 7):
        announce(f"  prefix of {t} noisy cycles")
        prm = tc.make_run_params(0.02, 0.02, t, 0, 5, FFPFF, n_shots=S, seed=1, perfect_final=0)
        _, _, e_g, _ = gpu_run(L, prm)
        assert np.array_equal(e_g, tr[t - 1]), t
    prm = tc.make_run_params(0.02, 0.02, 6, 0, 5, FFPFF, n_shots=S, seed=1)
    _, _, e_g, _ = gpu_run(L, prm)
    assert np.array_equal(e_g, tr[6])


@pytest.mark.parametrize("kind", ["flip", "pbp", "pbp_streaming"])
def test_resumed_run_equals_unsplit_run(kind):
    """Checkpoint / resume: a run split after cycle k (perfect_final = 0)
    and continued from its residual with cycle0 = k equals the unsplit run bit
    for bit, on the GPU, and equals the oracle's resumed run."""
    L, S = 6, 192
    kw = dict(flip=dict(bp_iters=0, n_sweeps=5, pflip_mask=FFPFF),
              pbp=dict(bp_iters=20, n_sweeps=6, pflip_mask=PFFPFF),
              pbp_streaming=dict(bp_iters=20, n_sweeps=6, pflip_mask=PFFPFF,
                                 bp_path=tc.BP_STREAMING))[kind]
    announce(f"resume {kind} L={L} S={S}")
    full = tc.make_run_params(0.05, 0.05, 5, n_shots=S, seed=8, shot0=128, **kw)
    m_full, odd_full, e_full, _ = gpu_run(L, full)
    for k in (1, 3):
        head = tc.make_run_params(0.05, 0.05, k, n_shots=S, seed=8, shot0=128, perfect_final=0,
                                  **kw)
        _, _, e_k, _ = gpu_run(L, head)
        tail = tc.make_run_params(0.05, 0.05, 5 - k, n_shots=S, seed=8, shot0=128, cycle0=k,
                                  **kw)
        from gpu_util import dev_plane_of_bits
        m, odd, e, _ = gpu_run(L, tail, err=dev_plane_of_bits(e_k))
        assert np.array_equal(e, e_full) and np.array_equal(m, m_full), k
        assert np.array_equal(odd, odd_full), k
    o = Oracle(L)
    kwo = {k: v for k, v in kw.items() if k != "bp_path"}
    prm_o = make_params(0.05, 0.05, 3, seed=8, cycle0=2, **kwo)
    e2 = o.run_cycles(make_params(0.05, 0.05, 2, seed=8, perfect_final=0, **kwo), S,
                      shot0=128)[2]
    m_o, _, e_o = o.run_cycles(prm_o, S, shot0=128, err=e2)
    same = ((e_o == e_full).all(axis=1) & (m_o == m_full)).sum()
    announce(f"  oracle resumed run: {same}/{S} shots identical")
    assert same == S if kind == "flip" else same >= S - 4


def test_run_continues_from_given_state_and_shot_offset():
    L, S = 5, 200
    o = Oracle(L)
    init = inputs.random_bits(9, S, o.n_edges, 0.01)
    prm_o = oracle_params(0.03, 0.03, 3, 0, 5, FFPFF, seed=44)
    m_o, odd_o, e_o = o.run_cycles(prm_o, S, shot0=640, err=init.copy())
    prm = tc.make_run_params(0.03, 0.03, 3, 0, 5, FFPFF, n_shots=S, seed=44, shot0=640)
    from gpu_util import dev_plane_of_bits
    d = dev_plane_of_bits(init)
    m_g, odd_g, e_g, _ = gpu_run(L, prm, err=d)
    assert np.array_equal(e_g, e_o) and np.array_equal(m_g, m_o)


def _compare_bp_run(L, S, p, noisy, seed=1):
    prm = tc.make_run_params(p, p, noisy, 20, 6, PFFPFF, n_shots=S, seed=seed)
    m_g, odd_g, e_g, _ = gpu_run(L, prm)
    o = Oracle(L)
    m_o, odd_o, e_o = oracle_run_parallel(o, oracle_params(p, p, noisy, 20, 6, PFFPFF, seed), S)
    same = (e_g == e_o).all(axis=1) & (m_g == m_o)
    n_div = int((~same).sum())
    f_g, f_o = (m_g & 1 != 0).mean(), (m_o & 1 != 0).mean()
    sig = math.sqrt(f_g * (1 - f_g) / S + f_o * (1 - f_o) / S)
    announce(f"  L={L} p={p}: diverged shots {n_div}/{S}; LER(x) gpu {f_g:.4f} "
             f"oracle {f_o:.4f}")
    return n_div, f_g, f_o, sig


@pytest.mark.parametrize("L,S,p,noisy", [(6, 512, 0.05, 6), (5, 256, 0.04, 5),
                                         (12, 128, 0.05, 3)])
def test_bp_pflip_run_matches_oracle(L, S, p, noisy):
    announce(f"run_cycles BP+p-flip L={L} S={S} p={p}")
    n_div, f_g, f_o, sig = _compare_bp_run(L, S, p, noisy)
    assert n_div <= max(2, S // 50)  # FP32 vs FP64 near-ties are rare
    assert abs(f_g - f_o) <= 3 * sig + 1e-12


@pytest.mark.parametrize("path", ["resident", "streaming", "split"])
def test_timed_run_counts_launches(path):
    L, S = 5, 128
    prm = tc.make_run_params(0.05, 0.05, 2, 7, 6, PFFPFF, n_shots=S, seed=3,
                             bp_path={"resident": tc.BP_RESIDENT, "streaming": tc.BP_STREAMING,
                                      "split": tc.BP_STREAMING_SPLIT}[path])
    m_a, _, e_a, t = gpu_run(L, prm, timed=True)
    m_b, _, e_b, _ = gpu_run(L, prm)
    assert np.array_equal(e_a, e_b) and np.array_equal(m_a, m_b)
    d = t.as_dict()
    cycles = 3
    if path == "resident":  # one launch decodes each cycle's batch inside LDS
        assert d["bp_iter"]["launches"] == cycles
        assert d["bp_first"]["launches"] == 0 and d["bp_post"]["launches"] == 0
    else:  # iteration 1 is implied by the syndrome; 2 reads only syndrome bits
        fused = path == "streaming"  # iteration 7 shares the posterior's launch
        assert d["bp_iter"]["launches"] == cycles * (7 - 2 - fused)
        assert d["bp_first"]["launches"] == cycles
        assert d["bp_post"]["launches"] == cycles
    assert d["sweep"]["launches"] == cycles * 6
    assert d["readout"]["launches"] == 2  # string parities, then the counts
    assert t.bp_decisions == cycles * 3 * L ** 3 * 128
    assert 0 <= t.bp_near_ties <= t.bp_decisions
    # class intervals are disjoint runs of launches inside the call's span
    assert sum(v["ms"] for v in d.values()) <= t.total_ms * 1.001 + 1e-3
    assert t.total_ms >= sum(v["ms"] for v in d.values()) * 0.5


def test_fused_last_iteration_run_equals_split_run():
    """A whole p-BP run at L = 16 (streaming kernels) with the last BP
    iteration fused into the posterior against the same run with the two
    launched separately: residuals, masks, odd counts and the near-tie
    counts bit for bit."""
    L, S = 16, 320
    out = {}
    for path in (tc.BP_STREAMING, tc.BP_STREAMING_SPLIT):
        prm = tc.make_run_params(0.06, 0.06, 4, 20, 6, PFFPFF, n_shots=S, seed=11,
                                 bp_path=path)
        m, o, e, t = gpu_run(L, prm, timed=True)
        out[path] = (m, o, e, t.bp_near_ties, t.bp_decisions)
    a, b = out[tc.BP_STREAMING], out[tc.BP_STREAMING_SPLIT]
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert a[3:] == b[3:]
    assert a[2].any()


def test_large_lattice_traversals_decode_alike():
    """From L = 72 the default traversal of the stored-message BP iterations
    is bands of 8 rows; whole planes (bp_tile = -L), 16 x 16 columns and the
    default decode every shot identically (p = q = 5%, 2 + 1 cycles)."""
    L, S = 72, 64
    out = []
    for tile in (0, -L, 16):
        prm = tc.make_run_params(0.05, 0.05, 2, 20, 6, PFFPFF, n_shots=S, seed=5,
                                 bp_tile=tile)
        m, o, e, _ = gpu_run(L, prm)
        out.append((m, o, e))
    for m, o, e in out[1:]:
        assert np.array_equal(m, out[0][0]) and np.array_equal(o, out[0][1])
        assert np.array_equal(e, out[0][2])
    assert out[0][2].any()


# ----------------------------------------------------------- full size
def test_full_size_sampled_shots_and_invariants():
    """L = 48, p = q = 0.05, BP 20 + P F F P F F, 2048 shots in one batch (the
    benchmark's launch configuration): sampled shots after one cycle against
    the oracle, then invariants of a longer run at full size."""
    import torch
    import geom
    L, S = 48, 2048
    announce(f"full size L={L} S={S}: one cycle")
    prm = tc.make_run_params(0.05, 0.05, 1, 20, 6, PFFPFF, n_shots=S, seed=1, perfect_final=0,
                             batch_shots=2048)
    m_g, odd_g, e_g, _ = gpu_run(L, prm)
    o = Oracle(L)
    samples = [0, 63, 64, 1001, 2047]
    import concurrent.futures as cf
    po = oracle_params(0.05, 0.05, 1, 20, 6, PFFPFF, perfect_final=0)
    with cf.ThreadPoolExecutor(len(samples)) as ex:
        res = list(ex.map(lambda s: o.run_cycles(po, 1, shot0=s), samples))
    n_same = 0
    for s, (m, odd, e) in zip(samples, res):
        diff = int((e[0] != e_g[s]).sum())
        announce(f"  shot {s}: residual weight gpu {int(e_g[s].sum())} oracle {int(e[0].sum())}"
                 f" differing edges {diff}")
        n_same += diff == 0
    assert n_same >= len(samples) - 1

    announce("full size: 3 noisy + 1 perfect cycle, invariants")
    prm = tc.make_run_params(0.05, 0.05, 3, 20, 6, PFFPFF, n_shots=S, seed=1,
                             batch_shots=2048)
    m1, odd1, e1, _ = gpu_run(L, prm)
    m2, odd2, e2, _ = gpu_run(L, prm)
    assert np.array_equal(e1, e2) and np.array_equal(m1, m2)  # reproducible
    prm.batch_shots = 1024
    m3, odd3, e3, _ = gpu_run(L, prm)
    assert np.array_equal(e1, e3) and np.array_equal(m1, m3)  # batch split
    # every residual syndrome is a valid closed-loop one: cube parities even
    lat = tc.make_lattice(L)
    d_e = torch.from_numpy(inputs.pack(e1).view(np.int64)).cuda()
    syn = torch.zeros_like(d_e)
    tc.syndrome(lat, d_e, syn, tc.n_words(S))
    N = L ** 3
    sy = syn.view(3, L, L, L, -1)  # [normal][z][y][x][word]
    par = torch.zeros_like(sy[0])
    for n in range(3):
        par ^= sy[n] ^ torch.roll(sy[n], shifts=-1, dims=2 - n)
    assert int(par.abs().sum()) == 0
    w_mean = e1.sum(axis=1).mean()
    announce(f"  mean residual weight {w_mean:.1f} of {3 * N}; failures {(m1 != 0).sum()}")
    # (the 48 + 1-cycle run is compared shot by shot with the oracle in
    # test_gpu_parity_configs.py)


def test_failing_regime_ler_parity():
    """Above threshold on a small lattice many shots fail, so the logical error
    rates compare non-trivially: flip + p-flip bit for bit, p-BP within 3
    sigma with diverged shots counted."""
    L, S = 4, 2048
    announce(f"failing regime flip+p-flip L={L} S={S}")
    prm = tc.make_run_params(0.06, 0.06, 10, 0, 5, FFPFF, n_shots=S, seed=5)
    m_g, odd_g, e_g, _ = gpu_run(L, prm)
    o = Oracle(L)
    m_o, odd_o, e_o = oracle_run_parallel(o, oracle_params(0.06, 0.06, 10, 0, 5, FFPFF, seed=5), S)
    assert np.array_equal(m_g, m_o) and np.array_equal(e_g, e_o)
    f = (m_g != 0).mean()
    announce(f"  flip+p-flip any-axis LER {f:.4f}")
    assert f > 0.05
    announce(f"failing regime p-BP L={L} S=1024")
    n_div, f_g, f_o, sig = _compare_bp_run(L, 1024, 0.08, 8, seed=6)
    assert f_o > 0.02
    assert abs(f_g - f_o) <= 3 * sig
    assert n_div <= 1024 // 20


def test_graph_run_equals_eager_run():
    """TC3D_RUN_GRAPH: the whole run captured into one HIP graph equals the
    eager run bit for bit, on three calls in a row with eager work of the
    program between them (flip family at L = 6, and p-BP streaming and
    resident)."""
    import torch
    for L, kw in ((6, dict(bp_iters=0, n_sweeps=5, pflip_mask=FFPFF)),
                  (6, dict(bp_iters=20, n_sweeps=6, pflip_mask=PFFPFF,
                           bp_path=tc.BP_STREAMING)),
                  (8, dict(bp_iters=20, n_sweeps=6, pflip_mask=PFFPFF))):
        for call in range(3):
            S = (700, 130, 1000)[call]
            prm = tc.make_run_params(0.04, 0.04, 4, n_shots=S, seed=30 + call, **kw)
            m_e, odd_e, e_e, _ = gpu_run(L, prm)
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work in between
            prm.flags = tc.RUN_GRAPH
            m_g, odd_g, e_g, _ = gpu_run(L, prm)
            assert float(junk) == float(junk)
            assert np.array_equal(e_g, e_e) and np.array_equal(m_g, m_e), (L, call)
            assert np.array_equal(odd_g, odd_e)
