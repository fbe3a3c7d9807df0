"""Batched jobs and autotuning on the GPU: a batch of mixed experiments run
by tc3d_run_jobs (sequential, concurrent streams, one captured graph, both)
equals every job run alone by tc3d_run_cycles bit for bit, and every setting
the autotuner may pick decodes identically."""
import numpy as np
import pytest

import paper_2212_06985_amd as tc
from gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    tc.lib()
    yield
    torch.cuda.synchronize()


# (L, p, noisy cycles, bp iterations, sweeps, p-flip mask, shots, seed, shot0)
JOBS = [
    (3, 0.05, 3, 20, 6, 0b001001, 100, 1, 0),
    (4, 0.03, 5, 0, 5, 0b00100, 64, 2, 0),
    (6, 0.06, 4, 10, 6, 0b001001, 200, 3, 64),
    (5, 0.04, 2, 20, 6, 0b001001, 1, 4, 128),
    (8, 0.05, 8, 20, 6, 0b001001, 130, 5, 0),
    (6, 0.02, 6, 0, 1, 0, 64, 6, 0),
]


def _buffers(L, shots):
    import torch
    n = 3 * L ** 3
    return (torch.zeros((n, tc.n_words(shots)), dtype=torch.int64, device="cuda"),
            torch.zeros(shots, dtype=torch.uint8, device="cuda"),
            torch.zeros((shots, 3), dtype=torch.int32, device="cuda"))


def _params(j):
    L, p, cyc, it, ns, mask, shots, seed, shot0 = j
    return tc.make_run_params(p, p, cyc, it, ns, mask, n_shots=shots, seed=seed, shot0=shot0)


def _alone():
    import torch
    out = []
    for j in JOBS:
        L = j[0]
        prm = _params(j)
        e, m, o = _buffers(L, j[6])
        ws = tc.alloc_workspace(tc.run_workspace_bytes(tc.make_lattice(L), prm))
        tc.run_cycles(tc.make_lattice(L), prm, e, m, o, ws)
        torch.cuda.synchronize()
        out.append((e.cpu().numpy(), m.cpu().numpy(), o.cpu().numpy()))
    return out


@pytest.mark.parametrize("flags", [0, tc.JOBS_CONCURRENT, tc.JOBS_GRAPH,
                                   tc.JOBS_CONCURRENT | tc.JOBS_GRAPH])
def test_jobs_equal_single_runs(flags):
    import torch
    announce(f"run_jobs flags={flags} with {len(JOBS)} mixed jobs")
    ref = _alone()
    bufs = [_buffers(j[0], j[6]) for j in JOBS]
    jobs = [tc.make_job(j[0], _params(j), *b) for j, b in zip(JOBS, bufs)]
    ws = tc.alloc_workspace(tc.run_jobs_workspace_bytes(jobs))
    # three calls in a row (a fresh graph each time when captured), with eager
    # work of the program in between; every call must reproduce the single runs
    for rep in range(3):
        for e, m, o in bufs:
            e.zero_()
            m.fill_(255)
            o.fill_(-1)
        tc.run_jobs(jobs, ws, flags)
        torch.cuda.synchronize()
        for (e, m, o), (re_, rm, ro), j in zip(bufs, ref, JOBS):
            assert np.array_equal(e.cpu().numpy(), re_), (rep, j)
            assert np.array_equal(m.cpu().numpy(), rm), (rep, j)
            assert np.array_equal(o.cpu().numpy(), ro), (rep, j)
        _ = torch.ones(1 << 20, device="cuda").sum().item()  # unrelated eager work


@pytest.mark.parametrize("L,S", [(12, 512), (16, 256)])
def test_autotune_choices_decode_identically(L, S):
    """Every candidate the tuner tried (BP schedule, traversal tile,
    occupancy, batch) decodes the run bit for bit like the others, and the
    choice written back is one of them."""
    import torch
    lat = tc.make_lattice(L)
    prm = tc.make_run_params(0.05, 0.05, 4, 20, 6, 0b001001, n_shots=S, seed=11)
    ws = tc.alloc_workspace(tc.autotune_workspace_bytes(lat, prm))
    tried = tc.autotune(lat, prm, ws, probe_cycles=1)
    announce(f"  autotune L={L} tried {len(tried)}: " + ", ".join(
        f"path {c['bp_path']} tile {c['bp_tile']} occ {c['bp_occupancy']} batch "
        f"{c['batch_shots']}: {c['ms']:.2f} ms" for c in tried))
    assert len(tried) >= 4
    keys = ("bp_path", "bp_tile", "bp_occupancy")
    chosen = tuple(getattr(prm, k) for k in keys)
    assert chosen in [tuple(c[k] for k in keys) for c in tried]
    if L == 16:  # beyond the resident decode: tiles and occupancies were tried
        assert len({c["bp_tile"] for c in tried}) > 3
        assert len({c["bp_occupancy"] for c in tried}) > 3
    else:
        assert {c["bp_path"] for c in tried} == {tc.BP_AUTO, tc.BP_STREAMING}
    results = []
    for c in tried:
        p2 = tc.make_run_params(0.05, 0.05, 4, 20, 6, 0b001001, n_shots=S, seed=11,
                                **{k: c[k] for k in keys + ("batch_shots",)})
        e, m, o = _buffers(L, S)
        w2 = tc.alloc_workspace(tc.run_workspace_bytes(lat, p2))
        tc.run_cycles(lat, p2, e, m, o, w2)
        torch.cuda.synchronize()
        results.append((e.cpu().numpy(), m.cpu().numpy()))
    for e, m in results[1:]:
        assert np.array_equal(e, results[0][0])
        assert np.array_equal(m, results[0][1])
