"""Decoder variants the paper proposes without running them, on the GPU
against the oracle: the subset p-flip of Dennis et al. (Section 3.2
footnote), bit for bit as a stage and inside whole runs, and longer flip /
p-flip schedules (Section 5: a longer schedule as a likely improvement)."""
import math

import numpy as np
import pytest

import inputs
import paper_2212_06985_amd as tc
from gpu_util import announce, bits_of_dev, dev_plane_of_bits, oracle_run_parallel
from oracle.oracle import Oracle, make_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    tc.lib()
    yield
    torch.cuda.synchronize()


def sync():
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("L", [4, 6])
@pytest.mark.parametrize("cls", [0, 5, 11])
def test_subset_sweep_bit_exact(L, cls):
    announce(f"subset p-flip sweep L={L} class={cls}")
    o = Oracle(L)
    lat = tc.make_lattice(L)
    n_shots, shot0 = 150, 128
    W = inputs.n_words(n_shots)
    full = 64 * W
    for density in (0.1, 0.5):
        syn = inputs.random_bits(int(density * 100) + cls, full, o.n_faces, density)
        corr = inputs.random_bits(9 + cls, full, o.n_edges, 0.05)
        d_syn, d_corr = dev_plane_of_bits(syn), dev_plane_of_bits(corr)
        ws = tc.alloc_workspace(tc.sweep_workspace_bytes(lat, W))
        seed, cycle, sweep = 0x1234567, 9, 4
        tc.subset_pflip_sweep(lat, d_syn, d_corr, W, seed, cycle, sweep, shot0, cls, ws)
        o.subset_pflip_sweep(syn, corr, seed, cycle, sweep, cls, shot0)
        sync()
        assert np.array_equal(bits_of_dev(d_syn, full), syn), density
        assert np.array_equal(bits_of_dev(d_corr, full), corr), density


def _gpu_run(L, prm):
    import torch
    lat = tc.make_lattice(L)
    S = prm.n_shots
    err = torch.zeros((lat.n_edges, tc.n_words(S)), dtype=torch.int64, device="cuda")
    mask = torch.zeros(S, dtype=torch.uint8, device="cuda")
    odd = torch.zeros((S, 3), dtype=torch.int32, device="cuda")
    ws = tc.alloc_workspace(tc.run_workspace_bytes(lat, prm))
    tc.run_cycles(lat, prm, err, mask, odd, ws)
    sync()
    return mask.cpu().numpy(), odd.cpu().numpy(), bits_of_dev(err, S)


# (L, shots, p, noisy cycles, sweeps, p-flip mask, subset mask)
FLIP_RUNS = [
    (4, 300, 0.03, 6, 5, 0b00000, 0b00100),                 # F F C F F
    (6, 200, 0.04, 5, 6, 0b000000, 0b001001),               # C F F C F F
    (6, 130, 0.04, 4, 12, 0b001001001001, 0),               # (P F F) x 4
    (4, 200, 0.05, 5, 9, 0b000100100, 0b100000001),         # C F P F F P F F C
]


@pytest.mark.parametrize("L,S,p,noisy,ns,pmask,smask", FLIP_RUNS)
def test_variant_schedules_without_bp_bit_exact(L, S, p, noisy, ns, pmask, smask):
    announce(f"run_cycles L={L} S={S} sweeps={ns} pflip={pmask:b} subset={smask:b}")
    prm = tc.make_run_params(p, p, noisy, 0, ns, pmask, n_shots=S, seed=21, subset_mask=smask)
    m_g, odd_g, e_g = _gpu_run(L, prm)
    o = Oracle(L)
    m_o, odd_o, e_o = oracle_run_parallel(
        o, make_params(p, p, noisy, 0, ns, pmask, seed=21, subset_mask=smask), S)
    assert np.array_equal(e_g, e_o)
    assert np.array_equal(m_g, m_o) and np.array_equal(odd_g, odd_o)


def test_subset_pbp_run_matches_oracle():
    """p-BP with its p-flip sweeps replaced by subset sweeps (C F F C F F)."""
    L, S, p, noisy = 6, 256, 0.05, 5
    prm = tc.make_run_params(p, p, noisy, 20, 6, 0, n_shots=S, seed=3, subset_mask=0b001001)
    m_g, _, e_g = _gpu_run(L, prm)
    o = Oracle(L)
    m_o, _, e_o = oracle_run_parallel(o, make_params(p, p, noisy, 20, 6, 0, seed=3,
                                                     subset_mask=0b001001), S)
    same = (e_g == e_o).all(axis=1) & (m_g == m_o)
    n_div = int((~same).sum())
    f_g, f_o = (m_g != 0).mean(), (m_o != 0).mean()
    sig = math.sqrt(f_g * (1 - f_g) / S + f_o * (1 - f_o) / S)
    announce(f"  diverged shots {n_div}/{S}; LER gpu {f_g:.4f} oracle {f_o:.4f}")
    assert n_div <= max(2, S // 50)
    assert abs(f_g - f_o) <= 3 * sig + 1e-12
