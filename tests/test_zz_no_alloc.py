"""tc3d_run_cycles_noalloc (the entry point for callers that cannot allocate)
against tc3d_run_cycles, through the C ABI: bit for bit on two calls in a row,
the second on a smaller input, for the flip family, resident p-BP (L = 12) and
streaming p-BP (L = 24, where one 64-shot word fills the fixed scratch); and
the refusals beyond the scratch's size."""
import numpy as np
import pytest

import paper_2212_06985_amd as tc
from gpu_util import announce, bits_of_dev

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


def _outputs(lat, S):
    import torch
    err = torch.zeros((lat.n_edges, tc.n_words(S)), dtype=torch.int64, device="cuda")
    mask = torch.full((S,), 255, dtype=torch.uint8, device="cuda")
    odd = torch.full((S, 3), -1, dtype=torch.int32, device="cuda")
    return err, mask, odd


def _pair(L, prm):
    """(run_cycles, run_cycles_noalloc) outputs for the same parameters."""
    import torch
    lat = tc.make_lattice(L)
    S = prm.n_shots
    out = []
    for which in ("ws", "noalloc"):
        err, mask, odd = _outputs(lat, S)
        if which == "ws":
            ws = tc.alloc_workspace(tc.run_workspace_bytes(lat, prm))
            tc.run_cycles(lat, prm, err, mask, odd, ws)
        else:
            tc.run_cycles_noalloc(lat, prm, err, mask, odd)
        torch.cuda.synchronize()
        out.append((bits_of_dev(err, S), mask.cpu().numpy(), odd.cpu().numpy()))
    return out


@pytest.mark.parametrize("L,kw,sizes", [
    (6, dict(bp_iters=0, n_sweeps=5, pflip_mask=FFPFF, noisy_cycles=6), (3000, 700)),
    (12, dict(bp_iters=20, n_sweeps=6, pflip_mask=PFFPFF, noisy_cycles=4), (2048, 130)),
    (24, dict(bp_iters=20, n_sweeps=6, pflip_mask=PFFPFF, noisy_cycles=2), (200, 64)),
])
def test_noalloc_equals_run_cycles_on_two_calls(L, kw, sizes):
    for k, S in enumerate(sizes):
        announce(f"noalloc L={L} call {k + 1}: {S} shots")
        prm = tc.make_run_params(0.05, 0.05, n_shots=S, seed=11 + k, **kw)
        (e_a, m_a, o_a), (e_b, m_b, o_b) = _pair(L, prm)
        assert np.array_equal(e_a, e_b)
        assert np.array_equal(m_a, m_b) and np.array_equal(o_a, o_b)
        assert m_b.max() < 8 and o_b.min() >= 0  # every shot was written


def test_noalloc_refuses_what_does_not_fit():
    import torch
    # L = 48: one word of BP messages is 340 MB
    lat = tc.make_lattice(48)
    prm = tc.make_run_params(0.05, 0.05, 1, 20, 6, PFFPFF, n_shots=64)
    err, mask, odd = _outputs(lat, 64)
    with pytest.raises(tc.Tc3dError, match="workspace"):
        tc.run_cycles_noalloc(lat, prm, err, mask, odd)
    # a given batch larger than the scratch
    lat = tc.make_lattice(24)
    prm = tc.make_run_params(0.05, 0.05, 1, 20, 6, PFFPFF, n_shots=256, batch_shots=256)
    err, mask, odd = _outputs(lat, 256)
    with pytest.raises(tc.Tc3dError, match="workspace"):
        tc.run_cycles_noalloc(lat, prm, err, mask, odd)
    torch.cuda.synchronize()
