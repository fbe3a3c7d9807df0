"""The paper's flip-family thresholds, reproduced by the GPU path.

With the flip rule applied once per cycle (Fig. 2) the paper finds the
failure curves of different L crossing at p = q = 2.611%; with five rule
applications per cycle, every third one p-flip (Table 1, n_A = 5,
lambda_p = 3: F F P F F), at 4.445%, both after 1000 cycles. Below the
crossing a larger lattice fails less often, above it more often. The test
brackets each printed threshold by two error rates, one on either side, and
requires L = 32 to fail significantly less often than L = 14 at the lower one
and significantly more often at the upper one."""
import math

import pytest

import golden_data as gd
from gpu_util import announce
from paper_2212_06985_amd import experiments as ex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "the GPU tests need an MI355X"
    yield
    torch.cuda.synchronize()


def _rate(L, p, n_a, lam, shots):
    r = ex.memory_run(L, p, 1000, "flip", shots, seed=1, n_a=n_a, lambda_p=lam)
    return ex.pfail(r)


def _printed(n_a, lam):
    """The threshold Table 1 prints for (n_A, lambda_p) (tests/golden/)."""
    cells = {(n, l): th for n, l, th, _ in gd.table1()}
    return cells[(n_a, lam)]


@pytest.mark.parametrize("n_a,lam,p_lo,p_hi", [
    (1, 2, 0.0258, 0.0264),   # Fig. 2: flip once per cycle (the shaded n_A = 1 cell)
    (5, 3, 0.0440, 0.0450),   # Table 1: F F P F F
])
def test_threshold_is_bracketed(n_a, lam, p_lo, p_hi):
    paper = _printed(n_a, lam)
    assert p_lo < paper < p_hi
    shots = 4096
    for p, below in ((p_lo, True), (p_hi, False)):
        f14, s14 = _rate(14, p, n_a, lam, shots)
        f32, s32 = _rate(32, p, n_a, lam, shots)
        announce(f"  n_A={n_a} lambda_p={lam} p={p}: p_fail L=14 {f14:.4f}+-{s14:.4f}, "
                 f"L=32 {f32:.4f}+-{s32:.4f}")
        gap = (f14 - f32) if below else (f32 - f14)
        assert gap > 3 * math.sqrt(s14 ** 2 + s32 ** 2), (p, f14, f32)


def test_memory_run_with_the_cnn_prior_is_run_cycles_cnn():
    """The experiment runner's CNN option is tc3d_run_cycles_cnn on the same
    shots: the same network blended the same way, the same failure masks."""
    import os

    import numpy as np
    import torch

    import paper_2212_06985_amd as tc
    from paper_2212_06985_amd.train_cnn import packed_prior
    L, p, cycles, shots, beta, it = 6, 0.06, 20, 512, 0.5, 8
    w = os.path.join(os.path.dirname(tc.__file__), "weights", "cnn_L12_long.npy")
    r = ex.memory_run(L, p, cycles, "pbp", shots, seed=5, bp_iters=it, cnn_weights=w,
                      beta=beta)
    packed = packed_prior(np.load(w), beta, p)
    lat = tc.make_lattice(L)
    prm = tc.make_run_params(p, p, cycles, it, 6, 0b001001, n_shots=shots, seed=5,
                             perfect_final=0)
    err = torch.zeros((lat.n_edges, tc.n_words(shots)), dtype=torch.int64, device="cuda")
    mask = torch.zeros(shots, dtype=torch.uint8, device="cuda")
    ws = tc.alloc_workspace(tc.run_cnn_workspace_bytes(lat, prm))
    tc.run_cycles_cnn(lat, prm, packed, err, mask, None, ws)
    hist = np.bincount(mask.cpu().numpy(), minlength=8)
    announce(f"  cnn memory run L={L}: {r['hist']}")
    assert r["hist"] == hist.tolist()
    assert r["cnn_weights"] == w and r["beta"] == beta
