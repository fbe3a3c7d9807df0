"""GPU parity of BP with meta-check factors (FP64 on both sides) against the
oracle: one iteration from oracle states, whole decodes, and whole runs."""
import math

import numpy as np
import pytest

import inputs
import paper_2212_06985_amd as tc
from gpu_util import announce, bits_of_dev, dev_plane_of_bits, oracle_run_parallel
from oracle.oracle import Oracle, make_params

pytestmark = pytest.mark.gpu
# A message x is computed from a product y of tanh values with 1 - |y| of
# order 2 e^{-|x|}, so rounding in either code (a few ulps of y) moves it by
# about 1e-16 e^{|x|}; the bar allows 100 times that beside 1e-9 relative.


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


def to_gpu_state(states, L):
    """[(nu [3N][4], lambda [3N], kappa [N][6])] per shot -> FP64 e^msg
    [W][N][21][64] (padding shots: zero messages)."""
    N = L ** 3
    S = len(states)
    W = inputs.n_words(S)
    out = np.ones((W, N, 21, 64), np.float64)
    for s, (nu, lam, kap) in enumerate(states):
        w, l = divmod(s, 64)
        for n in range(3):
            out[w, :, 4 * n:4 * n + 4, l] = np.exp(nu[n * N:(n + 1) * N, :])
            out[w, :, 12 + n, l] = np.exp(lam[n * N:(n + 1) * N])
        out[w, :, 15:21, l] = np.exp(kap)
    return out


def from_gpu_state(arr, L, S):
    N = L ** 3
    res = []
    for s in range(S):
        w, l = divmod(s, 64)
        nu = np.concatenate([np.log(arr[w, :, 4 * n:4 * n + 4, l]) for n in range(3)])
        lam = np.concatenate([np.log(arr[w, :, 12 + n, l]) for n in range(3)])
        kap = np.log(arr[w, :, 15:21, l])
        res.append((nu, lam, kap))
    return res


def close(g, o):
    bound = 1e-9 * np.maximum(np.abs(o), 1.0) + 1e-14 * np.exp(np.minimum(np.abs(o), 35.0))
    return bool((np.abs(g - o) <= bound).all()), float(np.abs(g - o).max())


@pytest.mark.parametrize("L,S,iters_before", [(4, 100, 0), (4, 100, 3), (6, 64, 7)])
def test_one_iteration_matches_oracle(L, S, iters_before):
    import torch
    announce(f"meta BP step L={L} S={S} after {iters_before} iterations")
    p = q = 0.05
    o = Oracle(L)
    lat = tc.make_lattice(L)
    syn = inputs.random_bits(60 + L + iters_before, S, o.n_faces, 0.2)
    states = []
    for s in range(S):
        st = None
        for _ in range(iters_before):
            st, _ = o.bp_meta_step(syn[s], p, q, st)
        states.append(st)
    W = inputs.n_words(S)
    d_syn = dev_plane_of_bits(np.concatenate([syn, np.zeros((64 * W - S, o.n_faces), np.uint8)]))
    shape = (W, L ** 3, 21, 64)
    d_in = (torch.from_numpy(to_gpu_state(states, L)).cuda() if iters_before else None)
    d_out = torch.zeros(shape, dtype=torch.float64, device="cuda")
    d_post = torch.zeros((W, 3 * L ** 3, 64), dtype=torch.float64, device="cuda")
    tc.bp_meta_step(lat, d_syn, S, p, q, d_in, d_out, d_post)
    sync()
    got = from_gpu_state(d_out.cpu().numpy(), L, S)
    post_g = d_post.cpu().numpy()
    worst = 0.0
    for s in range(S):
        want, post_o = o.bp_meta_step(syn[s], p, q, states[s])
        for g, w_ in zip(got[s], want):
            ok, dev = close(g, w_)
            worst = max(worst, dev)
            if not ok:
                i = np.unravel_index(np.argmax(np.abs(g - w_)), g.shape)
                raise AssertionError((s, dev, float(g[i]), float(w_[i])))
        wi, l = divmod(s, 64)
        ok, dev = close(post_g[wi, :, l], post_o)
        assert ok, (s, dev)
    announce(f"  max abs deviation {worst:.2e}")


@pytest.mark.parametrize("L,S", [(4, 130), (6, 64)])
def test_decode_matches_oracle(L, S):
    import torch
    p = q = 0.05
    o = Oracle(L)
    lat = tc.make_lattice(L)
    err = inputs.random_bits(70 + L, S, o.n_edges, 0.06)
    syn = o.syndrome(err) ^ inputs.random_bits(80 + L, S, o.n_faces, 0.04)
    corr_o, post_o = o.bp_meta_decode(syn, p, q, 20)
    W = inputs.n_words(S)
    full = np.concatenate([syn, np.zeros((64 * W - S, o.n_faces), np.uint8)])
    d_syn = dev_plane_of_bits(full)
    d_corr = torch.zeros((o.n_edges, W), dtype=torch.int64, device="cuda")
    d_post = torch.zeros((W, o.n_edges, 64), dtype=torch.float64, device="cuda")
    ws = tc.alloc_workspace(tc.bp_meta_workspace_bytes(lat, S))
    tc.bp_meta_decode(lat, d_syn, S, p, q, 20, d_corr, d_post, ws)
    sync()
    corr_g = bits_of_dev(d_corr, S)
    post_g = inputs.rows_from_gpu(d_post.cpu().numpy(), o.n_edges)[:S]
    # free-running: rounding differences of saturated messages compound over
    # the iterations (the one-step test above holds each iteration to the
    # rounding bar), so the decisions must agree away from ties and the
    # posteriors to 1% of their size
    near_tie = np.abs(post_o) < 1e-3
    assert np.array_equal(corr_g[~near_tie], corr_o[~near_tie])
    dev = np.abs(post_g - post_o)
    announce(f"  L={L}: flips {int(corr_o.sum())}, near-ties {int(near_tie.sum())}, "
             f"max posterior deviation {dev.max():.2e}")
    assert (dev <= 1e-2 * np.maximum(np.abs(post_o), 1.0)).all()


def test_runs_match_oracle():
    """p-BP with meta-check BP inside whole runs: shots whose BP never met a
    near-tie agree bit for bit; the logical error rates within 3 sigma."""
    L, S, p, noisy = 6, 256, 0.06, 6
    prm = tc.make_run_params(p, p, noisy, 20, 6, 0b001001, n_shots=S, seed=13, bp_meta=1)
    import torch
    lat = tc.make_lattice(L)
    err = torch.zeros((lat.n_edges, tc.n_words(S)), dtype=torch.int64, device="cuda")
    mask = torch.zeros(S, dtype=torch.uint8, device="cuda")
    odd = torch.zeros((S, 3), dtype=torch.int32, device="cuda")
    ws = tc.alloc_workspace(tc.run_workspace_bytes(lat, prm))
    tc.run_cycles(lat, prm, err, mask, odd, ws)
    sync()
    m_g, e_g = mask.cpu().numpy(), bits_of_dev(err, S)
    o = Oracle(L)
    m_o, _, e_o = oracle_run_parallel(o, make_params(p, p, noisy, 20, 6, 0b001001, seed=13,
                                                     bp_meta=1), S)
    same = (e_g == e_o).all(axis=1) & (m_g == m_o)
    n_div = int((~same).sum())
    f_g, f_o = (m_g != 0).mean(), (m_o != 0).mean()
    sig = math.sqrt(f_g * (1 - f_g) / S + f_o * (1 - f_o) / S)
    announce(f"  diverged shots {n_div}/{S}; LER gpu {f_g:.4f} oracle {f_o:.4f}")
    assert n_div <= max(2, S // 50)
    assert abs(f_g - f_o) <= 3 * sig + 1e-12
