"""GPU parity of the CNN prior against the oracle (same BF16-rounded weights;
the GPU also stores activations and gradients in BF16, the oracle keeps
everything in FP64), its training step, and its use as the BP prior.

Outputs and gradients are compared element by element against a bound derived
from the BF16 and FP32 rounding the GPU performs (tests/cnn_bounds.py): six
standard deviations of the propagated rounding error of that element."""
import math

import numpy as np
import pytest

import cnn_bounds
import inputs
import paper_2212_06985_amd as tc
from gpu_util import announce, bits_of_dev, dev_plane_of_bits, to_dev
from oracle.oracle import CNN_CHANNELS, Oracle, cnn_layers, cnn_param_count

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


def bf16_round(x):
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32."""
    a = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32)


def random_params(seed, gain=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(cnn_param_count(), np.float32)
    for W, b in cnn_layers(p):
        fan_in = W.shape[0] * W.shape[1]
        W[...] = rng.normal(0, gain * math.sqrt(2.0 / fan_in), W.shape)
        b[...] = rng.normal(0, 0.05, b.shape)
    return p


def oracle_params(p32):
    """FP64 parameters the GPU actually uses: BF16 weights, FP32 biases."""
    out = p32.astype(np.float64).copy()
    for W, _ in cnn_layers(out):
        W[...] = bf16_round(W.astype(np.float32)).astype(np.float64)
    return out


def packed_of(p32):
    import torch
    d = to_dev(p32)
    packed = torch.zeros(tc.cnn_packed_bytes(), dtype=torch.uint8, device="cuda")
    tc.cnn_pack(d, packed)
    return d, packed


def z_from_llr(llr, L, S):
    N = L ** 3
    rows = inputs.rows_from_gpu(llr.cpu().numpy(), 3 * N)[:S]  # [S][3N], e = c*N + v
    return -rows.reshape(S, 3, N).transpose(0, 2, 1).astype(np.float64)


@pytest.mark.parametrize("L,S", [(3, 64), (4, 100), (5, 64), (6, 64), (7, 64)])
def test_forward_parity(L, S):
    import torch
    announce(f"cnn forward L={L} S={S}")
    o = Oracle(L)
    lat = tc.make_lattice(L)
    W = inputs.n_words(S)
    full = 64 * W
    syn = inputs.random_bits(20 + L, full, o.n_faces, 0.3)
    prev = inputs.random_bits(30 + L, full, o.n_faces, 0.2)
    p32 = random_params(L)
    _, packed = packed_of(p32)
    llr = torch.zeros((W, 3 * L ** 3, 64), dtype=torch.float32, device="cuda")
    ws = tc.alloc_workspace(tc.cnn_workspace_bytes(lat, S))
    tc.cnn_forward(lat, dev_plane_of_bits(syn), dev_plane_of_bits(prev), S, packed, llr, ws)
    sync()
    z_g = z_from_llr(llr, L, full)
    po = oracle_params(p32)
    x0 = o.cnn_input(syn, prev)
    z_o = o.cnn_forward(x0, po)
    assert_within_bound(z_g, z_o, x0, po, L)
    # first cycle: no previous syndrome
    tc.cnn_forward(lat, dev_plane_of_bits(syn), None, S, packed, llr, ws)
    sync()
    x0 = o.cnn_input(syn, None)
    assert_within_bound(z_from_llr(llr, L, full), o.cnn_forward(x0, po), x0, po, L)


def assert_within_bound(z_g, z_o, x0, po, L):
    """Every logit within its rounding bound (6 sigma of the propagated BF16
    and FP32 rounding of its own inputs)."""
    z_b, bound = cnn_bounds.forward_bound(x0, cnn_layers(po), L)
    assert np.abs(z_b - z_o).max() < 1e-9  # the bound's network is the oracle's
    err = np.abs(z_g - z_o)
    assert (err[bound == 0] == 0).all()
    worst = float((err / np.where(bound > 0, bound, np.inf)).max())
    announce(f"  max |gpu - oracle| {err.max():.3e}; largest error / bound {worst:.3f} "
             f"(bound {bound.min():.2e} .. {bound.max():.2e}, |z| max {np.abs(z_o).max():.2f})")
    assert worst <= 1.0


@pytest.mark.parametrize("L,S", [(7, 1024), (5, 1536)])
def test_forward_parity_multi_plane_segments(L, S):
    """Enough shots that the z-marching layers walk segments of several planes
    with a short last one (on MI355X: 4 + 3 planes at L = 7, 3 + 2 at L = 5
    for the 32 -> 32 layers; 2 + 2 + 2 + 1 and 2 + 2 + 1 for 32 -> 3), so the
    ring of accumulators carries partial sums across planes. Sampled shots
    against the oracle, at the bars of test_forward_parity."""
    import torch
    announce(f"cnn forward multi-plane L={L} S={S}")
    o = Oracle(L)
    lat = tc.make_lattice(L)
    W = inputs.n_words(S)
    full = 64 * W
    syn = inputs.random_bits(40 + L, full, o.n_faces, 0.3)
    prev = inputs.random_bits(50 + L, full, o.n_faces, 0.2)
    p32 = random_params(60 + L)
    _, packed = packed_of(p32)
    llr = torch.zeros((W, 3 * L ** 3, 64), dtype=torch.float32, device="cuda")
    ws = tc.alloc_workspace(tc.cnn_workspace_bytes(lat, S))
    tc.cnn_forward(lat, dev_plane_of_bits(syn), dev_plane_of_bits(prev), S, packed, llr, ws)
    sync()
    z_g = z_from_llr(llr, L, full)
    idx = np.array([0, 15, 16, 333, S // 2 + 7, S - 1])
    po = oracle_params(p32)
    x0 = o.cnn_input(syn[idx], prev[idx])
    assert_within_bound(z_g[idx], o.cnn_forward(x0, po), x0, po, L)


@pytest.mark.parametrize("L,S", [(3, 64), (4, 128), (5, 64)])
def test_gradient_parity(L, S):
    import torch
    announce(f"cnn gradient L={L} S={S}")
    o = Oracle(L)
    lat = tc.make_lattice(L)
    W = inputs.n_words(S)
    full = 64 * W
    syn = inputs.random_bits(40 + L, full, o.n_faces, 0.3)
    prev = inputs.random_bits(50 + L, full, o.n_faces, 0.2)
    target = inputs.random_bits(60 + L, full, o.n_edges, 0.15)
    p32 = random_params(70 + L)
    _, packed = packed_of(p32)
    llr = torch.zeros((W, 3 * L ** 3, 64), dtype=torch.float32, device="cuda")
    grad = torch.zeros(cnn_param_count(), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = tc.alloc_workspace(tc.cnn_workspace_bytes(lat, S, training=True))
    tc.cnn_loss_grad(lat, dev_plane_of_bits(syn), dev_plane_of_bits(prev),
                     dev_plane_of_bits(target), S, packed, llr, grad, loss, ws)
    sync()
    po = oracle_params(p32)
    x0 = o.cnn_input(syn, prev)
    loss_o, grad_o = o.cnn_loss_grad(x0, po, target)
    t = target.reshape(full, 3, L ** 3).transpose(0, 2, 1).astype(np.float64)
    bounds, loss_b, loss_bound = cnn_bounds.gradient_bounds(x0, cnn_layers(po), L, t,
                                                            full * L ** 3 * 3)
    assert abs(loss_b - loss_o) < 1e-9
    g = grad.cpu().numpy().astype(np.float64)
    lg = float(loss.item())
    announce(f"  loss gpu {lg:.6f} oracle {loss_o:.6f} bound {loss_bound:.2e}")
    assert abs(lg - loss_o) <= loss_bound
    for l, ((Wg, bg), (Wo, bo), (_, bw, _, bb)) in enumerate(
            zip(cnn_layers(g), cnn_layers(grad_o), bounds)):
        for name, a, b, bd in (("W", Wg, Wo, bw), ("b", bg, bo, bb)):
            err = np.abs(a - b)
            # a zero bound (the weights of the two zero input channels) asks for an exact 0
            assert (err[bd == 0] == 0).all(), (l, name)
            worst = float((err / np.where(bd > 0, bd, np.inf)).max())
            announce(f"  layer {l + 1} d{name}: max |gpu - oracle| {err.max():.2e}, largest "
                     f"error / bound {worst:.3f}")
            assert worst <= 1.0, (l, name, worst)


def test_blended_pack_parity():
    """tc3d_cnn_pack with beta < 1 packs the network whose prior is
    l0 + beta (llr_cnn - l0): the oracle's forward with the last layer scaled
    by beta and its bias set to beta b - (1 - beta) l0, at the same bar."""
    import torch
    L, S, p, beta = 5, 64, 0.06, 0.4
    o = Oracle(L)
    lat = tc.make_lattice(L)
    syn = inputs.random_bits(91, S, o.n_faces, 0.3)
    prev = inputs.random_bits(92, S, o.n_faces, 0.2)
    p32 = random_params(93)
    d = to_dev(p32)
    packed = torch.zeros(tc.cnn_packed_bytes(), dtype=torch.uint8, device="cuda")
    tc.cnn_pack(d, packed, beta=beta, p=p)
    llr = torch.zeros((1, 3 * L ** 3, 64), dtype=torch.float32, device="cuda")
    ws = tc.alloc_workspace(tc.cnn_workspace_bytes(lat, S))
    tc.cnn_forward(lat, dev_plane_of_bits(syn), dev_plane_of_bits(prev), S, packed, llr, ws)
    sync()
    l0 = math.log((1 - p) / p)
    blended = p32.astype(np.float64).copy()
    W4, b4 = cnn_layers(blended)[3]
    W4 *= np.float32(beta)
    b4[...] = beta * b4 - (1 - beta) * l0
    po = blended.copy()
    for W, _ in cnn_layers(po):
        W[...] = bf16_round(W.astype(np.float32)).astype(np.float64)
    x0 = o.cnn_input(syn, prev)
    assert_within_bound(z_from_llr(llr, L, S), o.cnn_forward(x0, po), x0, po, L)


def test_apply_correction():
    """tc3d_apply_correction: err ^= corr over every row and word."""
    import torch
    L, S = 5, 200
    lat = tc.make_lattice(L)
    a = inputs.random_bits(71, S, lat.n_edges, 0.3)
    b = inputs.random_bits(72, S, lat.n_edges, 0.4)
    da, db = dev_plane_of_bits(a), dev_plane_of_bits(b)
    tc.apply_correction(lat, da, db, tc.n_words(S))
    sync()
    assert np.array_equal(bits_of_dev(da, S), a ^ b)


def test_training_lowers_the_loss():
    import torch
    L, S = 4, 256
    o = Oracle(L)
    lat = tc.make_lattice(L)
    W = inputs.n_words(S)
    # target: the error bits; inputs: their syndrome, so the task is learnable
    err = inputs.random_bits(80, S, o.n_edges, 0.05)
    syn = o.syndrome(err)
    d_syn, d_err = dev_plane_of_bits(syn), dev_plane_of_bits(err)
    p32 = random_params(81, gain=0.5)
    params, packed = packed_of(p32)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    llr = torch.zeros((W, 3 * L ** 3, 64), dtype=torch.float32, device="cuda")
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = tc.alloc_workspace(tc.cnn_workspace_bytes(lat, S, training=True))
    hist = []
    for step in range(1, 61):
        tc.cnn_loss_grad(lat, d_syn, None, d_err, S, packed, llr, grad, loss, ws)
        hist.append(float(loss.item()))
        tc.cnn_adam(params, grad, m, v, step, 3e-3, packed)
    sync()
    announce(f"  loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    assert hist[-1] < 0.5 * hist[0]
    assert np.all(np.isfinite(params.cpu().numpy()))


def _run(L, prm, packed=None):
    import torch
    lat = tc.make_lattice(L)
    S = prm.n_shots
    err = torch.zeros((lat.n_edges, tc.n_words(S)), dtype=torch.int64, device="cuda")
    mask = torch.zeros(S, dtype=torch.uint8, device="cuda")
    odd = torch.zeros((S, 3), dtype=torch.int32, device="cuda")
    if packed is None:
        ws = tc.alloc_workspace(tc.run_workspace_bytes(lat, prm))
        tc.run_cycles(lat, prm, err, mask, odd, ws)
    else:
        ws = tc.alloc_workspace(tc.run_cnn_workspace_bytes(lat, prm))
        tc.run_cycles_cnn(lat, prm, packed, err, mask, odd, ws)
    sync()
    return mask.cpu().numpy(), bits_of_dev(err, S)


def test_constant_cnn_prior_reproduces_the_paper_decoder():
    """All weights zero and output bias -l0: every prior is l0 = ln((1-p)/p)
    and the CNN-prior run is the paper's p-BP up to FP32 rounding."""
    L, S, p = 6, 256, 0.05
    l0 = math.log((1 - p) / p)
    p32 = np.zeros(cnn_param_count(), np.float32)
    cnn_layers(p32)[3][1][:] = -l0
    _, packed = packed_of(p32)
    prm = tc.make_run_params(p, p, 4, 20, 6, 0b001001, n_shots=S, seed=9)
    m_a, e_a = _run(L, prm)
    m_b, e_b = _run(L, prm, packed)
    same = ((e_a == e_b).all(axis=1) & (m_a == m_b)).sum()
    announce(f"  identical shots {same}/{S}")
    assert same >= S - 3


def test_cnn_run_equals_composed_stages():
    """tc3d_run_cycles_cnn equals the same cycle composed from the stage
    entry points: noise, syndrome, CNN (with the previous working syndrome),
    BP from the CNN priors, sweeps, carry."""
    import torch
    L, S, p, cycles, seed = 5, 128, 0.05, 3, 21
    lat = tc.make_lattice(L)
    W = tc.n_words(S)
    p32 = random_params(22, gain=0.5)
    _, packed = packed_of(p32)
    prm = tc.make_run_params(p, p, cycles, 10, 6, 0b001001, n_shots=S, seed=seed,
                             perfect_final=0)
    m_run, e_run = _run(L, prm, packed)
    n = lat.n_edges
    err = torch.zeros((n, W), dtype=torch.int64, device="cuda")
    prev = None
    llr = torch.zeros((W, n, 64), dtype=torch.float32, device="cuda")
    cws = tc.alloc_workspace(tc.cnn_workspace_bytes(lat, S))
    bws = tc.alloc_workspace(tc.bp_workspace_bytes(lat, S))
    sws = tc.alloc_workspace(tc.sweep_workspace_bytes(lat, W))
    for t in range(cycles):
        tc.sample_noise(lat, err, 0, p, seed, t, 0, S)
        syn = torch.zeros_like(err)
        tc.syndrome(lat, err, syn, W)
        tc.sample_noise(lat, syn, 1, p, seed, t, 0, S)
        tc.cnn_forward(lat, syn, prev, S, packed, llr, cws)
        corr = torch.zeros_like(err)
        tc.bp_decode(lat, syn, S, llr, 0.0, 1 - 2 * p, 10, corr, None, bws)
        tc.syndrome(lat, corr, syn, W, xor_into=True)
        for k in range(6):
            if (0b001001 >> k) & 1:
                tc.pflip_sweep(lat, syn, corr, W, seed, t, k, 0, sws)
            else:
                tc.flip_sweep(lat, syn, corr, W, sws)
        prev = syn.clone()
        err ^= corr
    sync()
    assert np.array_equal(bits_of_dev(err, S), e_run)


def test_trained_prior_lowers_the_logical_error_rate():
    """The committed network (trained by paper_2212_06985_amd.train_cnn at
    L = 12 on 3x10^7 simulated snapshots with p = q drawn from [4.5%, 7%]),
    blended with the channel prior at beta = 0.3, decodes better than the
    paper's p-BP on the same shots: L = 12, p = q = 0.065, 40 noisy cycles + 1
    perfect, 32768 shots."""
    import os
    from paper_2212_06985_amd import eval_cnn
    path = os.path.join(os.path.dirname(tc.__file__), "weights", "cnn_L12_mixed.npy")
    w = np.load(path, allow_pickle=False)
    assert w.shape == (cnn_param_count(),)
    base = eval_cnn.run(12, 32768, 0.065, 40, None, seed=777)
    cnn = eval_cnn.run(12, 32768, 0.065, 40, w, seed=777, beta=0.3)
    announce(f"  plain LER {base['ler_any']:.4f} residual syndrome {base['mean_residual_syndrome']:.2f}; "
             f"CNN LER {cnn['ler_any']:.4f} residual syndrome {cnn['mean_residual_syndrome']:.2f}")
    sig = math.sqrt(base["ler_any_sigma"] ** 2 + cnn["ler_any_sigma"] ** 2)
    assert base["ler_any"] - cnn["ler_any"] > 3 * sig
    assert cnn["mean_residual_syndrome"] < base["mean_residual_syndrome"]


def _roll_sites(a, L, t, site_axis):
    """Translate the sites of a per-site array by t = (tx, ty, tz): the value
    at v moves to v + t (periodic). `site_axis` holds 3 L^3 rows, class-major
    (row c L^3 + v, v = x + L y + L^2 z)."""
    shape = a.shape[:site_axis] + (3, L, L, L) + a.shape[site_axis + 1:]
    b = a.reshape(shape)
    tx, ty, tz = t
    b = np.roll(b, (tz, ty, tx), axis=(site_axis + 1, site_axis + 2, site_axis + 3))
    return b.reshape(a.shape)


@pytest.mark.parametrize("L,S", [(24, 1024), (25, 256)])
def test_forward_translation_equivariance_full_size(L, S):
    """The network commutes with lattice translations, and the kernels compute
    every site with the same operations in the same order, whatever its place
    in a wavefront's tile or a pass: translating the syndromes translates the
    priors bit for bit, at the workload's lattice size (L = 25: ragged tiles)."""
    import torch
    announce(f"cnn forward translation L={L} S={S}")
    lat = tc.make_lattice(L)
    W = inputs.n_words(S)
    full = 64 * W
    n = 3 * L ** 3
    syn = inputs.random_bits(5 + L, full, n, 0.1)
    prev = inputs.random_bits(6 + L, full, n, 0.05)
    _, packed = packed_of(random_params(7 + L))
    ws = tc.alloc_workspace(tc.cnn_workspace_bytes(lat, S))
    t = (1, 2, 5)
    outs = []
    for a, b in ((syn, prev), (_roll_sites(syn, L, t, 1), _roll_sites(prev, L, t, 1))):
        llr = torch.zeros((W, n, 64), dtype=torch.float32, device="cuda")
        tc.cnn_forward(lat, dev_plane_of_bits(a), dev_plane_of_bits(b), S, packed, llr, ws)
        sync()
        outs.append(llr.cpu().numpy())
    assert np.array_equal(_roll_sites(outs[0], L, t, 1), outs[1])


def test_folded_bp_translation_equivariance_full_size():
    """A whole decode with per-edge priors (folded into the state) commutes
    with lattice translations bit for bit at L = 24: every site runs the same
    arithmetic whatever the traversal order."""
    import torch
    L, S, iters = 24, 2048, 6
    announce(f"folded bp translation L={L} S={S}")
    lat = tc.make_lattice(L)
    W = inputs.n_words(S)
    n = 3 * L ** 3
    syn = inputs.random_bits(11, S, n, 0.05)
    llr = inputs.random_llr(12, S, n, 0.5, 5.0).astype(np.float32)
    ws = tc.alloc_workspace(tc.bp_workspace_bytes(lat, S))
    t = (3, 1, 2)
    posts, corrs = [], []
    for a, l0 in ((syn, llr), (_roll_sites(syn, L, t, 1), _roll_sites(llr, L, t, 1))):
        post = torch.zeros((W, n, 64), dtype=torch.float32, device="cuda")
        corr = torch.zeros((n, W), dtype=torch.int64, device="cuda")
        tc.bp_decode(lat, dev_plane_of_bits(a), S, to_dev(inputs.rows_to_gpu(l0)), 0.0,
                     1 - 2 * 0.05, iters, corr, post, ws)
        sync()
        posts.append(post.cpu().numpy())
        corrs.append(bits_of_dev(corr, S))
    assert np.array_equal(_roll_sites(posts[0], L, t, 1), posts[1])
    assert np.array_equal(_roll_sites(corrs[0], L, t, 1), corrs[1])


def test_resumed_cnn_run_equals_unsplit_run():
    """Checkpoint / resume with the CNN prior: the network's input at the
    first cycle of a resumed call is the working syndrome the previous cycle
    ended with, H e of the residual plus that cycle's check-outcome noise, so
    a run split after cycle k and resumed with cycle0 = k equals the unsplit
    run bit for bit."""
    import torch
    L, S, p = 6, 128, 0.05
    _, packed = packed_of(random_params(33, gain=0.5))
    lat = tc.make_lattice(L)
    full = tc.make_run_params(p, p, 5, 8, 6, 0b001001, n_shots=S, seed=4)
    m_full, e_full = _run(L, full, packed)
    for k in (1, 2):
        head = tc.make_run_params(p, p, k, 8, 6, 0b001001, n_shots=S, seed=4, perfect_final=0)
        _, e_k = _run(L, head, packed)
        tail = tc.make_run_params(p, p, 5 - k, 8, 6, 0b001001, n_shots=S, seed=4, cycle0=k)
        err = dev_plane_of_bits(e_k)
        mask = torch.zeros(S, dtype=torch.uint8, device="cuda")
        ws = tc.alloc_workspace(tc.run_cnn_workspace_bytes(lat, tail))
        tc.run_cycles_cnn(lat, tail, packed, err, mask, None, ws)
        sync()
        assert np.array_equal(bits_of_dev(err, S), e_full), k
        assert np.array_equal(mask.cpu().numpy(), m_full), k
