"""GPU parity, stage by stage: every entry point of the C ABI against the oracle
on the same seeded inputs. Bit planes must match bit for bit (padding shots of
the last word included: they are ordinary shots of the counter layout); BP
messages must match one step at a time within the FP32 tolerance."""
import math

import numpy as np
import pytest

import inputs
import paper_2212_06985_amd as tc
from gpu_util import (BP_FLOOR, BP_REL, LLR_TIE, announce, bits_of_dev, dev_plane_of_bits,
                      plane_from_dev, to_dev, within_bp_tol)
from oracle.oracle import Oracle

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


# ----------------------------------------------------------------- noise
@pytest.mark.parametrize("L", [3, 5, 6])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("n_shots,shot0", [(1, 0), (150, 128), (64, 64)])
def test_noise_bit_exact(L, kind, n_shots, shot0):
    announce(f"noise L={L} kind={kind} S={n_shots} shot0={shot0}")
    o = Oracle(L)
    lat = tc.make_lattice(L)
    W = inputs.n_words(n_shots)
    full = 64 * W
    for prob, seed, cycle in [(0.02, 1, 0), (0.05, 0x1234_5678_9ABC, 7), (0.3, 99, 3)]:
        init = inputs.random_bits(seed % 1000, full, o.n_edges, 0.5)
        ref = init.copy()
        o.sample_noise(ref, kind, prob, seed, cycle, shot0)
        dev = dev_plane_of_bits(init)
        tc.sample_noise(lat, dev, kind, prob, seed, cycle, shot0, n_shots)
        sync()
        assert np.array_equal(bits_of_dev(dev, full), ref), (prob, seed, cycle)


def test_noise_probability_zero_and_one():
    L = 4
    lat = tc.make_lattice(L)
    o = Oracle(L)
    init = inputs.random_bits(3, 128, o.n_edges, 0.5)
    dev = dev_plane_of_bits(init)
    tc.sample_noise(lat, dev, 0, 0.0, 1, 0, 0, 128)
    sync()
    assert np.array_equal(bits_of_dev(dev, 128), init)
    tc.sample_noise(lat, dev, 0, 1.0, 1, 0, 0, 128)  # threshold 2^32-1: all but 1 in 2^32
    ref = init.copy()
    o.sample_noise(ref, 0, 1.0, 1, 0, 0)
    sync()
    assert np.array_equal(bits_of_dev(dev, 128), ref)


# -------------------------------------------------------------- syndrome
@pytest.mark.parametrize("L", [3, 5, 6, 12])
@pytest.mark.parametrize("n_shots", [1, 100, 256])
def test_syndrome_bit_exact(L, n_shots):
    announce(f"syndrome L={L} S={n_shots}")
    o = Oracle(L)
    lat = tc.make_lattice(L)
    W = inputs.n_words(n_shots)
    full = 64 * W
    err = inputs.random_bits(L, full, o.n_edges, 0.1)
    s0 = inputs.random_bits(L + 1, full, o.n_faces, 0.5)
    ref = o.syndrome(err)
    d_err = dev_plane_of_bits(err)
    d_syn = dev_plane_of_bits(s0)
    tc.syndrome(lat, d_err, d_syn, W)
    sync()
    assert np.array_equal(bits_of_dev(d_syn, full), ref)
    # xor_into mode
    d_syn2 = dev_plane_of_bits(s0)
    tc.syndrome(lat, d_err, d_syn2, W, xor_into=True)
    sync()
    assert np.array_equal(bits_of_dev(d_syn2, full), ref ^ s0)


# ---------------------------------------------------------- flip / p-flip
@pytest.mark.parametrize("L", [3, 5, 6, 12])
@pytest.mark.parametrize("pflip", [False, True])
def test_sweeps_bit_exact(L, pflip):
    announce(f"sweep L={L} pflip={pflip}")
    o = Oracle(L)
    lat = tc.make_lattice(L)
    n_shots, shot0 = 150, 192
    W = inputs.n_words(n_shots)
    full = 64 * W
    for density in (0.08, 0.3, 0.5):
        syn = inputs.random_bits(int(density * 100) + L, full, o.n_faces, density)
        corr = inputs.random_bits(7 + L, full, o.n_edges, 0.05)
        d_syn, d_corr = dev_plane_of_bits(syn), dev_plane_of_bits(corr)
        ws = tc.alloc_workspace(tc.sweep_workspace_bytes(lat, W))
        seed, cycle, sweep = 0xABCDEF, 5, 3
        if pflip:
            tc.pflip_sweep(lat, d_syn, d_corr, W, seed, cycle, sweep, shot0, ws)
            o.pflip_sweep(syn, corr, seed, cycle, sweep, shot0)
        else:
            tc.flip_sweep(lat, d_syn, d_corr, W, ws)
            o.flip_sweep(syn, corr)
        sync()
        assert np.array_equal(bits_of_dev(d_syn, full), syn), density
        assert np.array_equal(bits_of_dev(d_corr, full), corr), density


def test_pflip_clears_corner_at_the_enumerated_rate():
    """The corner half-star of Fig. 3(a), decoded by P then F on many shots:
    the cleared fraction matches the exhaustive 44/64 within 4 sigma."""
    import geom
    L = 6
    o = Oracle(L)
    lat = tc.make_lattice(L)
    st = geom.star(L, 2, 2, 2)
    e0 = geom.bits_of(o.n_edges, [st[0], st[2], st[4]])
    S = 64 * 64
    err = np.tile(e0, (S, 1))
    d_err = dev_plane_of_bits(err)
    W = S // 64
    d_syn = dev_plane_of_bits(np.zeros((S, o.n_faces), np.uint8))
    d_corr = dev_plane_of_bits(np.zeros((S, o.n_edges), np.uint8))
    ws = tc.alloc_workspace(tc.sweep_workspace_bytes(lat, W))
    tc.syndrome(lat, d_err, d_syn, W)
    tc.pflip_sweep(lat, d_syn, d_corr, W, 1, 0, 0, 0, ws)
    tc.flip_sweep(lat, d_syn, d_corr, W, ws)
    res = err ^ bits_of_dev(d_corr, S)
    syn = bits_of_dev(d_syn, S)
    _, odd = o.logical_check(res)
    cleared = (syn.sum(axis=1) == 0) & (odd.sum(axis=1) == 0)
    frac = cleared.mean()
    sigma = math.sqrt(44 / 64 * 20 / 64 / S)
    assert abs(frac - 44 / 64) < 4 * sigma, frac


def test_flip_examples_of_the_paper():
    """The worked examples of Figs. 3-5 and Section 3.2 (tests/golden/
    flip_examples.txt), one per shot of one batch, through the GPU syndrome,
    two parallel flip sweeps and the readout: the unsatisfied-check counts,
    the errors after each sweep and the cleared cases are those the paper
    states."""
    import torch
    import golden_data as gd
    L = gd.EXAMPLE_L
    examples = gd.flip_examples()
    names = sorted(examples)
    announce(f"flip examples L={L}: {' '.join(names)}")
    lat = tc.make_lattice(L)
    n_edges, n_faces = 3 * L ** 3, 3 * L ** 3
    S = len(names)
    err = np.zeros((64, n_edges), np.uint8)
    for s, name in enumerate(names):
        err[s, sorted(examples[name]["support"])] = 1
    d_err = dev_plane_of_bits(err)
    d_syn = dev_plane_of_bits(np.zeros((64, n_faces), np.uint8))
    d_corr = dev_plane_of_bits(np.zeros((64, n_edges), np.uint8))
    ws = tc.alloc_workspace(tc.sweep_workspace_bytes(lat, 1))
    tc.syndrome(lat, d_err, d_syn, 1)
    sync()
    unsat = bits_of_dev(d_syn, 64).sum(axis=1)
    for s, name in enumerate(names):
        if "unsat" in examples[name]:
            assert unsat[s] == examples[name]["unsat"], name
    for key in ("after1", "after2"):
        tc.flip_sweep(lat, d_syn, d_corr, 1, ws)
        sync()
        res = err ^ bits_of_dev(d_corr, 64)
        for s, name in enumerate(names):
            if key in examples[name]:
                assert set(np.flatnonzero(res[s])) == examples[name][key], (name, key)
        if key == "after1":
            # the working syndrome is that of the residual error
            d_res = dev_plane_of_bits(res)
            d_chk = dev_plane_of_bits(np.zeros((64, n_faces), np.uint8))
            tc.syndrome(lat, d_res, d_chk, 1)
            mask = torch.zeros(S, dtype=torch.uint8, device="cuda")
            odd = torch.zeros((S, 3), dtype=torch.int32, device="cuda")
            tc.logical_check(lat, d_res, S, mask, odd)
            sync()
            syn1 = bits_of_dev(d_syn, 64)
            assert np.array_equal(syn1, bits_of_dev(d_chk, 64))
            odd = odd.cpu().numpy()
            for s, name in enumerate(names):
                if examples[name].get("cleared"):
                    assert syn1[s].sum() == 0 and odd[s].sum() == 0, name
    # padding shots stay empty
    assert not res[S:].any()


# ---------------------------------------------------------------- readout
@pytest.mark.parametrize("L", [3, 4, 6, 12])
@pytest.mark.parametrize("n_shots", [1, 77, 200])
def test_logical_check_bit_exact(L, n_shots):
    announce(f"readout L={L} S={n_shots}")
    import geom
    o = Oracle(L)
    lat = tc.make_lattice(L)
    err = inputs.random_bits(100 + L, n_shots, o.n_edges, 0.03)
    rng = np.random.default_rng(L)
    for s in range(0, n_shots, 3):  # plant logical membranes on some shots
        a = rng.integers(0, 3)
        err[s] ^= geom.bits_of(o.n_edges, geom.membrane(L, a, rng.integers(0, L)))
    mask_o, odd_o = o.logical_check(err)
    import torch
    d_err = dev_plane_of_bits(err)
    mask = torch.zeros(n_shots, dtype=torch.uint8, device="cuda")
    odd = torch.zeros((n_shots, 3), dtype=torch.int32, device="cuda")
    tc.logical_check(lat, d_err, n_shots, mask, odd)
    sync()
    assert np.array_equal(mask.cpu().numpy(), mask_o)
    assert np.array_equal(odd.cpu().numpy(), odd_o)


# --------------------------------------------------------------------- BP
def _bp_inputs(L, n_shots, seed):
    o = Oracle(L)
    W = inputs.n_words(n_shots)
    full = 64 * W
    err = inputs.random_bits(seed, full, o.n_edges, 0.05)
    syn = o.syndrome(err) ^ inputs.random_bits(seed + 1, full, o.n_faces, 0.05)
    return o, syn, W, full


@pytest.mark.parametrize("L,n_shots", [(3, 64), (5, 100), (6, 130)])
@pytest.mark.parametrize("per_edge_prior", [False, True])
def test_bp_one_step_parity(L, n_shots, per_edge_prior):
    """Each GPU iteration, recomputed by the oracle in FP64 from the GPU's own
    previous state, agrees within 1e-4 relative (absolute below 0.1). The GPU
    keeps messages as e^nu; they are compared as nu = ln(e^nu)."""
    announce(f"bp one-step L={L} S={n_shots} llr0={per_edge_prior}")
    import torch
    p = q = 0.05
    o, syn, W, full = _bp_inputs(L, n_shots, 17 + L)
    lat = tc.make_lattice(L)
    N = L ** 3
    d_syn = dev_plane_of_bits(syn)
    l0 = math.log((1 - p) / p)
    K = 1 - 2 * q
    llr_f32 = None
    d_llr = None
    if per_edge_prior:
        llr_f32 = inputs.random_llr(L, full, o.n_edges, 0.5, 5.0).astype(np.float32)
        d_llr = to_dev(inputs.rows_to_gpu(llr_f32))  # [W][3N][64]
    nu = [torch.zeros((W, N, 12, 64), dtype=torch.float32, device="cuda") for _ in range(2)]
    post = torch.zeros((W, 3 * N, 64), dtype=torch.float32, device="cuda")
    prev = None
    worst = 0.0
    for t in range(20):
        out = nu[t % 2]
        tc.bp_step(lat, d_syn, n_shots, d_llr, l0, K, prev, out, post)
        sync()
        # the GPU state is e^nu (multiplicative form); the oracle works on nu
        g_nu = np.log(inputs.nu_from_gpu(out.cpu().numpy(), L, full))
        g_post = inputs.rows_from_gpu(post.cpu().numpy(), 3 * N).astype(np.float64)
        g_prev = None if prev is None else np.log(inputs.nu_from_gpu(prev.cpu().numpy(), L,
                                                                     full))
        for s in range(full):
            o_nu, o_post = o.bp_step(
                syn[s], p, q, nu_in=None if g_prev is None else g_prev[s],
                llr0=None if llr_f32 is None else llr_f32[s].astype(np.float64))
            ok, rel, ab = within_bp_tol(g_nu[s], o_nu)
            assert ok, (t, s, rel, ab)
            # posterior from the GPU's new messages
            o_post2 = (llr_f32[s].astype(np.float64) if llr_f32 is not None else l0) + \
                _posterior_sum(o, g_nu[s])
            ok, rel, ab = within_bp_tol(g_post[s], o_post2)
            assert ok, ("post", t, s, rel, ab)
            worst = max(worst, rel)
        prev = out
    announce(f"  max relative deviation over 20 iterations: {worst:.3e}")


_INC = {}


def _posterior_sum(o, nu):
    """sum of the 4 incoming messages of every edge (E4 without the prior)."""
    key = o.L
    if key not in _INC:
        _INC[key] = o.incidence()
    _, ef, es = _INC[key]
    return nu[ef, es].sum(axis=1)


@pytest.mark.parametrize("L,n_shots", [(5, 100), (6, 256), (12, 64)])
def test_bp_decode_free_running(L, n_shots):
    """bp_decode (20 iterations, first iteration implied by the syndrome)
    against the oracle's free-running FP64 BP: hard decisions agree except on
    posteriors within 1e-3 of zero; the trajectory deviation is reported."""
    announce(f"bp decode L={L} S={n_shots}")
    import torch
    p = q = 0.05
    o, syn, W, full = _bp_inputs(L, n_shots, 31 + L)
    lat = tc.make_lattice(L)
    N = L ** 3
    d_syn = dev_plane_of_bits(syn)
    corr = torch.zeros((3 * N, W), dtype=torch.int64, device="cuda")
    post = torch.zeros((W, 3 * N, 64), dtype=torch.float32, device="cuda")
    ws = tc.alloc_workspace(tc.bp_workspace_bytes(lat, n_shots))
    tc.bp_decode(lat, d_syn, n_shots, None, math.log((1 - p) / p), 1 - 2 * q, 20, corr, post, ws)
    sync()
    c_o, p_o = o.bp_decode(syn[:n_shots], p, q, 20)
    c_g = bits_of_dev(corr, n_shots)
    p_g = inputs.rows_from_gpu(post.cpu().numpy(), 3 * N)[:n_shots].astype(np.float64)
    mism = c_g != c_o
    dev = np.abs(p_g - p_o)
    announce(f"  hard-decision mismatches {int(mism.sum())}, near-tie oracle posteriors "
             f"{int((np.abs(p_o) < LLR_TIE).sum())}, max |post dev| {dev.max():.3e}")
    assert (np.abs(p_o[mism]) < LLR_TIE).all(), np.abs(p_o[mism]).max()
    # one-iteration path (no stored messages at all)
    corr1 = torch.zeros_like(corr)
    tc.bp_decode(lat, d_syn, n_shots, None, math.log((1 - p) / p), 1 - 2 * q, 1, corr1, None, ws)
    sync()
    c1, _ = o.bp_decode(syn[:n_shots], p, q, 1)
    assert np.array_equal(bits_of_dev(corr1, n_shots), c1)


def test_bp_decode_matches_chained_steps():
    """bp_decode's stored-message-free first iteration and bp_step's explicit
    one give the same final posteriors to FP32 rounding."""
    import torch
    L, n_shots = 6, 64
    p = q = 0.05
    o, syn, W, full = _bp_inputs(L, n_shots, 5)
    lat = tc.make_lattice(L)
    N = L ** 3
    d_syn = dev_plane_of_bits(syn)
    l0, K = math.log((1 - p) / p), 1 - 2 * q
    post_a = torch.zeros((W, 3 * N, 64), dtype=torch.float32, device="cuda")
    corr = torch.zeros((3 * N, W), dtype=torch.int64, device="cuda")
    ws = tc.alloc_workspace(tc.bp_workspace_bytes(lat, n_shots))
    tc.bp_decode(lat, d_syn, n_shots, None, l0, K, 5, corr, post_a, ws)
    nu = [torch.zeros((W, N, 12, 64), dtype=torch.float32, device="cuda") for _ in range(2)]
    post_b = torch.zeros_like(post_a)
    prev = None
    for t in range(5):
        tc.bp_step(lat, d_syn, n_shots, None, l0, K, prev, nu[t % 2], post_b)
        prev = nu[t % 2]
    sync()
    a, b = post_a.cpu().numpy(), post_b.cpu().numpy()
    assert np.allclose(a, b, rtol=1e-5, atol=1e-5), np.abs(a - b).max()


@pytest.mark.parametrize("L,n_shots", [(5, 100), (6, 256)])
def test_bp_decode_per_edge_prior(L, n_shots):
    """A whole decode with per-edge priors keeps each edge's prior folded into
    one stored message; its posteriors equal those of chained bp_step calls
    (plain state) to FP32 rounding, and its hard decisions equal the oracle's
    free-running FP64 decode except on posteriors within 1e-3 of zero."""
    announce(f"bp decode per-edge prior L={L} S={n_shots}")
    import torch
    p = q = 0.05
    o, syn, W, full = _bp_inputs(L, n_shots, 41 + L)
    lat = tc.make_lattice(L)
    N = L ** 3
    d_syn = dev_plane_of_bits(syn)
    K = 1 - 2 * q
    llr_f32 = inputs.random_llr(L, full, o.n_edges, 0.5, 5.0).astype(np.float32)
    d_llr = to_dev(inputs.rows_to_gpu(llr_f32))
    iters = 12
    post_a = torch.zeros((W, 3 * N, 64), dtype=torch.float32, device="cuda")
    corr = torch.zeros((3 * N, W), dtype=torch.int64, device="cuda")
    ws = tc.alloc_workspace(tc.bp_workspace_bytes(lat, n_shots))
    tc.bp_decode(lat, d_syn, n_shots, d_llr, 0.0, K, iters, corr, post_a, ws)
    nu = [torch.zeros((W, N, 12, 64), dtype=torch.float32, device="cuda") for _ in range(2)]
    post_b = torch.zeros_like(post_a)
    prev = None
    for t in range(iters):
        tc.bp_step(lat, d_syn, n_shots, d_llr, 0.0, K, prev, nu[t % 2], post_b)
        prev = nu[t % 2]
    sync()
    a, b = post_a.cpu().numpy(), post_b.cpu().numpy()
    assert np.allclose(a, b, rtol=1e-4, atol=1e-4), np.abs(a - b).max()
    c_o, p_o = o.bp_decode(syn[:n_shots], p, q, iters,
                           llr0=llr_f32[:n_shots].astype(np.float64))
    c_g = bits_of_dev(corr, n_shots)
    mism = c_g != c_o
    announce(f"  hard-decision mismatches {int(mism.sum())}, max |post a-b| "
             f"{np.abs(a - b).max():.3e}")
    assert (np.abs(p_o[mism]) < LLR_TIE).all(), np.abs(p_o[mism]).max()


@pytest.mark.parametrize("L,n_shots,iters", [(3, 130, 20), (5, 100, 1), (6, 200, 2),
                                              (8, 150, 20), (12, 128, 20), (14, 64, 20)])
def test_bp_decode_resident_equals_streaming(L, n_shots, iters):
    """The whole-decode-in-LDS path (L <= 14, scalar prior) against the
    streaming kernels on the same syndromes, with the last iteration fused
    into the posterior and launched separately: corrections and posteriors bit
    for bit, padding shots of the last word included."""
    announce(f"resident BP L={L} S={n_shots} iters={iters}")
    out = decode_paths(L, n_shots, iters, 300 + L, 0.15, 0.9,
                       (tc.BP_RESIDENT, tc.BP_STREAMING, tc.BP_STREAMING_SPLIT))
    res = out[tc.BP_RESIDENT]
    for mode in (tc.BP_STREAMING, tc.BP_STREAMING_SPLIT):
        assert np.array_equal(res[0], out[mode][0])
        assert np.array_equal(res[1], out[mode][1])
    assert res[0].any()


def decode_paths(L, n_shots, iters, seed, density, K, modes, l0=math.log(19.0), llr=None):
    """tc3d_bp_decode of one random syndrome plane through each kernel path:
    {path: (correction words, posterior bits as int32)}. llr = (lo, hi): per-edge
    priors drawn uniformly from that range instead of the scalar l0."""
    import torch
    lat = tc.make_lattice(L)
    W = inputs.n_words(n_shots)
    syn = inputs.random_bits(seed, 64 * W, 3 * L ** 3, density)
    d_syn = dev_plane_of_bits(syn)
    d_llr = None
    if llr is not None:
        vals = inputs.random_llr(seed + 1, 64 * W, 3 * L ** 3, *llr)
        d_llr = to_dev(inputs.rows_to_gpu(vals))
    ws = tc.alloc_workspace(tc.bp_workspace_bytes(lat, n_shots))
    out = {}
    for mode in modes:
        corr = torch.full((3 * L ** 3, W), -1, dtype=torch.int64, device="cuda")
        post = torch.zeros((W, 3 * L ** 3, 64), dtype=torch.float32, device="cuda")
        tc.bp_decode(lat, d_syn, n_shots, d_llr, l0, K, iters, corr, post, ws, path=mode)
        sync()
        out[mode] = (corr.cpu().numpy(), post.cpu().numpy().view(np.int32))
    return out


@pytest.mark.parametrize("L,n_shots,iters,density,K", [
    (16, 64, 20, 0.05, 0.9), (16, 200, 2, 0.15, 0.9), (17, 130, 3, 0.1, 0.99),
    (24, 64, 1, 0.05, 0.9), (24, 128, 20, 0.02, 0.99), (48, 64, 20, 0.01, 0.9),
    (111, 64, 3, 0.01, 0.9), (112, 64, 2, 0.01, 0.9)])
def test_bp_last_iteration_fused_equals_split(L, n_shots, iters, density, K):
    """The last iteration fused with the posterior (one pass that recomputes
    the neighbouring faces' messages) against the iteration and posterior
    launched separately, on lattices too large for the resident kernel, odd L
    included: corrections and posteriors bit for bit. L = 111 is the largest
    lattice whose word of messages (L^3 x 3072 B) the fused pass addresses
    with 32-bit offsets; from L = 112 it uses 64-bit site addresses."""
    announce(f"fused last BP iteration L={L} S={n_shots} iters={iters} K={K}")
    out = decode_paths(L, n_shots, iters, 700 + L, density, K,
                       (tc.BP_STREAMING, tc.BP_STREAMING_SPLIT))
    fused, split = out[tc.BP_STREAMING], out[tc.BP_STREAMING_SPLIT]
    assert np.array_equal(fused[0], split[0])
    assert np.array_equal(fused[1], split[1])
    assert fused[0].any()


@pytest.mark.parametrize("L,n_shots,iters,lo,hi", [
    (5, 100, 2, -8.0, 8.0), (6, 130, 6, 0.5, 5.0), (16, 64, 6, -2.0, 6.0),
    (17, 64, 20, -8.0, 8.0), (48, 64, 6, 1.0, 4.0), (112, 64, 3, -8.0, 8.0)])
def test_bp_fused_last_iteration_with_per_edge_priors(L, n_shots, iters, lo, hi):
    """The fused last pass on a folded state (per-edge priors, as the CNN
    prior gives them, negative ones included) against the iteration and
    posterior launched separately: corrections and posteriors bit for bit
    (L = 112: 64-bit site addresses)."""
    announce(f"fused last BP iteration, per-edge priors L={L} S={n_shots} iters={iters}")
    out = decode_paths(L, n_shots, iters, 900 + L, 0.05, 0.9,
                       (tc.BP_STREAMING, tc.BP_STREAMING_SPLIT), l0=0.0, llr=(lo, hi))
    fused, split = out[tc.BP_STREAMING], out[tc.BP_STREAMING_SPLIT]
    assert np.array_equal(fused[0], split[0])
    assert np.array_equal(fused[1], split[1])
    assert fused[0].any()


def test_zero_syndrome_scalar_recursion_on_gpu():
    """With no unsatisfied check every posterior equals the closed-form scalar
    recursion l0 + 4 nu_T."""
    import torch
    L, n_shots, p, q = 4, 64, 0.05, 0.05
    lat = tc.make_lattice(L)
    d_syn = torch.zeros((3 * L ** 3, 1), dtype=torch.int64, device="cuda")
    corr = torch.zeros_like(d_syn)
    post = torch.zeros((1, 3 * L ** 3, 64), dtype=torch.float32, device="cuda")
    ws = tc.alloc_workspace(tc.bp_workspace_bytes(lat, n_shots))
    l0 = math.log((1 - p) / p)
    tc.bp_decode(lat, d_syn, n_shots, None, l0, 1 - 2 * q, 20, corr, post, ws)
    sync()
    nu = 0.0
    for _ in range(20):
        nu = 2 * math.atanh((1 - 2 * q) * math.tanh((l0 + 3 * nu) / 2) ** 3)
    assert np.allclose(post.cpu().numpy(), l0 + 4 * nu, rtol=1e-5)
    assert int(corr.abs().sum()) == 0


def test_empty_calls_are_noops():
    lat = tc.make_lattice(5)
    import torch
    t = torch.zeros(8, dtype=torch.int64, device="cuda")
    tc.sample_noise(lat, t, 0, 0.1, 1, 0, 0, 0)
    tc.syndrome(lat, t, t, 0)
    tc.logical_check(lat, t, 0, torch.zeros(8, dtype=torch.uint8, device="cuda"))
    sync()
    assert int(t.abs().sum()) == 0


def test_workspace_too_small_is_refused():
    import torch
    lat = tc.make_lattice(5)
    W = 2
    syn = torch.zeros((lat.n_faces, W), dtype=torch.int64, device="cuda")
    corr = torch.zeros_like(syn)
    ws = tc.alloc_workspace(256)
    with pytest.raises(tc.Tc3dError, match="workspace"):
        tc.flip_sweep(lat, syn, corr, W, ws)
