"""Host logic of bench.py: the roofline arithmetic and the one-GPU refusal."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _cls(**kw):
    base = {k: {"ms": 0.0, "launches": 0} for k in ("bp_iter", "bp_first", "bp_post", "cnn")}
    base.update(kw)
    return base


def test_bp_roofline_counts_32_bytes_per_edge_shot():
    # 10 launches of 2 ms, each over 3 * 1000 edges x 2048 shots
    pc = _cls(bp_iter={"ms": 20.0, "launches": 10})
    r = bench.roofline(pc, 3000, 2048, 1000, "none", shots_padded=2048)
    assert r["kernel"] == "bp_iter" and r["bound"] == "hbm"
    assert r["algo_bytes_per_launch"] == 32.0 * 3000 * 2048
    assert r["achieved"] == pytest.approx(32.0 * 3000 * 2048 / 2e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)  # rounded to 4 places


def test_per_edge_prior_adds_the_prior_read():
    pc = _cls(bp_iter={"ms": 20.0, "launches": 10})
    r = bench.roofline(pc, 3000, 2048, 1000, "none", shots_padded=2048, per_edge_prior=True)
    assert r["algo_bytes_per_unit"] == 36.0


def test_uneven_batches_average_the_shots_per_launch():
    # 5000 shots in batches of 2048: 3 launches per iteration carry 5000 / 3 shots each
    pc = _cls(bp_iter={"ms": 30.0, "launches": 3})
    r = bench.roofline(pc, 3000, 2048, 1000, "none", shots_padded=5000)
    assert r["algo_bytes_per_launch"] == pytest.approx(32.0 * 3000 * 5000 / 3)


def test_cnn_roofline_is_flop_over_all_forwards():
    pc = _cls(cnn={"ms": 50.0, "launches": 25}, bp_iter={"ms": 1.0, "launches": 1})
    r = bench.roofline(pc, 3000, 4096, 1000, "none", forwards=5, shots_padded=4096)
    assert r["bound"] == "mfma"
    flop = bench.CNN_FLOP_PER_SITE * 1000 * 4096 * 5
    assert r["achieved"] == pytest.approx(flop / 50e-3 / 1e12, rel=1e-3)


def test_cnn_flop_per_site_matches_the_network():
    ch = [8, 32, 32, 32, 3]
    assert bench.CNN_FLOP_PER_SITE == sum(2 * 27 * a * b for a, b in zip(ch, ch[1:]))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr


def test_traffic_is_looked_up_per_kernel_variant(tmp_path, monkeypatch):
    """The per-edge-prior BP iteration has counters of its own: a plain BP
    line never reports them, and counters taken on other sources are not
    reported at all."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    for wl, h in (("cx", _HASHES["bp_iter_prior"]), ("cy", "0123456789abcdef")):
        (prof / f"bp_iter_prior_{wl}_traffic.txt").write_text(
            f"hbm_bytes_per_launch: 123.0\nstream_ceiling_GBps: 6000\nsource_sha256: {h}\n")
    # the sources stay where they are; only the profiles folder moves
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda k="bp_iter": _HASHES[k])
    pc = _cls(bp_iter={"ms": 20.0, "launches": 10})
    r = bench.roofline(pc, 3000, 2048, 1000, "cx", shots_padded=2048, per_edge_prior=True)
    assert r["traffic"] == 123.0 and r["stream_ceiling"] == 6000.0
    r = bench.roofline(pc, 3000, 2048, 1000, "cx", shots_padded=2048)
    assert r["traffic"] is None and r["stream_ceiling"] is None
    r = bench.roofline(pc, 3000, 2048, 1000, "cy", shots_padded=2048, per_edge_prior=True)
    assert r["traffic"] is None


_HASHES = {k: bench.kernel_source_hash(k) for k in bench.KERNEL_SOURCES}


def test_path_roofline_model():
    # 20 BP iterations, scalar prior: iteration 2 writes 16 B, 3..19 read and
    # write 32 B, iteration 20 fused with the posterior reads 16 B; plus 20
    # syndrome bits and 4 B of bit planes
    r = bench.path_roofline(20, 1e10)
    assert r["bytes_per_unit"] == 16 + 32.0 * 17 + 16 + 20 / 8 + 4 == 582.5
    assert r["achieved"] == pytest.approx(1e10 * 582.5 / 1e9, rel=1e-6)
    assert r["frac"] == pytest.approx(1e10 * 582.5 / 8e12, abs=1e-4)
    # the last iteration and the posterior launched separately: 32 B more
    assert bench.path_roofline(20, 1e10, fused=False)["bytes_per_unit"] == 614.5
    # two iterations fused read only syndrome bits; one decodes from them
    assert bench.bp_message_bytes(2) == 0.0 and bench.bp_message_bytes(1) == 0.0
    assert bench.bp_message_bytes(2, fused=False) == 32.0
    # a per-edge prior: the first iteration writes and reads the prior, each
    # later one reads and writes, the posterior reads; fused, the last
    # iteration and the posterior read the state and the prior once
    assert bench.path_roofline(6, 1e10, per_edge_prior=True)["bytes_per_unit"] == \
        20 + 36.0 * 4 + 20 + 6 / 8 + 4
    assert bench.path_roofline(6, 1e10, per_edge_prior=True, fused=False)["bytes_per_unit"] == \
        20 + 36.0 * 5 + 16 + 6 / 8 + 4
    assert bench.bp_message_bytes(1, per_edge_prior=True) == 36.0
    # without BP there is no HBM model
    assert bench.path_roofline(0, 1e10) is None


def test_resident_bp_roofline_is_alu_bound():
    # L = 12 (1728 sites, 5184 edges), 20 iterations, one launch of 2 ms per batch
    pc = _cls(bp_iter={"ms": 2.0, "launches": 1})
    r = bench.roofline(pc, 5184, 4096, 1728, "none", shots_padded=4096, bp_iters=20)
    assert r["bound"] == "alu" and r["kernel"].startswith("bp_resident")
    # VALU issue cycles per site and iteration: per check 4 median clamps,
    # 8 (a -+ 1), 10 products and per output 2 fused multiply-adds, a product
    # and a reciprocal of two cycles; 30 products forming e^mu
    per_site = (3 * (22 + 4 * (2 + 1 + 2)) + 30) * 19 + 12
    assert per_site == 156 * 19 + 12
    assert r["algo_ops_per_unit"] == per_site
    assert r["algo_ops_per_launch"] == per_site * 1728 * 4096
    assert r["achieved"] == pytest.approx(per_site * 1728 * 4096 / 2e-3 / 1e12, abs=0.01)
    # one FP32 op per lane per clock: 256 CUs x 64 lanes x 2.4 GHz
    assert r["peak"] == pytest.approx(39.32, abs=0.01)
    # larger lattices, or a per-edge prior, stream their messages through HBM
    assert bench.roofline(pc, 3 * 4096, 4096, 4096, "none", shots_padded=4096,
                          bp_iters=20)["bound"] == "hbm"
    assert bench.roofline(pc, 5184, 4096, 1728, "none", shots_padded=4096, bp_iters=20,
                          per_edge_prior=True)["bound"] == "hbm"


def test_path_roofline_is_none_for_a_resident_decode():
    assert bench.path_roofline(20, 1e10, n_sites=1728) is None
    assert bench.path_roofline(20, 1e10, n_sites=48 ** 3)["bytes_per_unit"] == 582.5


def test_counter_summaries_apply_only_to_their_own_launches():
    assert bench.profile_key("c5") == "c5"
    assert bench.profile_key("c5", L=48, shots=2048) == "c5"
    assert bench.profile_key("c4", L=16) == "c4_custom"
    assert bench.profile_key("c5", shots=4096) == "c5_custom"
    assert bench.profile_key("c2", batch_shots=4096) == "c2_custom"
    assert bench.stored_traffic("cnn", bench.profile_key("c4", L=16)) is None
