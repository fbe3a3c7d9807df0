"""The C-ABI library loads and exports every entry point that include/tc3d.h
declares; size queries and argument checks that launch nothing behave as
documented. No GPU needed: nothing here launches a kernel."""
import ctypes
import os
import re

import pytest

import paper_2212_06985_amd as tc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc3d.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc3d_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tc.LIB_PATH):
        import paper_2212_06985_amd.build as b
        b.build()
    return tc.lib()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    for name in ("tc3d_make_lattice", "tc3d_sample_noise", "tc3d_syndrome", "tc3d_bp_decode",
                 "tc3d_flip_sweep", "tc3d_pflip_sweep", "tc3d_run_cycles",
                 "tc3d_logical_check"):
        assert name in syms


def test_make_lattice(lib):
    lat = tc.make_lattice(6)
    assert (lat.L, lat.n_sites, lat.n_edges, lat.n_faces) == (6, 216, 648, 648)
    bad = tc.Lattice()
    for L in (0, 2, 513, -4):
        assert lib.tc3d_make_lattice(L, ctypes.byref(bad)) == -1
    assert lib.tc3d_make_lattice(8, None) == -1


def test_workspace_sizes(lib):
    lat = tc.make_lattice(12)
    # one edge plane per sweep, rounded to 256 bytes
    assert tc.sweep_workspace_bytes(lat, 3) == ((5184 * 3 * 8 + 255) // 256) * 256
    # two FP32 message buffers of 12 L^3 S_pad
    assert tc.bp_workspace_bytes(lat, 100) == 2 * 12 * 1728 * 128 * 4
    # a run: syndrome, correction and flip planes of one batch, two message
    # buffers when BP streams them through HBM, 256 bytes of counters
    planes = 3 * ((5184 * 8 * 8 + 255) // 256) * 256
    prm = tc.make_run_params(0.05, 0.05, 12, 20, 6, 0b001001, n_shots=1000, batch_shots=512,
                             bp_path=tc.BP_STREAMING)
    assert tc.run_workspace_bytes(lat, prm) == planes + 2 * 12 * 1728 * 512 * 4 + 256
    # the resident decode (L <= 14) keeps its messages in LDS
    prm.bp_path = tc.BP_AUTO
    assert tc.run_workspace_bytes(lat, prm) == planes + 256
    prm.bp_path = tc.BP_RESIDENT
    assert tc.run_workspace_bytes(lat, prm) == planes + 256
    # a readout: the parities of the 3 L^2 strings of each word
    assert tc.logical_check_workspace_bytes(lat, 100) == ((3 * 144 * 2 * 8 + 8 + 255) // 256) * 256
    corrupt = tc.make_lattice(12)
    corrupt.n_edges = 7
    assert lib.tc3d_sweep_workspace_bytes(ctypes.byref(corrupt), 3) == 0


def test_invalid_parameters_are_rejected_before_any_launch(lib):
    lat = tc.make_lattice(6)
    cases = [
        dict(p=0.6),                       # probability out of range
        dict(shot0=10),                    # not a multiple of 64
        dict(batch_shots=100),             # not a multiple of 64
        dict(n_sweeps=40),                 # too many sweeps
        dict(p_dec=0.0),                   # BP prior must be in (0, 0.5)
        dict(q_dec=0.5),
        dict(perfect_final=2),
        dict(bp_path=4),                   # no such kernel choice
        dict(bp_path=-1),
        dict(cycle0=0xFFFFFFFF),           # cycle indices past 2^32
        dict(bp_damp=1.0),                 # damping in [0, 1)
        dict(bp_damp=-0.1),
        dict(bp_warm=2),
        dict(bp_warm=1, bp_iters=1),       # one iteration stores no messages
        dict(bp_warm=1, bp_meta=1),        # the readings are of the paper's BP
    ]
    for over in cases:
        kw = dict(p=0.02, q=0.02, noisy_cycles=6, bp_iters=20, n_sweeps=5, pflip_mask=4,
                  n_shots=100)
        kw.update({k: v for k, v in over.items() if k in kw})
        prm = tc.make_run_params(**kw)
        for k, v in over.items():
            setattr(prm, k, v)
        assert lib.tc3d_run_workspace_bytes(ctypes.byref(lat), ctypes.byref(prm)) == 0, over
        rc = lib.tc3d_run_cycles(ctypes.byref(lat), ctypes.byref(prm), None, None, None, None, 0,
                                 None)
        assert rc == -1, over
    # stage entry points
    assert lib.tc3d_sample_noise(ctypes.byref(lat), None, 2, 0.1, 1, 0, 0, 64, None) == -1
    assert lib.tc3d_sample_noise(ctypes.byref(lat), None, 0, 1.5, 1, 0, 0, 64, None) == -1
    assert lib.tc3d_sample_noise(ctypes.byref(lat), None, 0, 0.1, 1, 0, 32, 64, None) == -1
    assert lib.tc3d_bp_decode(ctypes.byref(lat), None, 64, None, 2.9, 1.0, 20, 0, None, None,
                              None, 0, None) == -1  # meas_factor must be < 1
    assert lib.tc3d_bp_decode(ctypes.byref(lat), None, 64, None, 2.9, 0.9, 0, 0, None, None,
                              None, 0, None) == -1  # iters >= 1
    assert lib.tc3d_bp_decode(ctypes.byref(lat), None, 64, None, 2.9, 0.9, 20, 4, None, None,
                              None, 0, None) == -1  # no such kernel choice
    big = tc.make_lattice(16)  # the resident kernel holds at most 3072 sites
    assert lib.tc3d_bp_decode(ctypes.byref(big), None, 64, None, 2.9, 0.9, 20, 2, None, None,
                              None, 0, None) == -1
    # empty calls are no-ops
    assert lib.tc3d_syndrome(ctypes.byref(lat), None, None, 0, 0, None) == 0
    assert lib.tc3d_logical_check(ctypes.byref(lat), None, 0, None, None, None, 0, None) == 0
    # a readout needs the string-parity scratch
    assert lib.tc3d_logical_check(ctypes.byref(lat), ctypes.c_void_p(256), 64,
                                  ctypes.c_void_p(512), None, None, 0, None) == -4


def test_misaligned_and_missing_buffers(lib):
    lat = tc.make_lattice(4)
    # misaligned plane pointer is refused before anything runs
    assert lib.tc3d_syndrome(ctypes.byref(lat), ctypes.c_void_p(4), ctypes.c_void_p(8), 1, 0,
                             None) == -2
    # workspace missing
    assert lib.tc3d_flip_sweep(ctypes.byref(lat), ctypes.c_void_p(256), ctypes.c_void_p(512), 1,
                               None, 0, None) == -4


def test_strerror(lib):
    assert lib.tc3d_strerror(0) == b"ok"
    assert b"workspace" in lib.tc3d_strerror(-4)


def test_batched_jobs_and_autotune_reject_bad_arguments(lib):
    """Argument errors come back before any stream, event or launch."""
    import ctypes
    import paper_2212_06985_amd as tc
    prm = tc.make_run_params(0.05, 0.05, 2, 20, 6, 0b001001, n_shots=64)
    good = tc.Job(L=6, reserved=0, prm=prm, err_state=None, mask_out=None, odd_out=None)
    arr = (tc.Job * 2)(good, good)
    L = tc.lib()
    assert L.tc3d_run_jobs_workspace_bytes(arr, 2) > 0
    assert L.tc3d_run_jobs_workspace_bytes(arr, 0) == 0
    bad = (tc.Job * 1)(tc.Job(L=2, reserved=0, prm=prm))
    assert L.tc3d_run_jobs_workspace_bytes(bad, 1) == 0
    assert L.tc3d_run_jobs(arr, 0, None, 0, 0, None) == -1           # no jobs
    assert L.tc3d_run_jobs(arr, 2, None, 0, 0, None) == -4           # no workspace
    assert L.tc3d_run_jobs(arr, 2, None, 0, 8, None) == -1           # unknown flag
    ws = ctypes.c_void_p(1 << 20)  # aligned, never dereferenced
    assert L.tc3d_run_jobs(arr, 2, ws, 16, 0, None) == -4            # too small
    n = L.tc3d_run_jobs_workspace_bytes(arr, 2)
    assert L.tc3d_run_jobs(arr, 2, ws, n, 0, None) == -1             # missing buffers
    lat = tc.make_lattice(6)
    out = (tc.TuneChoice * 4)()
    cnt = ctypes.c_int32(0)
    assert L.tc3d_autotune(ctypes.byref(lat), ctypes.byref(prm), 0, ws, 1 << 30, out, 4,
                           ctypes.byref(cnt), None) == -1            # probe_cycles 0
    assert L.tc3d_autotune(ctypes.byref(lat), ctypes.byref(prm), 1, None, 0, out, 4,
                           ctypes.byref(cnt), None) == -4            # no workspace


def test_subset_sweeps_need_even_L_and_a_schedule_slot(lib):
    import ctypes
    import paper_2212_06985_amd as tc
    L = tc.lib()
    odd = tc.make_lattice(5)
    even = tc.make_lattice(6)
    prm = tc.make_run_params(0.03, 0.03, 2, 0, 5, 0, n_shots=64, subset_mask=0b00100)
    assert L.tc3d_run_workspace_bytes(ctypes.byref(even), ctypes.byref(prm)) > 0
    assert L.tc3d_run_workspace_bytes(ctypes.byref(odd), ctypes.byref(prm)) == 0
    beyond = tc.make_run_params(0.03, 0.03, 2, 0, 5, 0, n_shots=64, subset_mask=0b100000)
    assert L.tc3d_run_workspace_bytes(ctypes.byref(even), ctypes.byref(beyond)) == 0
    ws = ctypes.c_void_p(1 << 20)
    for lat, cls in ((odd, 0), (even, -1), (even, 12)):
        assert L.tc3d_subset_pflip_sweep(ctypes.byref(lat), ws, ws, 1, 1, 0, 0, 0, cls, ws,
                                         1 << 30, None) == -1


def test_stream_copy_rejects_bad_arguments(lib):
    """Checked on the host before any launch: size a multiple of 16, the
    store flag 0 or 1, buffers present, 16-byte aligned and disjoint."""
    cp = lib.tc3d_stream_copy
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21)  # never dereferenced
    assert cp(b, a, 0, 1, None) == 0                    # nothing to copy
    assert cp(b, a, 24, 1, None) == -1                  # not a multiple of 16
    assert cp(b, a, -16, 1, None) == -1
    assert cp(b, a, 64, 2, None) == -1                  # store flag
    assert cp(None, a, 64, 1, None) == -1
    assert cp(ctypes.c_void_p((1 << 21) + 8), a, 64, 1, None) == -2   # misaligned
    assert cp(ctypes.c_void_p((1 << 20) + 32), a, 64, 0, None) == -1  # overlap
    assert cp(a, ctypes.c_void_p((1 << 20) + 48), 64, 0, None) == -1  # overlap


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding raises instead of falling back
    to anything else."""
    import subprocess
    import sys
    code = ("import paper_2212_06985_amd as tc\n"
            f"tc.LIB_PATH = {str(tmp_path / 'absent.so')!r}\n"
            "tc._lib = None\n"
            "try:\n"
            "    tc.make_lattice(6)\n"
            "except ImportError as e:\n"
            "    print('raised:', e)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=root, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "raised:" in out.stdout and "absent.so is missing" in out.stdout
