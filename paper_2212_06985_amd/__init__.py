"""Shot-parallel Monte Carlo decoding of the 3D toric code on AMD MI355X.

A thin ctypes binding of libtc3d.so (include/tc3d.h): every function takes
torch tensors that live on the GPU, passes their data pointers and the current
HIP stream to the C ABI, and raises on a non-zero return code. All work runs
in the library's HIP kernels; there is no CPU fallback. Build the library with
``python -m paper_2212_06985_amd.build`` (or ``__graft_entry__.build()``).

Layouts (see the header): bit planes are int64 tensors [3 L^3][ceil(S/64)]
holding uint64 words, bit i of word w = shot 64 w + i; per-shot floats are
[rows][64 ceil(S/64)].
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "Lattice", "RunParams", "Timing", "Tc3dError", "lib", "make_lattice", "sample_noise",
    "syndrome", "sweep_workspace_bytes", "flip_sweep", "pflip_sweep", "subset_pflip_sweep",
    "bp_meta_workspace_bytes", "bp_meta_decode", "bp_meta_step", "bp_workspace_bytes",
    "bp_decode", "bp_step", "logical_check", "run_workspace_bytes", "run_cycles",
    "run_cycles_timed", "n_words", "alloc_plane", "alloc_workspace", "KERNEL_CLASSES",
    "logical_check_workspace_bytes", "built_id", "BP_AUTO", "BP_STREAMING", "BP_RESIDENT",
    "BP_STREAMING_SPLIT",
    "run_cycles_noalloc", "apply_correction", "RUN_GRAPH",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtc3d.so")

KERNEL_CLASSES = ["bp_iter", "bp_first", "bp_post", "noise", "syndrome", "sweep", "apply",
                  "readout", "cnn"]


class Tc3dError(RuntimeError):
    pass


class Lattice(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_sites", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("n_faces", ctypes.c_int64)]


class RunParams(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_double), ("q", ctypes.c_double),
        ("p_dec", ctypes.c_double), ("q_dec", ctypes.c_double),
        ("noisy_cycles", ctypes.c_int32), ("perfect_final", ctypes.c_int32),
        ("final_qubit_noise", ctypes.c_int32), ("bp_iters", ctypes.c_int32),
        ("n_sweeps", ctypes.c_int32), ("pflip_mask", ctypes.c_uint32),
        ("seed", ctypes.c_uint64), ("shot0", ctypes.c_uint64),
        ("n_shots", ctypes.c_int64), ("batch_shots", ctypes.c_int64),
        ("bp_tile", ctypes.c_int32), ("subset_mask", ctypes.c_uint32),
        ("bp_meta", ctypes.c_int32), ("cycle0", ctypes.c_uint32),
        ("bp_path", ctypes.c_int32), ("bp_warm", ctypes.c_int32),
        ("bp_damp", ctypes.c_double), ("flags", ctypes.c_uint32),
        ("bp_occupancy", ctypes.c_int32),
    ]


class Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 9), ("launches", ctypes.c_int64 * 9),
                ("total_ms", ctypes.c_double), ("bp_decisions", ctypes.c_int64),
                ("bp_near_ties", ctypes.c_int64)]

    def as_dict(self):
        return {k: {"ms": self.ms[i], "launches": int(self.launches[i])}
                for i, k in enumerate(KERNEL_CLASSES)}


class Job(ctypes.Structure):
    """One experiment of a batched call (tc3d_job)."""
    _fields_ = [("L", ctypes.c_int32), ("reserved", ctypes.c_int32), ("prm", RunParams),
                ("err_state", ctypes.c_void_p), ("mask_out", ctypes.c_void_p),
                ("odd_out", ctypes.c_void_p)]


class TuneChoice(ctypes.Structure):
    _fields_ = [("bp_tile", ctypes.c_int32), ("bp_path", ctypes.c_int32),
                ("batch_shots", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bp_occupancy", ctypes.c_int32), ("reserved", ctypes.c_int32)]


JOBS_CONCURRENT = 1
JOBS_GRAPH = 2

# run flags: capture a run's launches into one HIP graph (tc3d_run_cycles blocks)
RUN_GRAPH = 1

# kernels of a BP decode (tc3d_bp_decode's bp_path; never changes a result)
BP_AUTO = 0
BP_STREAMING = 1
BP_RESIDENT = 2
BP_STREAMING_SPLIT = 3

_lib = None


def built_id():
    """The source hash libtc3d.so was built with, or None when it is missing."""
    if not os.path.exists(LIB_PATH):
        return None
    L = ctypes.CDLL(LIB_PATH)
    L.tc3d_build_id.restype = ctypes.c_char_p
    L.tc3d_build_id.argtypes = []
    return L.tc3d_build_id().decode()


def lib():
    """Load libtc3d.so; fail loudly when it has not been built, or was built
    from other sources than the ones in the tree."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2212_06985_amd.build`")
    from . import build as _build
    have, want = built_id(), _build.source_id()
    if have != want:
        raise ImportError(f"{LIB_PATH} was built from other sources ({have[:12]}, the tree "
                          f"is {want[:12]}): rebuild it with "
                          "`python -m paper_2212_06985_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, i64, u64, f32, f64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                             ctypes.c_int64, ctypes.c_uint64, ctypes.c_float,
                                             ctypes.c_double, ctypes.c_size_t)
    lat, prm = ctypes.POINTER(Lattice), ctypes.POINTER(RunParams)
    sigs = {
        "tc3d_make_lattice": (ctypes.c_int, [i32, lat]),
        "tc3d_sample_noise": (ctypes.c_int, [lat, vp, i32, f64, u64, u32, u64, i64, vp]),
        "tc3d_syndrome": (ctypes.c_int, [lat, vp, vp, i64, i32, vp]),
        "tc3d_sweep_workspace_bytes": (sz, [lat, i64]),
        "tc3d_flip_sweep": (ctypes.c_int, [lat, vp, vp, i64, vp, sz, vp]),
        "tc3d_pflip_sweep": (ctypes.c_int, [lat, vp, vp, i64, u64, u32, u32, u64, vp, sz, vp]),
        "tc3d_subset_pflip_sweep": (ctypes.c_int, [lat, vp, vp, i64, u64, u32, u32, u64, i32,
                                                   vp, sz, vp]),
        "tc3d_bp_workspace_bytes": (sz, [lat, i64]),
        "tc3d_bp_decode": (ctypes.c_int, [lat, vp, i64, vp, f32, f32, i32, i32, vp, vp, vp, sz,
                                          vp]),
        "tc3d_bp_step": (ctypes.c_int, [lat, vp, i64, vp, f32, f32, f32, vp, vp, vp, vp]),
        "tc3d_logical_check_workspace_bytes": (sz, [lat, i64]),
        "tc3d_logical_check": (ctypes.c_int, [lat, vp, i64, vp, vp, vp, sz, vp]),
        "tc3d_bp_meta_workspace_bytes": (sz, [lat, i64]),
        "tc3d_bp_meta_decode": (ctypes.c_int, [lat, vp, i64, f64, f64, i32, vp, vp, vp, sz, vp]),
        "tc3d_bp_meta_step": (ctypes.c_int, [lat, vp, i64, f64, f64, vp, vp, vp, vp]),
        "tc3d_run_workspace_bytes": (sz, [lat, prm]),
        "tc3d_run_cycles": (ctypes.c_int, [lat, prm, vp, vp, vp, vp, sz, vp]),
        "tc3d_run_cycles_noalloc": (ctypes.c_int, [lat, prm, vp, vp, vp, vp]),
        "tc3d_run_cycles_timed": (ctypes.c_int, [lat, prm, vp, vp, vp, vp, sz, vp,
                                                 ctypes.POINTER(Timing)]),
        "tc3d_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "tc3d_build_id": (ctypes.c_char_p, []),
        "tc3d_cnn_param_count": (i64, []),
        "tc3d_cnn_packed_bytes": (sz, []),
        "tc3d_cnn_pack": (ctypes.c_int, [vp, f32, f32, vp, vp]),
        "tc3d_apply_correction": (ctypes.c_int, [lat, vp, vp, i64, vp]),
        "tc3d_cnn_workspace_bytes": (sz, [lat, i64, i32]),
        "tc3d_cnn_forward": (ctypes.c_int, [lat, vp, vp, i64, vp, vp, vp, sz, vp]),
        "tc3d_cnn_loss_grad": (ctypes.c_int, [lat, vp, vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]),
        "tc3d_cnn_adam": (ctypes.c_int, [vp, vp, vp, vp, i32, f32, f32, f32, f32, vp, vp]),
        "tc3d_run_cnn_workspace_bytes": (sz, [lat, prm]),
        "tc3d_run_cycles_cnn": (ctypes.c_int, [lat, prm, vp, vp, vp, vp, vp, sz, vp]),
        "tc3d_run_cycles_cnn_timed": (ctypes.c_int, [lat, prm, vp, vp, vp, vp, vp, sz, vp,
                                                     ctypes.POINTER(Timing)]),
        "tc3d_stream_copy": (ctypes.c_int, [vp, vp, i64, i32, vp]),
        "tc3d_run_jobs_workspace_bytes": (sz, [ctypes.POINTER(Job), i32]),
        "tc3d_run_jobs": (ctypes.c_int, [ctypes.POINTER(Job), i32, vp, sz, i32, vp]),
        "tc3d_autotune_workspace_bytes": (sz, [lat, prm]),
        "tc3d_autotune": (ctypes.c_int, [lat, prm, i32, vp, sz, ctypes.POINTER(TuneChoice), i32,
                                         ctypes.POINTER(i32), vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return _lib


# ----------------------------------------------------------------- marshalling
def _check(rc: int, what: str):
    if rc != 0:
        raise Tc3dError(f"{what}: {lib().tc3d_strerror(rc).decode()} ({rc})")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def n_words(n_shots: int) -> int:
    return (int(n_shots) + 63) // 64


def make_lattice(L: int) -> Lattice:
    lat = Lattice()
    _check(lib().tc3d_make_lattice(int(L), ctypes.byref(lat)), "make_lattice")
    return lat


def alloc_plane(lat: Lattice, n_shots: int, device="cuda"):
    import torch
    return torch.zeros((lat.n_edges, n_words(n_shots)), dtype=torch.int64, device=device)


def alloc_workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def sample_noise(lat, plane, kind, prob, seed, cycle, shot0, n_shots, stream=None):
    _check(lib().tc3d_sample_noise(ctypes.byref(lat), _ptr(plane), int(kind), float(prob),
                                   int(seed), int(cycle), int(shot0), int(n_shots),
                                   _stream(stream)), "sample_noise")


def syndrome(lat, err, syn, nw, xor_into=False, stream=None):
    _check(lib().tc3d_syndrome(ctypes.byref(lat), _ptr(err), _ptr(syn), int(nw),
                               1 if xor_into else 0, _stream(stream)), "syndrome")


def apply_correction(lat, err, corr, nw, stream=None):
    """err ^= corr (apply a cycle's correction, carry the residual)."""
    _check(lib().tc3d_apply_correction(ctypes.byref(lat), _ptr(err), _ptr(corr), int(nw),
                                       _stream(stream)), "apply_correction")


def sweep_workspace_bytes(lat, nw) -> int:
    return int(lib().tc3d_sweep_workspace_bytes(ctypes.byref(lat), int(nw)))


def flip_sweep(lat, syn, corr, nw, ws, stream=None):
    _check(lib().tc3d_flip_sweep(ctypes.byref(lat), _ptr(syn), _ptr(corr), int(nw), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream)), "flip_sweep")


def pflip_sweep(lat, syn, corr, nw, seed, cycle, sweep, shot0, ws, stream=None):
    _check(lib().tc3d_pflip_sweep(ctypes.byref(lat), _ptr(syn), _ptr(corr), int(nw), int(seed),
                                  int(cycle), int(sweep), int(shot0), _ptr(ws),
                                  ws.numel() * ws.element_size(), _stream(stream)),
           "pflip_sweep")


def subset_pflip_sweep(lat, syn, corr, nw, seed, cycle, sweep, shot0, edge_class, ws,
                       stream=None):
    _check(lib().tc3d_subset_pflip_sweep(ctypes.byref(lat), _ptr(syn), _ptr(corr), int(nw),
                                         int(seed), int(cycle), int(sweep), int(shot0),
                                         int(edge_class), _ptr(ws),
                                         ws.numel() * ws.element_size(), _stream(stream)),
           "subset_pflip_sweep")


def bp_workspace_bytes(lat, n_shots) -> int:
    return int(lib().tc3d_bp_workspace_bytes(ctypes.byref(lat), int(n_shots)))


def bp_decode(lat, syn, n_shots, llr0, llr0_scalar, meas_factor, iters, corr_out, post_out, ws,
              stream=None, path=BP_AUTO):
    _check(lib().tc3d_bp_decode(ctypes.byref(lat), _ptr(syn), int(n_shots), _ptr(llr0),
                                float(llr0_scalar), float(meas_factor), int(iters), int(path),
                                _ptr(corr_out), _ptr(post_out), _ptr(ws),
                                ws.numel() * ws.element_size(), _stream(stream)), "bp_decode")


def bp_step(lat, syn, n_shots, llr0, llr0_scalar, meas_factor, nu_in, nu_out, post_out=None,
            stream=None, damp=0.0):
    _check(lib().tc3d_bp_step(ctypes.byref(lat), _ptr(syn), int(n_shots), _ptr(llr0),
                              float(llr0_scalar), float(meas_factor), float(damp), _ptr(nu_in),
                              _ptr(nu_out), _ptr(post_out), _stream(stream)), "bp_step")


def bp_meta_workspace_bytes(lat, n_shots) -> int:
    return int(lib().tc3d_bp_meta_workspace_bytes(ctypes.byref(lat), int(n_shots)))


def bp_meta_decode(lat, syn, n_shots, p_dec, q_dec, iters, corr_out, post_out, ws, stream=None):
    _check(lib().tc3d_bp_meta_decode(ctypes.byref(lat), _ptr(syn), int(n_shots), float(p_dec),
                                     float(q_dec), int(iters), _ptr(corr_out), _ptr(post_out),
                                     _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "bp_meta_decode")


def bp_meta_step(lat, syn, n_shots, p_dec, q_dec, state_in, state_out, post_out, stream=None):
    _check(lib().tc3d_bp_meta_step(ctypes.byref(lat), _ptr(syn), int(n_shots), float(p_dec),
                                   float(q_dec), _ptr(state_in), _ptr(state_out),
                                   _ptr(post_out), _stream(stream)), "bp_meta_step")


def logical_check_workspace_bytes(lat, n_shots) -> int:
    return int(lib().tc3d_logical_check_workspace_bytes(ctypes.byref(lat), int(n_shots)))


def logical_check(lat, err, n_shots, mask_out, odd_out=None, ws=None, stream=None):
    if ws is None:
        ws = alloc_workspace(logical_check_workspace_bytes(lat, n_shots))
    _check(lib().tc3d_logical_check(ctypes.byref(lat), _ptr(err), int(n_shots), _ptr(mask_out),
                                    _ptr(odd_out), _ptr(ws), ws.numel() * ws.element_size(),
                                    _stream(stream)), "logical_check")


def run_workspace_bytes(lat, prm: RunParams) -> int:
    n = int(lib().tc3d_run_workspace_bytes(ctypes.byref(lat), ctypes.byref(prm)))
    if n == 0:
        raise Tc3dError("run_workspace_bytes: invalid lattice or parameters")
    return n


def run_cycles(lat, prm: RunParams, err_state, mask_out, odd_out, ws, stream=None):
    _check(lib().tc3d_run_cycles(ctypes.byref(lat), ctypes.byref(prm), _ptr(err_state),
                                 _ptr(mask_out), _ptr(odd_out), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream)), "run_cycles")


def run_cycles_noalloc(lat, prm: RunParams, err_state, mask_out, odd_out=None, stream=None):
    """run_cycles with the library's fixed per-device scratch (no workspace)."""
    _check(lib().tc3d_run_cycles_noalloc(ctypes.byref(lat), ctypes.byref(prm), _ptr(err_state),
                                         _ptr(mask_out), _ptr(odd_out), _stream(stream)),
           "run_cycles_noalloc")


def run_cycles_timed(lat, prm: RunParams, err_state, mask_out, odd_out, ws,
                     stream=None) -> Timing:
    t = Timing()
    _check(lib().tc3d_run_cycles_timed(ctypes.byref(lat), ctypes.byref(prm), _ptr(err_state),
                                       _ptr(mask_out), _ptr(odd_out), _ptr(ws),
                                       ws.numel() * ws.element_size(), _stream(stream),
                                       ctypes.byref(t)), "run_cycles_timed")
    return t


# ------------------------------------------------------------------ CNN prior
def cnn_param_count() -> int:
    return int(lib().tc3d_cnn_param_count())


def cnn_packed_bytes() -> int:
    return int(lib().tc3d_cnn_packed_bytes())


def cnn_pack(params, packed, beta=1.0, p=None, stream=None):
    """Packs the network; with beta < 1 its prior is blended with the channel
    prior of error rate p: llr0 = l0 + beta (llr_cnn - l0)."""
    import math
    l0 = 0.0 if p is None else math.log((1 - p) / p)
    if beta != 1.0 and p is None:
        raise ValueError("cnn_pack: blending needs the channel error rate p")
    _check(lib().tc3d_cnn_pack(_ptr(params), float(beta), float(l0), _ptr(packed),
                               _stream(stream)), "cnn_pack")


def cnn_workspace_bytes(lat, n_shots, training=False) -> int:
    n = int(lib().tc3d_cnn_workspace_bytes(ctypes.byref(lat), int(n_shots), 1 if training else 0))
    if n == 0:
        raise Tc3dError("cnn_workspace_bytes: invalid lattice or shot count")
    return n


def cnn_forward(lat, syn, prev, n_shots, packed, llr_out, ws, stream=None):
    _check(lib().tc3d_cnn_forward(ctypes.byref(lat), _ptr(syn), _ptr(prev), int(n_shots),
                                  _ptr(packed), _ptr(llr_out), _ptr(ws),
                                  ws.numel() * ws.element_size(), _stream(stream)), "cnn_forward")


def cnn_loss_grad(lat, syn, prev, target, n_shots, packed, llr_out, grad, loss, ws, stream=None):
    _check(lib().tc3d_cnn_loss_grad(ctypes.byref(lat), _ptr(syn), _ptr(prev), _ptr(target),
                                    int(n_shots), _ptr(packed), _ptr(llr_out), _ptr(grad),
                                    _ptr(loss), _ptr(ws), ws.numel() * ws.element_size(),
                                    _stream(stream)), "cnn_loss_grad")


def cnn_adam(params, grad, m, v, step, lr, packed, beta1=0.9, beta2=0.999, eps=1e-8,
             stream=None):
    _check(lib().tc3d_cnn_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step),
                               float(lr), float(beta1), float(beta2), float(eps), _ptr(packed),
                               _stream(stream)), "cnn_adam")


def run_cnn_workspace_bytes(lat, prm: RunParams) -> int:
    n = int(lib().tc3d_run_cnn_workspace_bytes(ctypes.byref(lat), ctypes.byref(prm)))
    if n == 0:
        raise Tc3dError("run_cnn_workspace_bytes: invalid lattice or parameters")
    return n


def run_cycles_cnn(lat, prm: RunParams, packed, err_state, mask_out, odd_out, ws, stream=None):
    _check(lib().tc3d_run_cycles_cnn(ctypes.byref(lat), ctypes.byref(prm), _ptr(packed),
                                     _ptr(err_state), _ptr(mask_out), _ptr(odd_out), _ptr(ws),
                                     ws.numel() * ws.element_size(), _stream(stream)),
           "run_cycles_cnn")


def run_cycles_cnn_timed(lat, prm: RunParams, packed, err_state, mask_out, odd_out, ws,
                         stream=None) -> Timing:
    t = Timing()
    _check(lib().tc3d_run_cycles_cnn_timed(ctypes.byref(lat), ctypes.byref(prm), _ptr(packed),
                                           _ptr(err_state), _ptr(mask_out), _ptr(odd_out),
                                           _ptr(ws), ws.numel() * ws.element_size(),
                                           _stream(stream), ctypes.byref(t)),
           "run_cycles_cnn_timed")
    return t


__all__ += ["cnn_param_count", "cnn_packed_bytes", "cnn_pack", "cnn_workspace_bytes",
            "cnn_forward", "cnn_loss_grad", "cnn_adam", "run_cnn_workspace_bytes",
            "run_cycles_cnn", "run_cycles_cnn_timed"]


def make_run_params(p, q, noisy_cycles, bp_iters, n_sweeps, pflip_mask, n_shots, seed=1,
                    shot0=0, p_dec=None, q_dec=None, perfect_final=1, final_qubit_noise=1,
                    batch_shots=0, bp_tile=0, subset_mask=0, bp_meta=0, cycle0=0,
                    bp_path=BP_AUTO, bp_warm=0, bp_damp=0.0, flags=0,
                    bp_occupancy=0) -> RunParams:
    return RunParams(p=p, q=q, p_dec=p if p_dec is None else p_dec,
                     q_dec=q if q_dec is None else q_dec, noisy_cycles=noisy_cycles,
                     perfect_final=perfect_final, final_qubit_noise=final_qubit_noise,
                     bp_iters=bp_iters, n_sweeps=n_sweeps, pflip_mask=pflip_mask, seed=seed,
                     shot0=shot0, n_shots=n_shots, batch_shots=batch_shots, bp_tile=bp_tile,
                     subset_mask=subset_mask, bp_meta=int(bp_meta), cycle0=int(cycle0),
                     bp_path=int(bp_path), bp_warm=int(bp_warm), bp_damp=float(bp_damp),
                     flags=int(flags), bp_occupancy=int(bp_occupancy))


__all__.append("make_run_params")


# --------------------------------------------------------------- batched jobs
def make_job(L: int, prm: RunParams, err_state, mask_out, odd_out=None) -> Job:
    def addr(t):
        p = _ptr(t)
        return None if p is None else p.value
    return Job(L=int(L), reserved=0, prm=prm, err_state=addr(err_state),
               mask_out=addr(mask_out), odd_out=addr(odd_out))


def _job_array(jobs):
    arr = (Job * len(jobs))(*jobs)
    return arr, len(jobs)


def run_jobs_workspace_bytes(jobs) -> int:
    arr, n = _job_array(jobs)
    b = int(lib().tc3d_run_jobs_workspace_bytes(arr, n))
    if b == 0:
        raise Tc3dError("run_jobs_workspace_bytes: invalid jobs")
    return b


def run_jobs(jobs, ws, flags=JOBS_CONCURRENT | JOBS_GRAPH, stream=None):
    """Runs every job (blocking); each equals run_cycles on its own buffers."""
    arr, n = _job_array(jobs)
    _check(lib().tc3d_run_jobs(arr, n, _ptr(ws), ws.numel() * ws.element_size(), int(flags),
                               _stream(stream)), "run_jobs")


def autotune_workspace_bytes(lat, prm: RunParams) -> int:
    b = int(lib().tc3d_autotune_workspace_bytes(ctypes.byref(lat), ctypes.byref(prm)))
    if b == 0:
        raise Tc3dError("autotune_workspace_bytes: invalid lattice or parameters")
    return b


def autotune(lat, prm: RunParams, ws, probe_cycles=2, stream=None):
    """Times candidate settings of the knobs that never change results (BP
    schedule, traversal tile, occupancy, batch) on the first probe_cycles
    cycles of prm's shots and writes the fastest into prm. Returns the list of
    dicts {bp_path, bp_tile, bp_occupancy, batch_shots, ms} tried."""
    out = (TuneChoice * 64)()
    n = ctypes.c_int32(0)
    _check(lib().tc3d_autotune(ctypes.byref(lat), ctypes.byref(prm), int(probe_cycles), _ptr(ws),
                               ws.numel() * ws.element_size(), out, 64, ctypes.byref(n),
                               _stream(stream)), "autotune")
    return [dict(bp_path=out[i].bp_path, bp_tile=out[i].bp_tile,
                 bp_occupancy=out[i].bp_occupancy, batch_shots=out[i].batch_shots,
                 ms=out[i].ms) for i in range(min(n.value, 64))]


__all__ += ["Job", "TuneChoice", "JOBS_CONCURRENT", "JOBS_GRAPH", "make_job",
            "run_jobs_workspace_bytes", "run_jobs", "autotune_workspace_bytes", "autotune"]


def stream_copy(dst, src, nontemporal=True, stream=None):
    """dst[:] = src[:] by the library's streaming copy kernel (same byte size)."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("stream_copy: sizes differ")
    _check(lib().tc3d_stream_copy(_ptr(dst), _ptr(src), int(n), 1 if nontemporal else 0,
                                  _stream(stream)), "stream_copy")


__all__.append("stream_copy")
