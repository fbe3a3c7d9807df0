"""ctypes wrapper of the plain CPU oracle (tc3d_oracle.c).

TEST INFRASTRUCTURE: imported only by the test suite, the smoke check and the
CPU-baseline leg of the benchmark. The oracle follows the paper's definitions
one shot at a time (uint8 bits, FP64 belief propagation) and shares no code
with the GPU library.

Arrays are numpy, C-contiguous, shaped [shot][site].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tc3d_oracle.c")
LIB_PATH = os.path.join(_HERE, "libtc3d_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math), again whenever
    its source or header is newer than the library."""
    hdr = os.path.splitext(_SRC)[0] + ".h"
    stale = not os.path.exists(LIB_PATH) or max(os.path.getmtime(_SRC), os.path.getmtime(hdr)) > \
        os.path.getmtime(LIB_PATH)
    if force or stale:
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
             _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_double), ("q", ctypes.c_double),
        ("p_dec", ctypes.c_double), ("q_dec", ctypes.c_double),
        ("noisy_cycles", ctypes.c_int32), ("perfect_final", ctypes.c_int32),
        ("final_qubit_noise", ctypes.c_int32), ("bp_iters", ctypes.c_int32),
        ("n_sweeps", ctypes.c_int32), ("pflip_mask", ctypes.c_uint32),
        ("seed", ctypes.c_uint64), ("subset_mask", ctypes.c_uint32),
        ("bp_meta", ctypes.c_int32), ("cycle0", ctypes.c_uint32),
        ("bp_warm", ctypes.c_int32), ("bp_damp", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
        sig = {
            "tco_lattice_new": (vp, [i32]),
            "tco_lattice_free": (None, [vp]),
            "tco_n_edges": (i64, [vp]),
            "tco_incidence": (None, [vp, vp, vp, vp]),
            "tco_philox4x32_10": (None, [vp, vp, vp]),
            "tco_threshold": (u64, [f64]),
            "tco_uniform": (u32, [u64, u32, u32, u64, u32]),
            "tco_coin": (ctypes.c_int, [u64, u32, u32, u32, u64]),
            "tco_sample_noise": (None, [vp, vp, i32, f64, u64, u32, u64, i64]),
            "tco_syndrome": (None, [vp, vp, vp, i64, i32]),
            "tco_flip_sweep": (None, [vp, vp, vp, i64]),
            "tco_pflip_sweep": (None, [vp, vp, vp, u64, u32, u32, u64, i64]),
            "tco_edge_class": (i32, [vp, i64]),
            "tco_bp_meta_step": (None, [vp, vp, f64, f64, vp, vp, vp, vp, vp, vp, vp]),
            "tco_bp_meta_decode": (None, [vp, vp, i64, f64, f64, i32, vp, vp]),
            "tco_subset_class": (i32, [i32, i32, u32]),
            "tco_subset_pflip_sweep": (None, [vp, vp, vp, u64, u32, u32, u64, i64, i32]),
            "tco_pflip_sweep_coins": (None, [vp, vp, vp, vp]),
            "tco_sequential_flip": (i64, [vp, vp, vp, i64]),
            "tco_bp_step": (None, [vp, vp, vp, f64, f64, vp, vp, vp]),
            "tco_bp_step_damped": (None, [vp, vp, vp, f64, f64, f64, vp, vp, vp]),
            "tco_bp_decode": (None, [vp, vp, i64, vp, f64, f64, i32, vp, vp]),
            "tco_logical_check": (None, [vp, vp, i64, vp, vp]),
            "tco_run_cycles": (None, [vp, ctypes.POINTER(Params), u64, i64, vp, vp, vp, vp]),
            "tco_cnn_param_count": (i64, []),
            "tco_cnn_input": (None, [vp, i64, vp, vp, vp]),
            "tco_cnn_forward": (None, [vp, i64, vp, vp, vp, vp]),
            "tco_cnn_loss_grad": (ctypes.c_double, [vp, i64, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _chk(a, dtype, shape=None):
    assert isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous, (
        a.dtype, dtype)
    if shape is not None:
        assert a.shape == tuple(shape), (a.shape, shape)
    return a


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().tco_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def threshold(prob: float) -> int:
    return int(lib().tco_threshold(float(prob)))


def uniform(seed, site, cycle, shot, tag) -> int:
    return int(lib().tco_uniform(seed, site, cycle, shot, tag))


def coin(seed, edge, cycle, sweep, shot) -> int:
    return int(lib().tco_coin(seed, edge, cycle, sweep, shot))


class Oracle:
    """The oracle on one lattice size L."""

    def __init__(self, L: int):
        self.L = int(L)
        self.n_sites = self.L ** 3
        self.n_edges = 3 * self.n_sites
        self.n_faces = 3 * self.n_sites
        self._h = lib().tco_lattice_new(self.L)
        if not self._h:
            raise ValueError(f"bad lattice size {L}")

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.tco_lattice_free(h)

    # geometry ---------------------------------------------------------------
    def incidence(self):
        fe = np.zeros((self.n_faces, 4), np.int32)
        ef = np.zeros((self.n_edges, 4), np.int32)
        es = np.zeros((self.n_edges, 4), np.int32)
        lib().tco_incidence(self._h, _p(fe), _p(ef), _p(es))
        return fe, ef, es

    # stages -------------------------------------------------------------------
    def sample_noise(self, bits, kind, prob, seed, cycle, shot0=0):
        n = self.n_edges if kind == 0 else self.n_faces
        _chk(bits, np.uint8)
        assert bits.shape[-1] == n
        S = bits.size // n
        lib().tco_sample_noise(self._h, _p(bits), kind, prob, seed, cycle, shot0, S)
        return bits

    def syndrome(self, err, syn=None, xor_into=False):
        _chk(err, np.uint8)
        S = err.size // self.n_edges
        if syn is None:
            syn = np.zeros((S, self.n_faces), np.uint8)
        _chk(syn, np.uint8)
        lib().tco_syndrome(self._h, _p(err), _p(syn), S, 1 if xor_into else 0)
        return syn

    def flip_sweep(self, syn, corr):
        _chk(syn, np.uint8)
        _chk(corr, np.uint8)
        S = syn.size // self.n_faces
        lib().tco_flip_sweep(self._h, _p(syn), _p(corr), S)

    def pflip_sweep(self, syn, corr, seed, cycle, sweep, shot0=0):
        _chk(syn, np.uint8)
        _chk(corr, np.uint8)
        S = syn.size // self.n_faces
        lib().tco_pflip_sweep(self._h, _p(syn), _p(corr), seed, cycle, sweep, shot0, S)

    def edge_class(self, edge):
        return int(lib().tco_edge_class(self._h, int(edge)))

    def subset_pflip_sweep(self, syn, corr, seed, cycle, sweep, edge_class, shot0=0):
        _chk(syn, np.uint8)
        _chk(corr, np.uint8)
        S = syn.size // self.n_faces
        lib().tco_subset_pflip_sweep(self._h, _p(syn), _p(corr), seed, cycle, sweep, shot0, S,
                                     int(edge_class))

    def pflip_sweep_coins(self, syn, corr, coins):
        _chk(syn, np.uint8, (self.n_faces,))
        _chk(corr, np.uint8, (self.n_edges,))
        _chk(coins, np.uint8, (self.n_edges,))
        lib().tco_pflip_sweep_coins(self._h, _p(syn), _p(corr), _p(coins))

    def sequential_flip(self, syn, corr, max_flips=1 << 30):
        _chk(syn, np.uint8, (self.n_faces,))
        _chk(corr, np.uint8, (self.n_edges,))
        return int(lib().tco_sequential_flip(self._h, _p(syn), _p(corr), max_flips))

    def bp_step(self, syn, p_dec, q_dec, nu_in=None, llr0=None):
        _chk(syn, np.uint8, (self.n_faces,))
        if nu_in is not None:
            _chk(nu_in, np.float64, (self.n_faces, 4))
        if llr0 is not None:
            _chk(llr0, np.float64, (self.n_edges,))
        nu_out = np.zeros((self.n_faces, 4), np.float64)
        post = np.zeros(self.n_edges, np.float64)
        lib().tco_bp_step(self._h, _p(syn), _p(llr0), p_dec, q_dec, _p(nu_in), _p(nu_out),
                          _p(post))
        return nu_out, post

    def bp_step_damped(self, syn, p_dec, q_dec, damp, nu_in=None):
        _chk(syn, np.uint8, (self.n_faces,))
        if nu_in is not None:
            _chk(nu_in, np.float64, (self.n_faces, 4))
        nu_out = np.zeros((self.n_faces, 4), np.float64)
        post = np.zeros(self.n_edges, np.float64)
        lib().tco_bp_step_damped(self._h, _p(syn), None, p_dec, q_dec, damp, _p(nu_in),
                                 _p(nu_out), _p(post))
        return nu_out, post

    def bp_decode(self, syn, p_dec, q_dec, iters, llr0=None):
        _chk(syn, np.uint8)
        S = syn.size // self.n_faces
        if llr0 is not None:
            _chk(llr0, np.float64, (S, self.n_edges))
        corr = np.zeros((S, self.n_edges), np.uint8)
        post = np.zeros((S, self.n_edges), np.float64)
        lib().tco_bp_decode(self._h, _p(syn), S, _p(llr0), p_dec, q_dec, iters, _p(corr),
                            _p(post))
        return corr, post

    def bp_meta_step(self, syn, p_dec, q_dec, state=None):
        """One meta-check BP iteration of one shot; state = (nu [m][4],
        lambda [m], kappa [N][6]) or None for the first. Returns (state, post)."""
        _chk(syn, np.uint8, (self.n_faces,))
        nu = np.zeros((self.n_faces, 4), np.float64)
        lam = np.zeros(self.n_faces, np.float64)
        kap = np.zeros((self.n_sites, 6), np.float64)
        post = np.zeros(self.n_edges, np.float64)
        if state is None:
            a = b = c = None
        else:
            a, b, c = (np.ascontiguousarray(x, np.float64) for x in state)
            assert a.shape == nu.shape and b.shape == lam.shape and c.shape == kap.shape
        lib().tco_bp_meta_step(self._h, _p(syn), p_dec, q_dec, _p(a), _p(b), _p(c), _p(nu),
                               _p(lam), _p(kap), _p(post))
        return (nu, lam, kap), post

    def bp_meta_decode(self, syn, p_dec, q_dec, iters):
        _chk(syn, np.uint8)
        S = syn.size // self.n_faces
        corr = np.zeros((S, self.n_edges), np.uint8)
        post = np.zeros((S, self.n_edges), np.float64)
        lib().tco_bp_meta_decode(self._h, _p(syn), S, p_dec, q_dec, iters, _p(corr), _p(post))
        return corr, post

    def logical_check(self, err):
        _chk(err, np.uint8)
        S = err.size // self.n_edges
        mask = np.zeros(S, np.uint8)
        odd = np.zeros((S, 3), np.int32)
        lib().tco_logical_check(self._h, _p(err), S, _p(mask), _p(odd))
        return mask, odd

    def run_cycles(self, params: Params, n_shots: int, shot0: int = 0, err=None,
                   trace=False):
        if err is None:
            err = np.zeros((n_shots, self.n_edges), np.uint8)
        _chk(err, np.uint8, (n_shots, self.n_edges))
        mask = np.zeros(n_shots, np.uint8)
        odd = np.zeros((n_shots, 3), np.int32)
        cycles = params.noisy_cycles + (1 if params.perfect_final else 0)
        tr = np.zeros((cycles, n_shots, self.n_edges), np.uint8) if trace else None
        lib().tco_run_cycles(self._h, ctypes.byref(params), shot0, n_shots, _p(err), _p(mask),
                             _p(odd), _p(tr))
        return (mask, odd, err, tr) if trace else (mask, odd, err)


# CNN prior --------------------------------------------------------------------
CNN_CHANNELS = (8, 32, 32, 32, 3)


def cnn_param_count() -> int:
    return int(lib().tco_cnn_param_count())


def cnn_layers(params: np.ndarray):
    """Views (W [27][cin][cout], b [cout]) of each layer in a parameter vector."""
    out, o = [], 0
    for cin, cout in zip(CNN_CHANNELS[:-1], CNN_CHANNELS[1:]):
        W = params[o:o + 27 * cin * cout].reshape(27, cin, cout)
        o += 27 * cin * cout
        b = params[o:o + cout]
        o += cout
        out.append((W, b))
    return out


def _cnn_methods():
    def cnn_input(self, syn, prev=None):
        _chk(syn, np.uint8)
        S = syn.size // self.n_faces
        x0 = np.zeros((S, self.n_sites, 8), np.float64)
        lib().tco_cnn_input(self._h, S, _p(syn), _p(prev), _p(x0))
        return x0

    def cnn_forward(self, x0, params, with_acts=False):
        _chk(x0, np.float64)
        _chk(params, np.float64, (cnn_param_count(),))
        S = x0.size // (self.n_sites * 8)
        z = np.zeros((S, self.n_sites, 3), np.float64)
        acts = np.zeros((3, S, self.n_sites, 32), np.float64) if with_acts else None
        lib().tco_cnn_forward(self._h, S, _p(x0), _p(params), _p(z), _p(acts))
        return (z, acts) if with_acts else z

    def cnn_loss_grad(self, x0, params, target):
        _chk(x0, np.float64)
        _chk(params, np.float64, (cnn_param_count(),))
        _chk(target, np.uint8)
        S = x0.size // (self.n_sites * 8)
        grad = np.zeros(cnn_param_count(), np.float64)
        loss = lib().tco_cnn_loss_grad(self._h, S, _p(x0), _p(params), _p(target), _p(grad))
        return float(loss), grad

    Oracle.cnn_input = cnn_input
    Oracle.cnn_forward = cnn_forward
    Oracle.cnn_loss_grad = cnn_loss_grad


_cnn_methods()


def make_params(p, q, noisy_cycles, bp_iters, n_sweeps, pflip_mask, seed=1, p_dec=None,
                q_dec=None, perfect_final=1, final_qubit_noise=1, subset_mask=0,
                bp_meta=0, cycle0=0, bp_warm=0, bp_damp=0.0) -> Params:
    return Params(p=p, q=q, p_dec=p if p_dec is None else p_dec,
                  q_dec=q if q_dec is None else q_dec, noisy_cycles=noisy_cycles,
                  perfect_final=perfect_final, final_qubit_noise=final_qubit_noise,
                  bp_iters=bp_iters, n_sweeps=n_sweeps, pflip_mask=pflip_mask, seed=seed,
                  subset_mask=subset_mask, bp_meta=bp_meta, cycle0=cycle0, bp_warm=bp_warm,
                  bp_damp=bp_damp)


def subset_class(j, m, cycle):
    """Edge class of the j-th subset sweep (of m per cycle) in cycle `cycle`."""
    return int(lib().tco_subset_class(int(j), int(m), int(cycle)))
