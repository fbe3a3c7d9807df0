"""Train the CNN prior for BP on the GPU with data the simulator generates.

Every training step is one simulated code cycle of a batch of shots: noise,
syndrome measurement (this cycle's syndrome and the previous cycle's final
working syndrome are the network input, the error before decoding is the
target), one forward + backward pass and one Adam step, then the cycle is
decoded (by the paper's p-BP, or by the CNN-prior decoder itself in the
on-policy phase) and the residual carries over. After `cycles` cycles a fresh
batch of shots starts. Everything runs in the library's kernels; the initial
weights are drawn on the host from a seeded generator.

    python -m paper_2212_06985_amd.train_cnn --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import paper_2212_06985_amd as tc  # noqa: E402

CHANNELS = (8, 32, 32, 32, 3)


def init_params(seed: int, p: float) -> np.ndarray:
    """He-normal weights, zero biases; the output bias starts at the channel
    prior's logit so that the untrained network gives BP the paper's prior."""
    rng = np.random.default_rng(seed)
    out = []
    for li, (cin, cout) in enumerate(zip(CHANNELS[:-1], CHANNELS[1:])):
        W = rng.normal(0.0, math.sqrt(2.0 / (27 * cin)), size=(27, cin, cout))
        if li == 3:
            W *= 0.1
        b = np.zeros(cout)
        if li == 3:
            b[:] = math.log(p / (1 - p))
        out += [W.ravel(), b]
    return np.concatenate(out).astype(np.float32)


def packed_prior(params: np.ndarray, beta: float, p: float):
    """Device copy of a network in the kernels' packed layout, its prior
    blended with the channel prior of error rate p at strength beta (by the
    library's packing kernel): llr0 = l0 + beta (llr_cnn - l0). beta = 0 gives
    the paper's decoder, beta = 1 the network as trained."""
    import torch
    d = torch.from_numpy(np.ascontiguousarray(params, np.float32)).cuda()
    packed = torch.zeros(tc.cnn_packed_bytes(), dtype=torch.uint8, device="cuda")
    tc.cnn_pack(d, packed, beta=beta, p=p)
    return packed


class Trainer:
    def __init__(self, L, shots, p, q, seed, params=None):
        import torch
        self.torch = torch
        self.L, self.S, self.p, self.q, self.seed = L, shots, p, q, seed
        self.lat = tc.make_lattice(L)
        self.W = tc.n_words(shots)
        n = self.lat.n_edges
        dev = "cuda"
        p0 = init_params(seed, p) if params is None else np.asarray(params, np.float32)
        self.params = torch.from_numpy(p0.copy()).to(dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.packed = torch.zeros(tc.cnn_packed_bytes(), dtype=torch.uint8, device=dev)
        self.packed_dec = torch.zeros_like(self.packed)  # blended, for on-policy decoding
        tc.cnn_pack(self.params, self.packed)
        self.err = torch.zeros((n, self.W), dtype=torch.int64, device=dev)
        self.syn = torch.zeros_like(self.err)
        self.prev = torch.zeros_like(self.err)
        self.corr = torch.zeros_like(self.err)
        self.llr = torch.zeros((self.W, n, 64), dtype=torch.float32, device=dev)
        self.ws_train = tc.alloc_workspace(tc.cnn_workspace_bytes(self.lat, shots, training=True))
        self.ws_bp = tc.alloc_workspace(tc.bp_workspace_bytes(self.lat, shots))
        self.ws_sw = tc.alloc_workspace(tc.sweep_workspace_bytes(self.lat, self.W))
        self.step = 0
        self.batch = 0
        self.t = 0

    def new_batch(self, p=None):
        """Start a fresh batch of shots (error rate p = q, or unchanged)."""
        self.err.zero_()
        self.t = 0
        self.batch += 1
        if p is not None:
            self.p = self.q = float(p)

    def train_cycle(self, lr, on_policy=False, n_sweeps=6, mask=0b001001, bp_iters=20,
                    beta=1.0):
        """One training step on one simulated cycle of the current batch."""
        L, S, W, lat = self.L, self.S, self.W, self.lat
        shot0 = 64 * W * self.batch
        seed = self.seed
        tc.sample_noise(lat, self.err, 0, self.p, seed, self.t, shot0, S)
        tc.syndrome(lat, self.err, self.syn, W)
        tc.sample_noise(lat, self.syn, 1, self.q, seed, self.t, shot0, S)
        prev = None if self.t == 0 else self.prev
        # one gradient step on (syndrome, previous working syndrome) -> error
        tc.cnn_loss_grad(lat, self.syn, prev, self.err, S, self.packed, self.llr, self.grad,
                         self.loss, self.ws_train)
        self.step += 1
        tc.cnn_adam(self.params, self.grad, self.m, self.v, self.step, lr, self.packed)
        # decode this cycle and carry the residual
        if on_policy:  # priors of the updated network, blended as when decoding
            tc.cnn_pack(self.params, self.packed_dec, beta=beta, p=self.p)
            tc.cnn_forward(lat, self.syn, prev, S, self.packed_dec, self.llr, self.ws_train)
            llr = self.llr
        else:
            llr = None
        l0 = math.log((1 - self.p) / self.p)
        tc.bp_decode(lat, self.syn, S, llr, l0, 1 - 2 * self.q, bp_iters, self.corr, None,
                     self.ws_bp)
        tc.syndrome(lat, self.corr, self.syn, W, xor_into=True)
        for k in range(n_sweeps):
            if (mask >> k) & 1:
                tc.pflip_sweep(lat, self.syn, self.corr, W, seed, self.t, k, shot0, self.ws_sw)
            else:
                tc.flip_sweep(lat, self.syn, self.corr, W, self.ws_sw)
        self.prev.copy_(self.syn)
        tc.apply_correction(lat, self.err, self.corr, W)
        self.t += 1

    def params_numpy(self):
        return self.params.cpu().numpy().copy()


def train(L=12, shots=4096, p=0.05, cycles=13, snapshots=10_000_000, on_policy_frac=0.2,
          lr_max=2e-3, lr_min=5e-5, seed=12345, log=print, p_max=None, on_policy_iters=20,
          on_policy_beta=1.0):
    """p_max: draw each batch's error rate uniformly from [p, p_max] (seeded)."""
    steps = max(1, snapshots // shots)
    tr = Trainer(L, shots, p, p, seed)
    rng = np.random.default_rng(seed + 1)
    t0 = time.perf_counter()
    history = []
    for step in range(steps):
        if tr.t == cycles:
            tr.new_batch(None if p_max is None else rng.uniform(p, p_max))
        frac = step / max(1, steps - 1)
        lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + math.cos(math.pi * frac))
        on = frac >= 1.0 - on_policy_frac
        tr.train_cycle(lr, on_policy=on, bp_iters=on_policy_iters if on else 20,
                       beta=on_policy_beta)
        if step % 100 == 0 or step == steps - 1:
            loss = float(tr.loss.item())
            history.append((step, loss))
            log(f"[train] step {step}/{steps} cycle {tr.t} lr {lr:.2e} loss {loss:.5f} "
                f"{time.perf_counter() - t0:.1f}s")
    tr.torch.cuda.synchronize()
    return tr, history, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="where to write the FP32 parameters (.npy)")
    ap.add_argument("--L", type=int, default=12)
    ap.add_argument("--shots", type=int, default=4096)
    ap.add_argument("--p", type=float, default=0.05)
    ap.add_argument("--cycles", type=int, default=13)
    ap.add_argument("--snapshots", type=int, default=10_000_000)
    ap.add_argument("--seed", type=int, default=12345)
    ap.add_argument("--p-max", type=float, default=None,
                    help="draw each batch's p = q uniformly from [p, p_max]")
    ap.add_argument("--on-policy-frac", type=float, default=0.2,
                    help="last fraction of steps that decode with the network being trained")
    ap.add_argument("--on-policy-iters", type=int, default=20,
                    help="BP iterations of that decoder")
    ap.add_argument("--on-policy-beta", type=float, default=1.0,
                    help="prior strength of that decoder (see packed_prior)")
    args = ap.parse_args()
    tr, hist, secs = train(args.L, args.shots, args.p, args.cycles, args.snapshots,
                           args.on_policy_frac, seed=args.seed,
                           log=lambda m: print(m, flush=True), p_max=args.p_max,
                           on_policy_iters=args.on_policy_iters,
                           on_policy_beta=args.on_policy_beta)
    np.save(args.out, tr.params_numpy(), allow_pickle=False)
    print(json.dumps({"out": args.out, "seconds": secs, "steps": tr.step,
                      "snapshots": tr.step * args.shots, "final_loss": hist[-1][1]}), flush=True)


if __name__ == "__main__":
    main()
