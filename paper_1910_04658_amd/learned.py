"""Learned Jaccard estimator: data, training and evaluation drivers.

A 4 -> 64 -> 64 -> 1 network (BF16 weights, FP32 accumulation) corrects the
closed-form Jaccard estimate (Algorithms 1-3) from the three sketch counts of
a pair and the width N, where sketches saturate. Everything that touches the
data runs in the library's kernels: bs_sketch for the sketches,
bs_pair_popcount for |a_s|, |b_s| and |a_s AND b_s|, bs_mlp_train_step for the
forward, backward and Adam step, bs_mlp_forward for inference. This module
only moves tensors between those calls (batch slices, one shuffle).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import binding as bs

H = 64


@dataclasses.dataclass
class PairCounts:
    xa: torch.Tensor     # int32[n] |a_s|
    xb: torch.Tensor     # int32[n] |b_s|
    xab: torch.Tensor    # int32[n] |a_s AND b_s|
    label: torch.Tensor  # float32[n] exact Jaccard
    N: int

    def __len__(self):
        return self.xa.numel()

    def slice(self, lo, hi):
        return PairCounts(self.xa[lo:hi], self.xb[lo:hi], self.xab[lo:hi], self.label[lo:hi], self.N)


def sketch_pairs(pairs, pi: np.ndarray, N: int, device) -> PairCounts:
    """Sketch every vector of a datagen.PairSet and count each listed pair."""
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
    words, _ = bs.sketch(to(pairs.csr.indptr), to(pairs.csr.indices), to(pi), N)
    ia, ib = to(pairs.ia.astype(np.int32)), to(pairs.ib.astype(np.int32))
    xa = bs.pair_popcount(words, ia, words, ia, N)    # |a_s AND a_s| = |a_s|
    xb = bs.pair_popcount(words, ib, words, ib, N)
    xab = bs.pair_popcount(words, ia, words, ib, N)
    label = to(pairs.jaccard.astype(np.float32))
    return PairCounts(xa, xb, xab, label, N)


def init_master(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-uniform hidden layers, zero output layer (the untrained network
    returns the closed form), as a float32[4545] master vector."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H, 4)) * math.sqrt(6.0 / 4)
    W2 = rng.uniform(-1, 1, (H, H)) * math.sqrt(6.0 / H)
    theta = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), np.zeros(H), np.zeros(1)])
    return torch.from_numpy(theta.astype(np.float32)).to(device)


class Model:
    """FP32 master weights, their BF16 copy and Adam moments, all on the device."""

    def __init__(self, master: torch.Tensor):
        n = bs.mlp_param_count()
        assert master.numel() == n
        self.master = master.contiguous().clone()
        self.w = torch.empty(n, dtype=torch.int16, device=master.device)
        self.m = torch.zeros(n, dtype=torch.float32, device=master.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=master.device)
        self.step = 0
        bs.mlp_to_bf16(self.master, self.w)

    def train(self, data: PairCounts, steps: int, batch: int, lr: float = 3e-3, lr_min: float = 3e-4,
              seed: int = 0, log_every: int = 0):
        """Adam on shuffled contiguous batches with a cosine learning-rate decay."""
        g = torch.Generator(device=data.xa.device)
        g.manual_seed(seed)
        n = len(data)
        perm = torch.randperm(n, generator=g, device=data.xa.device)
        d = PairCounts(data.xa[perm].contiguous(), data.xb[perm].contiguous(), data.xab[perm].contiguous(),
                       data.label[perm].contiguous(), data.N)
        batch = min(batch, n)
        ws = bs.mlp_workspace(batch, data.N, data.xa.device)
        loss = torch.zeros(1, dtype=torch.float32, device=data.xa.device)
        losses = []
        nb = max(1, n // batch)
        for t in range(steps):
            k = t % nb
            b = d.slice(k * batch, (k + 1) * batch)
            self.step += 1
            lr_t = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * t / max(1, steps - 1)))
            bs.mlp_train_step(self.master, self.w, self.m, self.v, self.step, lr_t, b.xa, b.xb, b.xab,
                              b.label, data.N, loss=loss, workspace=ws)
            if log_every and (t % log_every == 0 or t == steps - 1):
                losses.append((t, float(loss.item())))
        return losses

    def predict(self, data: PairCounts) -> torch.Tensor:
        return bs.mlp_forward(self.w, data.xa, data.xb, data.xab, data.N)


def closed_form(data: PairCounts) -> torch.Tensor:
    """The closed-form Jaccard estimate (clamped to [0, 1]): the network with a
    zero output layer."""
    zero = torch.zeros(bs.mlp_param_count(), dtype=torch.int16, device=data.xa.device)
    return bs.mlp_forward(zero, data.xa, data.xb, data.xab, data.N)


def mse(pred: torch.Tensor, data: PairCounts) -> float:
    return float(torch.mean((pred.double() - data.label.double()) ** 2).item())
