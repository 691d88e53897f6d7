"""Element-wise error bounds for the learned estimator's GPU forward pass and
gradient against the FP64 oracle (oracle/mlp.py).

The GPU evaluates the same model in FP32 with BF16 operands at the same
rounding points, so the two differ only by
  (a) FP32 rounding of the intermediates. The features f = x/N are exact for
      power-of-two N, and the closed-form base is the same IEEE float
      expression on both sides (one float ulp is allowed for it all the same);
  (b) FP32 accumulation of the batch sums. Summing n terms in FP32 in any
      order (any tree) is within (n - 1) ulp-sized steps of the exact sum:
      |error| <= (n - 1) * 2u * sum|terms| with u = 2^-24 (Higham, "Accuracy
      and Stability of Numerical Algorithms", 2nd ed., Section 4.2; 2u rather
      than u per step also covers a matrix-core accumulator that does not
      round to nearest). The chains inside one term (a 64-term sum for z2 and
      dh1, a few products) add at most 96 more such steps;
  (c) discrete decisions taken on FP32 values that lie within their FP32
      error of a boundary: a BF16 rounding of h1 or dz2 that goes to the other
      neighbour, or a ReLU mask of z1 or z2 that flips.
The bound of gradient element j is therefore
  2u (n + 96) S_j + E_j + F_j,
where S_j is the backward pass of element j with every operand in absolute
value (the sum of |terms|), E_j carries the absolute error of dL/dy (which
suffers the cancellation in p - label) through that same absolute backward
pass, and F_j adds, to first order, the change each operand within its error
radius of a boundary makes when it is taken as flipped. The forward bound is
the error radius of p = base + w3 . relu(z2) + b3 built the same way.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp

U = 2.0 ** -24


def bf16_ulp(v):
    """Spacing of BF16 values at |v| (8 significant bits); 0 for v = 0."""
    a = np.abs(v)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    return np.where(a > 0, 2.0 ** (e - 7), 0.0)


def near_bf16_midpoint(v, radius):
    """True where v lies within `radius` of a point at which rounding to BF16
    changes its result (the midpoint between two BF16 neighbours)."""
    ulp = bf16_ulp(v)
    safe = np.where(ulp > 0, ulp, 1.0)
    frac = np.abs(v) / safe
    dist = np.abs(frac - np.floor(frac) - 0.5) * ulp
    return (ulp > 0) & (dist <= radius)


def abs_backward(w, P, af, ah1, m1, ah2, m2):
    """sum_n w_n |dy_n/dtheta| with every operand in absolute value (w_n >= 0):
    the backward pass of the network output, all terms taken positive."""
    aw3 = np.abs(P["w3"])
    gz2 = w[:, None] * aw3[None, :] * m2
    g = {"b3": np.sum(w), "w3": ah2.T @ w, "b2": gz2.sum(0), "W2": gz2.T @ ah1}
    gz1 = (gz2 @ np.abs(P["W2"])) * m1
    g["b1"] = gz1.sum(0)
    g["W1"] = gz1.T @ af
    return mlp.pack(g)


class Bounds:
    """Oracle values (BF16 rounding points, FP64) of one batch, and the
    largest difference the FP32 GPU evaluation may show from each."""

    def __init__(self, theta, xa, xb, xab, label, N):
        P = mlp.unpack(theta)
        n = len(xa)
        base = mlp.closed_form(xa, xb, xab, N)
        p, c = mlp.forward(theta, xa, xb, xab, N, bf16=True, base=base)
        self.loss, self.grad = mlp.loss_and_grad(theta, xa, xb, xab, label, N, bf16=True, base=base)
        self.p = p
        f, z1, h1q, z2, h2 = c["f"], c["z1"], c["h1q"], c["z2"], c["h2"]
        t = np.asarray(label, np.float64)
        af, aW1, aW2, aw3 = np.abs(f), np.abs(P["W1"]), np.abs(P["W2"]), np.abs(P["w3"])
        m1 = (z1 > 0).astype(np.float64)
        m2 = (z2 > 0).astype(np.float64)
        # error radii of the pre-activations: z1 is 4 FMAs; z2 a 64-term sum
        rz1 = 16 * U * (af @ aW1.T + np.abs(P["b1"]))
        # h1: a BF16 rounding near a midpoint or a ReLU decision near zero
        amb1 = near_bf16_midpoint(np.maximum(z1, 0.0), rz1) | (np.abs(z1) <= rz1)
        dh1 = np.where(amb1, bf16_ulp(np.maximum(np.abs(z1), rz1)) + rz1, 0.0)
        rz2 = 160 * U * (np.abs(h1q) @ aW2.T + np.abs(P["b2"])) + dh1 @ aW2.T
        amb2 = np.abs(z2) <= rz2
        # forward: h2 = relu(z2) is within rz2 of the oracle's (a flipped mask
        # included); y = w3 . h2 + b3; p = base + y (one float ulp of the base)
        self.p_bound = rz2 @ aw3 + 160 * U * (np.abs(h2) @ aw3 + abs(P["b3"])) + \
            4 * U * (np.abs(base) + np.abs(p))
        # dL/dy = 2 (p - label) / n and its absolute error
        r = p - t
        dr = self.p_bound + 2 * U * (np.abs(p) + np.abs(t))
        gy = 2.0 * r / n
        dgy = 2.0 * dr / n + 4 * U * np.abs(gy)
        self.loss_bound = float(np.sum(2 * np.abs(r) * dr + dr * dr)) / n + 2 * U * (n + 8) * self.loss
        # dz2 = gy w3 (z2 > 0): its BF16 rounding near a midpoint, or a mask
        # flip (the whole value)
        gz2 = np.outer(gy, P["w3"]) * m2
        rg2 = np.outer(dgy, aw3) + 4 * U * np.abs(gz2)
        whole = np.abs(np.outer(gy, P["w3"])) + rg2
        d_g2q = np.where(near_bf16_midpoint(gz2, rg2) & (m2 > 0), bf16_ulp(np.abs(gz2) + rg2), 0.0) + \
            np.where(amb2, whole * (1 + 2.0 ** -7), 0.0)
        # dz1 = (bf16(dz2) W2) (z1 > 0): the dz2 changes, and z1 mask flips
        gh1 = mlp.bf16_round(gz2) @ P["W2"]
        d_gz1 = (d_g2q @ aW2) * np.maximum(m1, amb1) + np.where(np.abs(z1) <= rz1, np.abs(gh1), 0.0)
        agz2q = np.abs(mlp.bf16_round(gz2))
        F = {"b3": 0.0, "w3": np.abs(gy) @ rz2, "b2": np.where(amb2, whole, 0.0).sum(0),
             "W2": d_g2q.T @ (np.abs(h1q) + dh1) + agz2q.T @ dh1,
             "b1": d_gz1.sum(0), "W1": d_gz1.T @ af}
        m1x, m2x = np.maximum(m1, amb1), np.maximum(m2, amb2)
        ah1, ah2 = np.abs(h1q) + dh1, np.abs(h2) + rz2
        S = abs_backward(np.abs(gy) + dgy, P, af, ah1, m1x, ah2, m2x)
        E = abs_backward(dgy, P, af, ah1, m1x, ah2, m2x)
        self.grad_bound = 2 * U * (n + 96) * S + E + mlp.pack(F)
