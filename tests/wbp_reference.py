"""Plain-PyTorch (CPU) unrolled weighted min-sum with damping: the autograd
reference for the weighted decoder's gradients.  Test infrastructure only.

The forward map of one representation [H; H_t] (flooding schedule):
  q^(0) = mu on every edge, r^(0) = 0,
  r^(t) = clamp((1 - beta_t) * S * (alpha_t * M) + beta_t * r^(t-1))   for t = 1..T,
    M the smallest |q^(t-1)| over the row's other edges, S the product of their
    signs and of (-1)^{s_j},
  q^(t) = mu + the other checks' r^(t) (exclusion sums, ascending check order),
  P^(T) = mu + the sum of r^(T) over the variable's checks.
Operations are written in the order a single-precision decoder evaluates them, so
float32 forward values can be compared bit for bit; gradients come from
autograd.  Subgradient conventions: |x| = where(x < 0, -x, x) (derivative +1 at
0), the minimum over the other slots by torch.min along the row (the first index
among equal values, in the row's column order), sign factors constant, the clamp
passes the gradient only strictly inside (-rmax, rmax).
"""

from __future__ import annotations

import numpy as np
import torch


class Rep:
    """Edge tables of one representation: H plus the appended copies of H rows."""

    def __init__(self, h: np.ndarray, rows):
        h = np.asarray(h, np.uint8)
        rows = np.asarray(rows, np.int64)
        m, n = h.shape
        aug = np.vstack([h, h[rows]]) if rows.size else h.copy()
        self.m, self.n, self.M = m, n, aug.shape[0]
        self.src = np.concatenate([np.arange(m), rows]).astype(np.int64)
        cols = [np.flatnonzero(aug[j]) for j in range(self.M)]
        self.dmax = max(len(c) for c in cols)
        E = int(sum(len(c) for c in cols))
        self.E = E
        cedge = np.full((self.M, self.dmax), E, np.int64)
        cmask = np.zeros((self.M, self.dmax), bool)
        evar = np.zeros(E, np.int64)
        vedges = [[] for _ in range(n)]
        e = 0
        for j, c in enumerate(cols):
            for k, v in enumerate(c):
                cedge[j, k] = e
                cmask[j, k] = True
                evar[e] = v
                vedges[v].append(e)
                e += 1
        self.dvmax = max(len(v) for v in vedges)
        vedge = np.full((n, self.dvmax), E, np.int64)
        vmask = np.zeros((n, self.dvmax), bool)
        for v in range(n):
            vedge[v, : len(vedges[v])] = vedges[v]
            vmask[v, : len(vedges[v])] = True
        self.cedge = torch.as_tensor(cedge)
        self.cmask = torch.as_tensor(cmask)
        self.evar = torch.as_tensor(evar)
        self.vedge = torch.as_tensor(vedge)
        self.vmask = torch.as_tensor(vmask)
        self.vperm = torch.as_tensor(vedge[vmask])  # edge id of every (variable, slot) in row-major order


def forward(rep: Rep, syn_bits: np.ndarray, mu: torch.Tensor, alpha: torch.Tensor, beta: torch.Tensor,
            T: int, rmax: float = 65536.0) -> torch.Tensor:
    """P^(T) [shots, n] for syndromes syn_bits (0/1 [shots, m]); mu [n] or [shots, n];
    alpha, beta [T] of this representation (iteration t at index t - 1)."""
    dt = mu.dtype
    S = syn_bits.shape[0]
    n, E = rep.n, rep.E
    sb = torch.as_tensor(np.asarray(syn_bits, np.uint8)[:, rep.src].astype(bool))
    mu_s = mu.expand(S, n) if mu.dim() == 1 else mu
    inf = torch.full((S, 1), float("inf"), dtype=dt)
    zero = torch.zeros((S, 1), dtype=dt)
    R = torch.tensor(rmax, dtype=dt)
    q = mu_s[:, rep.evar]
    r = torch.zeros((S, E), dtype=dt)
    P = mu_s
    eye = torch.eye(rep.dmax, dtype=torch.bool)
    for t in range(T):
        qrow = torch.cat([q, inf], 1)[:, rep.cedge]
        neg = qrow < 0
        a = torch.where(neg, -qrow, qrow)
        parity = (neg.sum(-1) % 2 == 1) ^ sb
        rprev = torch.cat([r, zero], 1)[:, rep.cedge]
        keep = 1 - beta[t]
        cols = []
        for k in range(rep.dmax):
            mk, _ = torch.where(eye[k], torch.full_like(a, float("inf")), a).min(dim=-1)
            u = alpha[t] * mk
            v = torch.where(parity ^ neg[..., k], -u, u)
            w = keep * v + beta[t] * rprev[..., k]
            inside = (w > -R) & (w < R)
            cols.append(torch.where(inside, w, torch.where(w >= R, R, -R)))
        r = torch.stack(cols, -1)[:, rep.cmask]
        rv = torch.cat([r, zero], 1)[:, rep.vedge]
        P = mu_s
        for k in range(rep.dvmax):
            P = P + rv[..., k]
        qcols = []
        for k in range(rep.dvmax):
            acc = mu_s
            for k2 in range(rep.dvmax):
                if k2 != k:
                    acc = acc + rv[..., k2]
            qcols.append(acc)
        qv = torch.stack(qcols, -1)[:, rep.vmask]
        q = torch.zeros((S, E), dtype=dt).index_copy(1, rep.vperm, qv)
    return P


def loss_fn(P: torch.Tensor, target: torch.Tensor, weight: torch.Tensor = None) -> torch.Tensor:
    """Binary cross-entropy between the error bits and sigma(-P), averaged (or
    weighted by `weight`, which then sums to one)."""
    x = torch.nn.functional.binary_cross_entropy_with_logits(-P, target.to(P.dtype), reduction="none")
    if weight is None:
        return x.mean()
    return (x * weight).sum()
