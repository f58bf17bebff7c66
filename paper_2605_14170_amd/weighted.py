"""Weighted (differentiable) form of the decoder: a torch.autograd.Function over the
library's training forward (mbbp_wbp_forward) and adjoint (mbbp_wbp_backward)
kernels, the training loss and an Adam training loop.

The weighted rule scales each iteration's min-sum check message by alpha_{t,l} and
damps it with beta_{t,l} (r^(t) = clamp((1 - beta) S alpha M + beta r^(t-1)));
one [T, L] pair of weight tables is shared by the X and Z parts.  The loss is
the binary cross-entropy between each qubit's true error bit and sigma(-P^(T)),
averaged over shots, representations, qubits and both parts.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, Optional

from . import Decoder, prior_llr


def _torch():
    import torch
    return torch


def unpack_bits(words, n: int):
    """int64 [shots, W] words (bit i at bit i % 64 of word i // 64) -> float32 [shots, n]."""
    torch = _torch()
    idx = torch.arange(n, device=words.device)
    w = words[:, idx // 64]
    return ((w >> (idx % 64)) & 1).to(torch.float32)


class WeightedBP:
    """autograd Function: (alpha, beta) -> P^(T) [2, shots, L, n] of both parts."""

    _fn = None

    @classmethod
    def fn(cls):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, alpha, beta, dec, syn_x, syn_z, prior_x, prior_z, ckpt_every):
                    a = alpha.detach().contiguous()
                    b = beta.detach().contiguous()
                    px, ckx = dec.wbp_forward(0, syn_x, prior_x, a, b, ckpt_every)
                    pz, ckz = dec.wbp_forward(1, syn_z, prior_z, a, b, ckpt_every)
                    ctx.dec, ctx.every = dec, int(ckpt_every)
                    ctx.save_for_backward(a, b, syn_x, syn_z, prior_x, prior_z, ckx, ckz)
                    return torch.stack([px, pz])

                @staticmethod
                def backward(ctx, grad_p):
                    a, b, sx, sz, px, pz, ckx, ckz = ctx.saved_tensors
                    g = grad_p.contiguous()
                    ga = torch.zeros_like(a)
                    gb = torch.zeros_like(b)
                    ctx.dec.wbp_backward(0, sx, px, a, b, ctx.every, ckx, g[0].contiguous(), ga, gb)
                    ctx.dec.wbp_backward(1, sz, pz, a, b, ctx.every, ckz, g[1].contiguous(), ga, gb)
                    return ga, gb, None, None, None, None, None, None

            cls._fn = _F
        return cls._fn

    @classmethod
    def apply(cls, alpha, beta, dec: Decoder, syn_x, syn_z, prior_x, prior_z, ckpt_every: int = 5):
        return cls.fn().apply(alpha, beta, dec, syn_x, syn_z, prior_x, prior_z, ckpt_every)


def loss_fn(P, err_x, err_z, n: int):
    """Mean binary cross-entropy between the error bits and sigma(-P^(T))."""
    torch = _torch()
    y = torch.stack([unpack_bits(err_x, n), unpack_bits(err_z, n)])[:, :, None, :]
    return torch.nn.functional.binary_cross_entropy_with_logits(-P, y.expand_as(P))


@dataclasses.dataclass
class TrainResult:
    alpha: object            # [T, L] after the last step
    beta: object
    losses: list             # training loss of every step
    best_alpha: object       # weights of the best validation score (the last ones without validation)
    best_beta: object
    best_step: int           # step after which they were taken (-1: initial weights)
    validation: list         # (step, score) of every validation


def train(dec: Decoder, seed: int, p: float, batch: int, steps: int, lr: float = 1e-3,
          alpha0: float = 0.875, ckpt_every: int = 5, shot0: int = 0,
          callback: Optional[Callable[[int, float], None]] = None,
          validate: Optional[Callable[[object, object], float]] = None, val_every: int = 0) -> TrainResult:
    """Adam on (alpha, beta) from alpha = alpha0, beta = 0.  Step k trains on the fresh
    shots [shot0 + k * batch, shot0 + (k + 1) * batch) of the counter-based sampler
    at error rate p.  With `validate` (weights -> score, lower is better) the
    initial weights and those after every val_every steps are scored and the best
    are kept as well."""
    torch = _torch()
    alpha = torch.full((dec.T, dec.L), float(alpha0), dtype=torch.float32, device="cuda", requires_grad=True)
    beta = torch.zeros((dec.T, dec.L), dtype=torch.float32, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([alpha, beta], lr=lr)
    prior = torch.full((dec.n,), prior_llr(p), dtype=torch.float32, device="cuda")
    losses, vals = [], []
    best = (float("inf"), -1, alpha.detach().clone(), beta.detach().clone())

    def check(k):
        nonlocal best
        v = float(validate(alpha.detach().clone(), beta.detach().clone()))
        vals.append((k, v))
        if v < best[0]:
            best = (v, k, alpha.detach().clone(), beta.detach().clone())

    if validate is not None and val_every > 0:
        check(-1)
    for k in range(steps):
        ex, ez, sx, sz = dec.sample(seed, p, shot0 + k * batch, batch)
        P = WeightedBP.apply(alpha, beta, dec, sx, sz, prior, prior, ckpt_every)
        loss = loss_fn(P, ex, ez, dec.n)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        v = float(loss.detach())
        losses.append(v)
        if callback is not None:
            callback(k, v)
        if validate is not None and val_every > 0 and (k + 1) % val_every == 0:
            check(k)
    a, b = alpha.detach().clone(), beta.detach().clone()
    if validate is None or val_every <= 0:
        return TrainResult(a, b, losses, a, b, steps - 1, vals)
    return TrainResult(a, b, losses, best[2], best[3], best[1], vals)
