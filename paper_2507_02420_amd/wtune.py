"""Gradient-based tuning of the base matrix W (the function-encoding idea of
§4.2: choose W so that the transformed vector concentrates its energy in few
coefficients), driven by the GPU transform, top-k selection and backward.

Objective for a batch x and a number k of kept coefficients:
    E(W) = sum over instances of sum_{i in S(W)} |y_i|^2,  y = G_N(W) x,
with S(W) the indices of the k largest |y_i| (gtt_compress).  For a fixed S
the Euclidean gradient of E with respect to W is gtt_backward's gW for the
output gradient gy = 2 y on S and 0 elsewhere (gradients in the convention
dE/dRe + i dE/dIm).  W stays unitary (orthogonal for real dtypes): the ascent
direction is the skew-Hermitian A = gW W^H - W gW^H, and the step is the
Cayley retraction W <- (I - t/2 A)^{-1} (I + t/2 A) W.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import gtt as G


@dataclass
class TuneResult:
    W: torch.Tensor
    kept_fraction: list = field(default_factory=list)   # E(W) / ||x||^2 per step


def kept_energy(plan: G.Plan, W: torch.Tensor, x: torch.Tensor, k: int):
    """(E(W), indices, values) with E the energy of the k dominant coefficients."""
    idx, val, _ = plan.compress(W, x, k, reconstruct=False)
    e = torch.sum(torch.abs(val.to(torch.complex128 if val.is_complex() else torch.float64)) ** 2)
    return float(e.item()), idx, val


def riemannian_direction(W: torch.Tensor, gW: torch.Tensor) -> torch.Tensor:
    """Skew-Hermitian ascent direction A = gW W^H - W gW^H."""
    WH = W.conj().transpose(0, 1)
    gWH = gW.conj().transpose(0, 1)
    return gW @ WH - W @ gWH


def cayley_step(W: torch.Tensor, A: torch.Tensor, t: float) -> torch.Tensor:
    I = torch.eye(W.shape[0], dtype=W.dtype, device=W.device)
    # linalg.solve returns a column-major matrix; the transform reads W row-major
    return torch.linalg.solve(I - 0.5 * t * A, (I + 0.5 * t * A) @ W).contiguous()


def tune(x: torch.Tensor, W0: torch.Tensor, b: int, n: int, k: int, steps: int = 50, lr: float = 0.5,
         backtrack: bool = True) -> TuneResult:
    """Ascend E(W) from W0; x is (batch, b**n) on the GPU."""
    x = x.reshape(-1, b ** n).contiguous()
    batch = x.shape[0]
    plan = G.Plan(b, n, batch, x.dtype)
    W = W0.clone().contiguous()
    total = float(torch.sum(torch.abs(x.to(torch.complex128 if x.is_complex() else torch.float64)) ** 2).item())
    res = TuneResult(W=W)
    e, idx, val = kept_energy(plan, W, x, k)
    res.kept_fraction.append(e / total)
    t = lr
    for _ in range(steps):
        gy = torch.zeros_like(x)
        gy.scatter_(1, idx, 2 * val)
        _, gW = plan.backward(W, x, gy, want_gx=False)
        A = riemannian_direction(W, gW.to(W.dtype))
        nrm = float(torch.linalg.matrix_norm(A).item())
        if nrm == 0.0:
            break
        A = A / nrm
        while True:
            Wn = cayley_step(W, A, t)
            en, idxn, valn = kept_energy(plan, Wn, x, k)
            if en >= e or not backtrack or t < 1e-6:
                break
            t *= 0.5
        if en < e and backtrack:
            break
        W, e, idx, val = Wn.contiguous(), en, idxn, valn
        res.kept_fraction.append(e / total)
        t = min(lr, 2 * t)
    res.W = W
    return res
