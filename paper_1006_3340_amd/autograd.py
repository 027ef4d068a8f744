"""torch.autograd.Function over the pathwise adjoint.

``CapletPrice.apply(L0, vol_levels, ts, n_paths, seed)`` returns the product
prices (strike 0 of each caplet, or of each co-terminal swaption when
``ts.product`` is 1) of the term structure ``ts`` with its initial
forwards replaced by ``L0`` and its vol curves shifted so that
lambda(t, T_i) = vol_levels[i] + (ts.vol[k, i] - base_levels[i]) (a parallel
shift of each rate's curve).  The forward pass is a FULL pricing pass; the
backward pass is the GPU's vector-Jacobian product ``lll_plan_greeks_vjp``
with the incoming gradient as the weights (one reverse sweep, on the forward
pass's random streams), not the full Jacobian.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib


def shifted(ts, L0: np.ndarray, levels: np.ndarray, base_levels: np.ndarray):
    """Copy of ts with forwards L0 and each rate's vol curve shifted by levels - base."""
    vol = ts.vol.copy()
    s = ts.steps_per_period
    for k in range(vol.shape[0]):
        m = k // s
        vol[k, m:] += (levels - base_levels)[m:]
    return ts.copy(L0=np.asarray(L0, dtype=np.float64).copy(), vol=vol)


class CapletPrice(torch.autograd.Function):
    @staticmethod
    def forward(ctx, L0: torch.Tensor, levels: torch.Tensor, ts, n_paths: int, seed: int = 1,
                base_levels=None):
        base = np.zeros(ts.n_rates) if base_levels is None else np.asarray(base_levels, float)
        ts2 = shifted(ts, L0.detach().cpu().double().numpy(), levels.detach().cpu().double().numpy(),
                      base)
        plan = _lib.Plan(ts2, precision=_lib.FP32, max_paths=n_paths)
        plan.execute(_lib.FULL, n_paths, seed=seed)
        price = plan.results()["price"][:, 0].copy()
        ctx.plan, ctx.n_paths, ctx.seed, ctx.dev = plan, n_paths, seed, L0.device
        return torch.from_numpy(price).to(L0.device, L0.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        plan = ctx.plan
        plan.greeks_vjp(ctx.n_paths, grad_out.detach().cpu().double().numpy(), seed=ctx.seed)
        r = plan.greeks_vjp_results()
        plan.close()
        gL = torch.from_numpy(r["vjp_L0"]).to(ctx.dev, grad_out.dtype)
        gV = torch.from_numpy(r["vjp_vol"]).to(ctx.dev, grad_out.dtype)
        return gL, gV, None, None, None, None
