"""torch.autograd.Function over the pathwise adjoint, resident on the device.

``CapletPricer(ts, n_paths, seed, base_levels)`` owns one plan of the term
structure ``ts`` (FP32, up to ``n_paths`` paths) for its whole life; calling
it with CUDA tensors ``L0`` [N] and ``levels`` [N] returns the product prices
(strike 0 of each caplet, or of each co-terminal swaption when
``ts.product`` is 1) with the initial forwards replaced by ``L0`` and each
rate's vol curve shifted in parallel by ``levels - base_levels``:
lambda(t, T_i) = ts.vol[k, i] + levels[i] - base_levels[i].

Everything stays on the device and on torch's current stream: the forward
pass writes the inputs into the plan (``lll_plan_set_inputs_dev``), runs a
FULL pricing pass and copies the prices into a new tensor
(``lll_plan_results_dev``), with no host synchronisation; the backward pass
is the vector-Jacobian product ``lll_plan_greeks_vjp_dev`` with the incoming
gradient as the weights (one reverse sweep on the forward pass's random
streams), written into the gradient tensors on the device.  The plan is
released by ``close()`` (or the ``with`` block), not by garbage collection.
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


class CapletPricer:
    """Differentiable prices of one term structure's products on one GPU."""

    def __init__(self, ts, n_paths: int, seed: int = 1, base_levels=None, device="cuda"):
        self.device = torch.device(device)
        self.N, self.S = ts.n_rates, ts.n_strikes
        self.n_paths, self.seed = int(n_paths), int(seed)
        base = np.zeros(self.N) if base_levels is None else np.asarray(base_levels, np.float64)
        self.base = torch.tensor(base, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self.plan = _lib.Plan(ts, precision=_lib.FP32, max_paths=self.n_paths)

    def __call__(self, L0: torch.Tensor, levels: torch.Tensor) -> torch.Tensor:
        return CapletPrice.apply(L0, levels, self)

    def close(self):
        plan = getattr(self, "plan", None)
        if plan is not None:
            torch.cuda.current_stream(self.device).synchronize()
            plan.close()
            self.plan = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class CapletPrice(torch.autograd.Function):
    @staticmethod
    def forward(ctx, L0: torch.Tensor, levels: torch.Tensor, pricer: CapletPricer):
        if pricer.plan is None:
            raise RuntimeError("CapletPricer is closed")
        if not (L0.is_cuda and levels.is_cuda):
            raise ValueError("CapletPrice takes CUDA tensors (the plan lives on the device)")
        stream = torch.cuda.current_stream(L0.device)
        L0d = L0.detach().to(torch.float64).contiguous()
        shift = (levels.detach().to(torch.float64) - pricer.base).contiguous()
        plan = pricer.plan
        plan.set_inputs_dev(L0=L0d, vol_shift=shift, stream=stream)
        plan.execute(_lib.FULL, pricer.n_paths, seed=pricer.seed, stream=stream)
        price = torch.empty((pricer.N, pricer.S), dtype=torch.float64, device=L0.device)
        plan.results_dev(price=price, stream=stream)
        ctx.save_for_backward(L0d, shift)
        ctx.pricer = pricer
        return price[:, 0].to(L0.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        L0d, shift = ctx.saved_tensors
        pricer = ctx.pricer
        if pricer.plan is None:
            raise RuntimeError("CapletPricer is closed")
        stream = torch.cuda.current_stream(grad_out.device)
        plan = pricer.plan
        # the inputs of this forward pass (the plan may have priced others since)
        plan.set_inputs_dev(L0=L0d, vol_shift=shift, stream=stream)
        g = grad_out.detach().to(torch.float64).contiguous()
        plan.greeks_vjp_dev(pricer.n_paths, g, seed=pricer.seed, stream=stream)
        gL = torch.empty(pricer.N, dtype=torch.float64, device=grad_out.device)
        gV = torch.empty(pricer.N, dtype=torch.float64, device=grad_out.device)
        plan.greeks_vjp_results_dev(vjp_L0=gL, vjp_vol=gV, stream=stream)
        return gL.to(grad_out.dtype), gV.to(grad_out.dtype), None
