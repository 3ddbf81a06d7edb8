"""torch.autograd wrapper of the library's adjoint: the time-averaged
bottom-wall heat flux J = (1/N) sum_n q^n (Sec. 3.2 of arXiv:1501.03857) as a
differentiable function of the heater temperatures and the wall strength G_w.

The forward pass calls lbb_adjoint once, which returns J and its gradient
(a hand-written discrete adjoint with checkpointing); backward scales the
stored gradient by the incoming one.  PyTorch only carries the autograd
plumbing: every step runs in the HIP kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lbboil as L


class HeatFluxFn(torch.autograd.Function):
    """J = HeatFluxFn.apply(T_heater, Gw, domain, heater_idx, n_steps, K).

    T_heater: FP64 tensor [len(heater_idx)], the bottom-wall temperatures of
    the heater nodes (the other bottom nodes keep the domain's current T_b);
    Gw: FP64 scalar tensor, the bottom wall strength.  The domain's heater and
    G_w are set to these values; its state is left unchanged."""

    @staticmethod
    def forward(ctx, T_heater, Gw, domain: L.Domain, heater_idx, n_steps: int, K: int = 0):
        idx = np.asarray(heater_idx, dtype=np.int64)
        Tb = domain.bottom_temperature().copy()
        Tb[idx] = T_heater.detach().cpu().double().numpy()
        domain.set_heater(Tb)
        domain.set_wettability(float(Gw.detach().cpu()))
        J, gTb, gGw = domain.adjoint(n_steps, K, heater_idx=idx)
        ctx.save_for_backward(torch.as_tensor(gTb, dtype=torch.float64),
                              torch.tensor(gGw, dtype=torch.float64))
        ctx.dev = (T_heater.device, Gw.device)
        return torch.tensor(J, dtype=torch.float64, device=T_heater.device)

    @staticmethod
    def backward(ctx, gJ):
        gT, gG = ctx.saved_tensors
        gJ = gJ.detach().cpu().double()
        return (gJ * gT).to(ctx.dev[0]), (gJ * gG).to(ctx.dev[1]), None, None, None, None
