"""torch.autograd bindings of the NLL kernels.

``nll(theta, model, data)`` returns the NLL of Eq. 1 as a 0-d CUDA tensor
whose first derivative comes from the fused gradient kernel and whose second
derivative (Hessian-vector products, for double backward) comes from the
Hessian pass.  theta is a float64 CUDA tensor holding every parameter; the
derivative with respect to a fixed parameter is zero (fixed parameters are
constants of the model).
"""
import numpy as np
import torch

from . import uml


def _free_index(model, device):
    return torch.as_tensor(np.flatnonzero(model.free), dtype=torch.long, device=device)


class _Grad(torch.autograd.Function):
    """theta -> dNLL/dtheta (forward: the already computed gradient;
    backward: H @ v from the Hessian kernel)."""

    @staticmethod
    def forward(ctx, theta, g_full, model, data):
        ctx.save_for_backward(theta)
        ctx.model, ctx.data = model, data
        return g_full.clone()

    @staticmethod
    def backward(ctx, v):
        (theta,) = ctx.saved_tensors
        model = ctx.model
        th = theta.detach().double().cpu().numpy()
        _, _, h = uml.uml_eval_hessian(model, ctx.data, th)
        idx = np.flatnonzero(model.free)
        H = np.zeros((model.n_params, model.n_params))
        H[np.ix_(idx, idx)] = h
        Ht = torch.as_tensor(H, dtype=v.dtype, device=v.device)
        return Ht @ v, None, None, None


class _NLL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, model, data):
        th = theta.detach().to(torch.float64).contiguous()
        out = torch.empty(1 + model.n_free, dtype=torch.float64, device=theta.device)
        uml.uml_eval_nll_grad_dev(model, data, th, out)
        g_full = torch.zeros_like(th)
        g_full[_free_index(model, th.device)] = out[1:]
        ctx.save_for_backward(theta, g_full)
        ctx.model, ctx.data = model, data
        return out[0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        theta, g_full = ctx.saved_tensors
        g = _Grad.apply(theta, g_full, ctx.model, ctx.data)
        return grad_out * g, None, None


def nll(theta, model, data):
    """Differentiable NLL (twice) of `data` under `model` at `theta`."""
    return _NLL.apply(theta, model, data)
