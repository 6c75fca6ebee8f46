"""-2 ln L as a torch.autograd.Function backed by libmipwa.

The library computes the value and the full gradient in one fused pass (forward and adjoint in the
same kernel), so backward only scales the stored gradient.  Two forms:

* ``MipwaNLL.apply(theta, ctx)``: theta is a float64 CPU tensor of P parameters; the evaluation is
  synchronous and the result is a 0-d float64 tensor on theta's device.
* ``nll_on_device(theta, ctx)``: enqueues the evaluation on torch's current HIP stream and returns a
  device tensor [nll, grad...] without a host synchronisation (torch owns the memory and the stream).
"""
from __future__ import annotations

import torch


class MipwaNLL(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta, mctx):
        th = theta.detach().to("cpu", torch.float64).contiguous().numpy()
        nll, grad = mctx.eval(th)
        fctx.save_for_backward(torch.from_numpy(grad).to(theta.device))
        return torch.tensor(nll, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(fctx, g):
        (grad,) = fctx.saved_tensors
        return g * grad.to(g.dtype), None


def nll_on_device(theta, mctx, device="cuda"):
    th = theta.detach().to("cpu", torch.float64).contiguous().numpy()
    mctx.set_params(th)
    out = torch.empty(1 + mctx.n_params, dtype=torch.float64, device=device)
    stream = torch.cuda.current_stream(out.device)
    mctx.eval_async(stream.cuda_stream, out.data_ptr())
    return out
