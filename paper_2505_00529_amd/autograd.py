"""torch.autograd bindings of the cost, gradient and Hessian-vector product.

PyTorch provides device memory and the current HIP stream only; every number is computed by
the library's kernels through the C ABI (``*_dev`` entry points, enqueued on torch's current
stream).

* ``QocCost.apply(theta, problem)`` -> scalar cost C(theta).  Its backward returns
  ``grad_output * QocGrad.apply(theta, problem)``, so a second differentiation is available.
* ``QocGrad.apply(theta, problem)`` -> gradient g(theta) (first-order adjoint, Alg. 1 of the
  paper).  Its backward is the Hessian-vector product H(theta) v (the tangent and
  second-adjoint sweeps of Alg. 2 for one direction).

With ``problem.set_checkpoint_interval(k)`` both the gradient and the HVP keep eigen-data for
k steps at a time and recompute it segment by segment in their backward sweeps.

Every forward and backward waits for its evaluation and checks the handle's device status
(``problem.sync()``), so that a device-side failure (a Jacobi step that reached the sweep cap,
``QOC_ERR_NOCONV``) raises ``qoc.QocError`` in the call that produced it instead of returning a
tensor.
"""
from __future__ import annotations

import torch

from . import qoc

__all__ = ["QocCost", "QocGrad", "cost", "grad"]


def _prepare(theta: torch.Tensor, problem: "qoc.Problem") -> torch.Tensor:
    if theta.device.type != "cuda" or theta.dtype != torch.float64:
        raise TypeError("theta must be a float64 tensor on a HIP device")
    if theta.numel() != problem.P:
        raise ValueError(f"theta has {theta.numel()} entries, the control model has {problem.P}")
    stream = torch.cuda.current_stream(theta.device).cuda_stream   # 0 for torch's default stream
    if getattr(problem, "_torch_stream", None) != stream:
        problem.set_stream(stream)
        problem._torch_stream = stream
    return theta.detach().contiguous()


class QocGrad(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, problem):
        th = _prepare(theta, problem)
        g = torch.empty_like(th)
        problem.grad_dev(th.data_ptr(), None, g.data_ptr())
        problem.sync()
        ctx.problem = problem
        ctx.save_for_backward(th)
        return g

    @staticmethod
    def backward(ctx, v):
        (th,) = ctx.saved_tensors
        problem = ctx.problem
        vv = _prepare(v.to(torch.float64), problem)
        hv = torch.empty_like(th)
        problem.hvp_dev(th.data_ptr(), vv.data_ptr(), hv.data_ptr())
        problem.sync()
        return hv, None


class QocCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, problem):
        th = _prepare(theta, problem)
        c = torch.empty((), dtype=torch.float64, device=th.device)
        problem.cost_dev(th.data_ptr(), c.data_ptr())
        problem.sync()
        ctx.problem = problem
        ctx.save_for_backward(theta)
        return c

    @staticmethod
    def backward(ctx, gout):
        (theta,) = ctx.saved_tensors
        return gout * QocGrad.apply(theta, ctx.problem), None


def cost(theta: torch.Tensor, problem: "qoc.Problem") -> torch.Tensor:
    return QocCost.apply(theta, problem)


def grad(theta: torch.Tensor, problem: "qoc.Problem") -> torch.Tensor:
    return QocGrad.apply(theta, problem)
