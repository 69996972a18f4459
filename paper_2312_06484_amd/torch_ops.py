"""torch.autograd.Function over the AIRPF C ABI.

``AirpfLogZ.apply(theta, problem)`` returns log Zhat(theta) as a 0-d float64
tensor; when theta requires grad the forward calls airpf_score and the
backward returns grad_out * (path-space score).  PyTorch supplies only the
tensor plumbing and the stream: every step of the filter runs in the HIP
kernels of libairpf.so (theta is a handful of numbers, read on the host).
"""
import numpy as np
import torch

from . import airpf


class Problem:
    """Fixed part of a filtering problem: model, data, sizes, seed, options."""

    def __init__(self, kind, y, m, N, seed, tau=0.3, fp64=False, dx=1, dy=1, consts=None, ckpt_every=0,
                 device=0):
        self.kind, self.y, self.m, self.N, self.seed = kind, np.asarray(y, dtype=np.float64), m, N, seed
        self.tau, self.fp64, self.dx, self.dy, self.consts, self.ckpt_every = tau, fp64, dx, dy, consts, ckpt_every
        stream = torch.cuda.current_stream(device).cuda_stream if torch.cuda.is_available() else None
        self.ctx = airpf.Context(device, stream=stream)

    def _kw(self):
        return dict(tau=self.tau, fp64=self.fp64, dx=self.dx, dy=self.dy, consts=self.consts)


class AirpfLogZ(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta, problem):
        th = theta.detach().to("cpu", torch.float64).numpy()
        if theta.requires_grad:
            _, lz, g = problem.ctx.score(problem.kind, th, problem.y, problem.m, problem.N, problem.seed,
                                         ckpt_every=problem.ckpt_every, **problem._kw())
            fctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
        else:
            _, lz = problem.ctx.run(problem.kind, th, problem.y, problem.m, problem.N, problem.seed, **problem._kw())
        return torch.tensor(lz, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(fctx, grad_out):
        (g,) = fctx.saved_tensors
        return grad_out.to(g.dtype) * g, None


def log_z(theta, problem):
    """log Zhat(theta) with the path-space score as its gradient."""
    return AirpfLogZ.apply(theta, problem)
