"""Helpers shared by the GPU tests: build a library discretisation and the
oracle's twin from the same seeded inputs, move arrays between them."""
import numpy as np

import workloads as wl


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


class Pair:
    """The same mesh and order on the GPU library and on the CPU oracle."""

    def __init__(self, ctx, dim, P, xy, e2v, precision=0):
        import oracle
        from paper_2301_11238_amd import bsw
        self.mesh = bsw.Mesh(ctx, dim, xy, e2v)
        self.disc = bsw.Disc(self.mesh, P, precision)
        self.orc = oracle.Oracle(dim, P, xy, e2v)
        self.ctx = ctx
        self.dim, self.P = dim, P
        self.shape = self.disc.shape

    def dev(self, a):
        import torch
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=self.ctx.torch_device, dtype=self.disc.dtype)

    @staticmethod
    def host(t):
        import torch
        torch.cuda.synchronize()
        return t.detach().to("cpu", torch.float64).numpy()


def mesh_for(dim, n):
    """1-D: n elements on [0, 10]; 2-D: n x n jittered squares on [0, 20]^2."""
    if dim == 1:
        return wl.mesh_1d(n, 0.0, 10.0)
    return wl.mesh_tri(n, 20.0, 20.0, 0.1, 7)


def relerr(a, b):
    """max |a - b| / max |b|, per field row block, worst over fields."""
    out = 0.0
    for f in range(b.shape[0]):
        scale = max(np.abs(b[f]).max(), 1e-300)
        out = max(out, np.abs(a[f] - b[f]).max() / scale)
    return out
