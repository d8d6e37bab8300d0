"""bsw_stage_update_noalloc (no device allocation; reduction scratch in the
library's fixed per-device array) against bsw_stage_update through the C ABI:
two calls in a row, the second on a smaller discretisation, each against a
fresh bsw_stage_update of the same inputs.  The update is the same kernel
(bitwise equal states); the norms go through the same reductions of the same
partials, so they are equal too (FP64: max |alpha dW|, max |W|, mass,
active%)."""
import numpy as np
import pytest

import workloads as wl
from _gpu_util import have_gpu, mesh_for

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


def _case(ctx, dim, P, n, precision, seed):
    import torch
    from paper_2301_11238_amd import bsw
    xy, e2v = mesh_for(dim, n)
    mesh = bsw.Mesh(ctx, dim, xy, e2v)
    disc = bsw.Disc(mesh, P, precision)
    W = torch.from_numpy(wl.random_state(dim, P, disc.n_el, seed)).to(ctx.torch_device, disc.dtype)
    dW = torch.from_numpy(wl.random_vector(dim, P, disc.n_el, seed + 1)).to(ctx.torch_device, disc.dtype)
    return mesh, disc, W, dW


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_stage_update(precision):
    import torch
    from paper_2301_11238_amd import bsw
    print(f"noalloc stage update, precision {precision}", flush=True)
    ctx = bsw.Context(0)
    prm = bsw.make_params(wl.Params(sigma0=40.0, gamma=1e3, beta=1e3, reg=2))
    # first a large discretisation (several reduction workgroups, ragged tail),
    # then a smaller one: the scratch keeps the first call's partials, which
    # the second must not pick up
    for (dim, P, n, seed) in [(2, 3, 37, 11), (2, 1, 5, 12), (1, 2, 333, 13)]:
        mesh, disc, W, dW = _case(ctx, dim, P, n, precision, seed)
        for params in (prm, None):
            Wa, Wb = W.clone(), W.clone()
            ref = disc.stage_update(params, Wa, dW, 0.37)
            got = disc.stage_update_noalloc(params, Wb, dW, 0.37)
            torch.cuda.synchronize()
            assert torch.equal(Wa, Wb), (dim, P, n)
            assert got == ref, (dim, P, n, got, ref)
            assert ref[0] > 0 and ref[1] > 0
            if params is not None:
                assert ref[2] > 0 and 0.0 <= ref[3] <= 100.0 * (1.0 + 1e-5)  # FP32 metrics round the area
        del disc, mesh, W, dW
    ctx.close()


def test_noalloc_rejects_null_arguments():
    import ctypes as C
    from paper_2301_11238_amd import bsw
    ctx = bsw.Context(0)
    mesh, disc, W, dW = _case(ctx, 2, 2, 4, 0, 3)
    out = (C.c_double * 4)()
    rc = bsw.lib().bsw_stage_update_noalloc(disc.h, None, None, C.c_void_p(dW.data_ptr()), 1.0, out)
    assert rc == -1
    del disc, mesh
    ctx.close()
