"""The 64^3x128 configuration, two-flavour sector: a 12-shift multishift
solve at 33.5M sites through the tiled field of test_gpu_64x128 (the operator
there is checked against the oracle).  A context of its own holds only the
fields this solve needs: twelve FP64 two-flavour solutions are 77 GB.
"""
import gc

import numpy as np
import pytest

from helpers import CSW, EPSBAR, KAPPA, MUBAR, rel_l2, to_dev
from oracle import Oracle
from paper_2212_06635_amd import synth
from test_gpu_64x128 import BASE, DIMS, MU, REP, mem, tile_cb


@pytest.fixture(scope="module")
def F():
    import torch

    import paper_2212_06635_amd.tmx as tmx

    print("\n[gpu 64^3x128 nd] base 16^3x128 eps=0.25 seed=5, tiled 4x4x4", flush=True)
    U0 = synth.gauge_links(BASE, 0.25, 5)
    o = Oracle(BASE, U0, KAPPA, CSW, mu=MU, mubar=MUBAR, epsbar=EPSBAR)
    U = np.tile(U0, (1, REP[2], REP[1], REP[0], 1, 1, 1))
    gc.collect()
    torch.cuda.empty_cache()
    ctx = tmx.Context(DIMS)
    ctx.set_params(tmx.Params(KAPPA, CSW, MU, MUBAR, EPSBAR, -1))
    ctx.load_gauge(U, 5.0)
    del U
    gc.collect()
    mem("gauge loaded")
    yield tmx, o, ctx
    ctx.close()
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.gpu
def test_64x128_multishift_nd(F):
    """Twelve shifts of the two-flavour operator at 33.5M sites (FP16-storage
    multishift, FP64-reliable refinement; FP16 keeps the twelve shift vectors
    and directions within HBM next to the twelve FP64 solutions): every
    shift's FP64 true residual (its FP64 operator is checked in test_gpu_64x128)
    <= 1e-10, and the largest shift against the tiled oracle solution."""
    import torch

    tmx, o, ctx = F
    torch.cuda.empty_cache()
    mem("before multishift")
    shifts = 2.08 * 10.0 ** (-5.0 + 5.0 * np.arange(12) / 11.0)
    b0 = synth.gaussian_cb_spinor(BASE, 5, 2, 2)
    b = to_dev(tile_cb(b0))
    n = b.numel()
    x = torch.zeros(12 * n, dtype=torch.complex128, device="cuda")
    rc, info = ctx.multishift_solve(x, b, shifts, op=2, tol=1e-10, inner_prec=2)
    mem("after multishift")
    assert rc == tmx.TMX_OK
    assert max(i["true_residual"] for i in info) <= 1e-10
    x11 = x[11 * n:].cpu().numpy().reshape((-1,) + b0.shape[1:])
    ref, _, rel = o.cg(b0, nf=2, shift=shifts[11], tol=1e-11)
    assert rel <= 1e-11
    assert rel_l2(x11, tile_cb(ref)) < 5e-8
    del x, b
    torch.cuda.empty_cache()
