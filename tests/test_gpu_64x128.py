"""The 64^3x128 configuration (33.5M sites, the whole field on one GPU).

No oracle run is affordable at this size, so the test uses a property that
holds at any size: a 16x16x16x128 field tiled 4x in x, y and z is a 64^3x128
field, and on it the operator applied to the tiled source is the tiling of the
operator on the base lattice (periodic space directions; the time extent is
kept, since an even number of copies in an antiperiodic direction would not
reproduce the boundary).  Every index, stride and 64-bit offset of the GPU
path is exercised at the full size; the values are the oracle's.
"""
import gc

import numpy as np
import pytest

from helpers import CSW, EPSBAR, KAPPA, MUBAR, rel_l2, to_dev, to_host
from oracle import Oracle
from paper_2212_06635_amd import synth

BASE = (16, 16, 16, 128)
REP = (4, 4, 4)  # copies in x, y, z
DIMS = (64, 64, 64, 128)
MU = 0.00072
TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3}


def tile_full(v, base=BASE):
    """Full-lattice field in lexicographic order (x fastest) -> tiled in x, y, z."""
    lx, ly, lz, lt = base
    a = v.reshape((lt, lz, ly, lx) + v.shape[1:])
    a = np.tile(a, (1, REP[2], REP[1], REP[0]) + (1,) * (v.ndim - 1))
    return a.reshape((-1,) + v.shape[1:])


def tile_cb(v_cb):
    """Odd-checkerboard field of the base lattice -> the same of the tiled lattice."""
    return synth.full_to_cb(tile_full(synth.cb_to_full(v_cb, BASE)), DIMS)


@pytest.fixture(scope="module")
def F():
    import torch

    import paper_2212_06635_amd.tmx as tmx

    print("\n[gpu 64^3x128] base 16^3x128 eps=0.25 seed=5, tiled 4x4x4", flush=True)
    U0 = synth.gauge_links(BASE, 0.25, 5)
    o = Oracle(BASE, U0, KAPPA, CSW, mu=MU, mubar=MUBAR, epsbar=EPSBAR)
    U = np.tile(U0, (1, REP[2], REP[1], REP[0], 1, 1, 1))
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


def test_tiling_map():
    """The tiling helper itself: a tiled field is periodic with the base extents."""
    v = np.arange(np.prod(BASE), dtype=np.float64)
    t = tile_full(v).reshape(DIMS[::-1])
    assert np.array_equal(t[:, :, :, :16], t[:, :, :, 16:32])
    assert np.array_equal(t[:, 16:32, :, :], t[:, :16, :, :])
    assert np.array_equal(t[:, :16, :16, :16].reshape(-1), v)


def mem(tag):
    import torch

    free, total = torch.cuda.mem_get_info()
    print(f"[gpu 64^3x128] {tag}: {free / 1e9:.0f} of {total / 1e9:.0f} GB free", flush=True)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("op,nf", [(1, 1), (2, 2)])
def test_64x128_mhat(F, op, nf, prec):
    tmx, o, ctx = F
    kind = tmx.TMX_FIELD_ODD if nf == 1 else tmx.TMX_FIELD_ODD_ND
    v0 = synth.gaussian_cb_spinor(BASE, 5, 0, nf)
    ref = tile_cb(o.mhat(v0, nf=nf, sgn=1))
    v = tile_cb(v0)
    out = ctx.empty(kind, prec)
    ctx.apply_mhat(out, ctx.pack(to_dev(v), kind, prec), op, prec)
    got = to_host(ctx.unpack(out, kind, prec), v.shape)
    assert rel_l2(got, ref) < TOL[prec]


@pytest.mark.gpu
def test_64x128_mpcg_f16(F):
    """MP-CG (FP16 inner) at 33.5M sites against the tiled oracle CG solution.
    Both solutions have relative residual <= 1e-10, so they differ by at most
    cond(N) * 2e-10 (cond(N) ~ 40 on these fields)."""
    tmx, o, ctx = F
    b0 = synth.gaussian_cb_spinor(BASE, 5, 1)
    x0, _, rel = o.cg(b0, tol=1e-11)
    assert rel <= 1e-11
    b = tile_cb(b0)
    x = to_dev(np.zeros_like(b))
    rc, info = ctx.solve(x, to_dev(b), 1, kind=tmx.TMX_SOLVER_MPCG_F16, op=1, tol=1e-10)
    assert rc == tmx.TMX_OK
    assert info[0]["true_residual"] <= 1e-10
    assert rel_l2(to_host(x, b.shape), tile_cb(x0)) < 5e-8


@pytest.mark.gpu
def test_64x128_pcg_learned_preconditioner(F):
    """CG on N preconditioned by K K^dagger (the learned network, FP16 inner
    iterations) at 33.5M sites: every network layer indexes activations of
    67M sites x 8 channels (offsets beyond 2^32 bytes).  The network is the
    seeded identity-plus-noise initialisation (K K^dagger is Hermitian
    positive definite whatever the weights); the solution is checked against
    the tiled oracle CG solution as for MP-CG."""
    from oracle import nn_oracle as nn

    tmx, o, ctx = F
    ctx.pc_set_weights(nn.identity_init(np.random.default_rng(3), 1e-2))
    b0 = synth.gaussian_cb_spinor(BASE, 5, 2)
    x0, _, rel = o.cg(b0, tol=1e-11)
    assert rel <= 1e-11
    b = tile_cb(b0)
    x = to_dev(np.zeros_like(b))
    mem("before the preconditioned solve")
    rc, info = ctx.solve(x, to_dev(b), 1, kind=tmx.TMX_SOLVER_PCG_NN, op=1, tol=1e-10, inner_prec=2)
    mem("after the preconditioned solve")
    print("[gpu 64^3x128] PCG-NN iterations", info[0]["iters"], "fallback", info[0]["fallback"], flush=True)
    assert rc == tmx.TMX_OK
    assert info[0]["fallback"] == 0  # converged on the preconditioned path itself
    assert info[0]["true_residual"] <= 1e-10
    assert rel_l2(to_host(x, b.shape), tile_cb(x0)) < 5e-8
