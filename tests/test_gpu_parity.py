"""GPU parity: every operator of the HIP library against the FP64 CPU oracle.

Bars: relative L2 <= 1e-13 (FP64), <= 1e-6 (FP32), <= 5e-3 (FP16 storage).
Lattices span a 2^4 lattice (x +- mu are the same site), a ragged volume
whose site count is not a multiple of the wavefront or block size, and
volumes covering many thread blocks.
"""
import sys

import numpy as np
import pytest

from helpers import CSW, EPSBAR, KAPPA, MU, MUBAR, oracle_T_to_blocks, rel_l2, to_dev, to_host
from oracle import Oracle
from paper_2212_06635_amd import synth

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3}

CASES = [
    ((2, 2, 2, 2), 0.4, 5),
    ((6, 4, 2, 10), 0.3, 3),
    ((8, 8, 8, 8), 0.3, 1),
    ((16, 8, 8, 16), 0.25, 2),
]


class Setup:
    def __init__(self, dims, eps, seed):
        import paper_2212_06635_amd.tmx as tmx

        self.tmx = tmx
        self.dims = dims
        self.U = synth.gauge_links(dims, eps, seed)
        self.o = Oracle(dims, self.U, KAPPA, CSW, mu=MU, mubar=MUBAR, epsbar=EPSBAR)
        self.ctx = tmx.Context(dims)
        self.ctx.set_params(tmx.Params(KAPPA, CSW, MU, MUBAR, EPSBAR, -1))
        self.ctx.load_gauge(self.U, gauge_id=float(seed))
        self.V, self.Vh = self.o.V, self.o.Vh


@pytest.fixture(scope="module", params=CASES, ids=lambda c: "x".join(map(str, c[0])))
def S(request):
    dims, eps, seed = request.param
    print(f"\n[gpu parity] lattice {dims} eps={eps} seed={seed}", flush=True)
    s = Setup(dims, eps, seed)
    yield s
    s.ctx.close()


def test_clover_built_on_device(S):
    T = S.ctx.get_clover()
    ref = oracle_T_to_blocks(S.o.T)
    assert np.abs(T - ref).max() < 1e-14


OPS = [(1, 1), (-1, 1), (2, 2)]  # (op, nflavours)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("op,nf", OPS)
def test_apply_D(S, op, nf, prec):
    tmx = S.tmx
    kind = tmx.TMX_FIELD_FULL if nf == 1 else tmx.TMX_FIELD_FULL_ND
    psi = synth.gaussian_spinor(S.V, 11, 0, nf)
    sgn = 1 if op == 2 else op
    ref = S.o.D(psi, nf=nf, sgn=sgn)
    inp = S.ctx.pack(to_dev(psi), kind, prec)
    out = S.ctx.empty(kind, prec)
    S.ctx.apply_D(out, inp, op, prec)
    got = to_host(S.ctx.unpack(out, kind, prec), psi.shape)
    assert rel_l2(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("dagger", [0, 1])
@pytest.mark.parametrize("op,nf", OPS)
def test_apply_mhat(S, op, nf, dagger, prec):
    tmx = S.tmx
    kind = tmx.TMX_FIELD_ODD if nf == 1 else tmx.TMX_FIELD_ODD_ND
    v = synth.gaussian_cb_spinor(S.dims, 12, 0, nf)
    sgn = 1 if op == 2 else op
    ref = S.o.mhat(v, nf=nf, sgn=sgn, dagger=bool(dagger))
    inp = S.ctx.pack(to_dev(v), kind, prec)
    out = S.ctx.empty(kind, prec)
    S.ctx.apply_mhat(out, inp, op, prec, dagger=dagger)
    got = to_host(S.ctx.unpack(out, kind, prec), v.shape)
    assert rel_l2(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("op,nf", OPS)
def test_apply_mdagm(S, op, nf, prec):
    tmx = S.tmx
    kind = tmx.TMX_FIELD_ODD if nf == 1 else tmx.TMX_FIELD_ODD_ND
    v = synth.gaussian_cb_spinor(S.dims, 13, 0, nf)
    sgn = 1 if op == 2 else op
    ref = S.o.mdagm(v, nf=nf, sgn=sgn)
    inp = S.ctx.pack(to_dev(v), kind, prec)
    out = S.ctx.empty(kind, prec)
    S.ctx.apply_mdagm(out, inp, op, prec)
    got = to_host(S.ctx.unpack(out, kind, prec), v.shape)
    assert rel_l2(got, ref) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("nrhs", [3, 12])
def test_multi_rhs_mhat(S, nrhs, prec):
    """n right-hand sides in one launch equal n single applies of the oracle."""
    tmx = S.tmx
    for op, nf in OPS:
        kind = tmx.TMX_FIELD_ODD if nf == 1 else tmx.TMX_FIELD_ODD_ND
        vs = np.stack([synth.gaussian_cb_spinor(S.dims, 14, k, nf) for k in range(nrhs)])
        sgn = 1 if op == 2 else op
        inp = S.ctx.pack(to_dev(vs), kind, prec, nvec=nrhs)
        out = S.ctx.empty(kind, prec, nvec=nrhs)
        S.ctx.apply_mhat(out, inp, op, prec, dagger=0, nrhs=nrhs)
        got = to_host(S.ctx.unpack(out, kind, prec, nvec=nrhs), vs.shape)
        for k in range(nrhs):
            assert rel_l2(got[k], S.o.mhat(vs[k], nf=nf, sgn=sgn)) < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_pack_roundtrip(S, prec):
    tmx = S.tmx
    v = synth.gaussian_cb_spinor(S.dims, 15, 0, 2)
    got = to_host(S.ctx.unpack(S.ctx.pack(to_dev(v), tmx.TMX_FIELD_ODD_ND, prec), tmx.TMX_FIELD_ODD_ND, prec), v.shape)
    if prec == 0:
        assert np.array_equal(got, v)
    else:
        assert rel_l2(got, v) < {1: 1e-7, 2: 1e-3}[prec]


def test_host_clover_load(S):
    """A clover term uploaded from the host gives the same operator."""
    tmx = S.tmx
    ctx = tmx.Context(S.dims)
    ctx.set_params(tmx.Params(KAPPA, CSW, MU, MUBAR, EPSBAR, -1))
    ctx.load_gauge(S.U, 1.0)
    ctx.load_clover(oracle_T_to_blocks(S.o.T))
    v = synth.gaussian_cb_spinor(S.dims, 16, 0, 1)
    out = ctx.empty(tmx.TMX_FIELD_ODD, 0)
    ctx.apply_mhat(out, ctx.pack(to_dev(v), tmx.TMX_FIELD_ODD, 0), 1, 0)
    got = to_host(ctx.unpack(out, tmx.TMX_FIELD_ODD, 0), v.shape)
    assert rel_l2(got, S.o.mhat(v)) < 1e-13
    bad = oracle_T_to_blocks(S.o.T)
    bad[0, 0, 0, 1] += 1e-3
    with pytest.raises(tmx.TmxError) as e:
        ctx.load_clover(bad)
    assert e.value.code == tmx.TMX_EINVAL
    ctx.close()
