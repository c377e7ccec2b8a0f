"""The allocation-free Schur operator (tmx_apply_mhat_noalloc) against
tmx_apply_mhat: the same kernels on the same inputs, so the outputs agree bit
for bit; two calls in a row, the second on a smaller input, share the static
scratch; oversized requests and missing fields are refused before anything
runs."""
import numpy as np
import pytest

from helpers import CSW, EPSBAR, KAPPA, MUBAR, to_dev
from paper_2212_06635_amd import synth

pytestmark = pytest.mark.gpu

MU0 = 0.01


def _ctx(tmx, dims, seed):
    U = synth.gauge_links(dims, 0.3, seed)
    ctx = tmx.Context(dims)
    ctx.set_params(tmx.Params(KAPPA, CSW, MU0, MUBAR, EPSBAR, -1))
    ctx.load_gauge(U, float(seed))
    return ctx


def _both(tmx, ctx, dims, op, prec, dagger, nrhs, seed):
    nf = 2 if op == tmx.TMX_OP_ND else 1
    kind = tmx.TMX_FIELD_ODD_ND if nf == 2 else tmx.TMX_FIELD_ODD
    v = np.stack([synth.gaussian_cb_spinor(dims, seed, k, nf) for k in range(nrhs)])
    src = ctx.pack(to_dev(v), kind, prec, nrhs)
    ref = ctx.empty(kind, prec, nrhs)
    ctx.apply_mhat(ref, src, op, prec, dagger, nrhs)
    got = ctx.empty(kind, prec, nrhs)
    got.fill_(0xAB)
    ctx.apply_mhat_noalloc(got, src, op, prec, dagger, nrhs)
    return ref, got


def test_noalloc_matches_apply_mhat_on_two_calls():
    import torch

    import paper_2212_06635_amd.tmx as tmx

    big, small = (16, 16, 16, 32), (8, 8, 8, 8)
    print(f"\n[gpu no-alloc] {big} then {small}", flush=True)
    ca = _ctx(tmx, big, 21)
    cb = _ctx(tmx, small, 22)
    cases = [(1, 0, 0, 3), (-1, 1, 1, 1), (2, 1, 0, 2), (2, 2, 1, 1), (3, 0, 0, 1)]
    for op, prec, dagger, nrhs in cases:
        # first call: the larger input; second call: a smaller one on the same scratch
        ra, ga = _both(tmx, ca, big, op, prec, dagger, nrhs, 30 + nrhs)
        rb, gb = _both(tmx, cb, small, op, prec, dagger, 1, 40)
        torch.cuda.synchronize()
        assert torch.equal(ra, ga), (op, prec, dagger, nrhs)
        assert torch.equal(rb, gb), (op, prec, dagger)
    ca.close()
    cb.close()


def test_noalloc_refusals():
    import paper_2212_06635_amd.tmx as tmx

    dims = (16, 16, 16, 32)
    ctx = _ctx(tmx, dims, 23)
    kind = tmx.TMX_FIELD_ODD_ND
    # 32 two-flavour FP64 right-hand sides need 805 MB of intermediate: refused
    # (the fields themselves are real, so nothing could go astray either way)
    a, b = ctx.empty(kind, 0, 32), ctx.empty(kind, 0, 32)
    a.zero_()
    with pytest.raises(tmx.TmxError) as e:
        ctx.apply_mhat_noalloc(b, a, 2, 0, 0, 32)
    assert e.value.code == tmx.TMX_EINVAL and "scratch" in str(e.value)
    del a, b
    out = ctx.empty(tmx.TMX_FIELD_ODD, 2)
    inp = ctx.empty(tmx.TMX_FIELD_ODD, 2)
    # nothing of FP16 has been built yet in this context
    with pytest.raises(tmx.TmxError) as e:
        ctx.apply_mhat_noalloc(out, inp, 1, 2, 0, 1)
    assert e.value.code == tmx.TMX_ENOTLOADED
    ctx.close()
