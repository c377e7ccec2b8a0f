"""The autotuner: it picks a launch shape per kernel key, the tuned operator
matches the FP64 oracle to the precision's bound (and is bit-identical to the
untuned one: each site is computed by one thread whatever the launch shape),
and the choice is cached in the file named by TMX_TUNE_CACHE, which a new
context of the same volume reads back."""
import numpy as np
import pytest

from helpers import CSW, EPSBAR, KAPPA, MUBAR, rel_l2, to_dev, to_host
from oracle import Oracle
from paper_2212_06635_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (16, 8, 8, 16)
TOL = {0: 1e-13, 1: 1e-6, 2: 5e-3}


@pytest.mark.parametrize("prec,op,nrhs", [(0, 1, 1), (1, 2, 1), (2, 1, 3)])
def test_tuned_launch_changes_nothing_and_is_cached(tmp_path, monkeypatch, prec, op, nrhs):
    import paper_2212_06635_amd.tmx as tmx

    print(f"\n[gpu tuner] {DIMS} prec={prec} op={op} nrhs={nrhs}", flush=True)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TMX_TUNE_CACHE", str(cache))
    U = synth.gauge_links(DIMS, 0.3, 7)
    nf = 2 if op == 2 else 1
    kind = tmx.TMX_FIELD_ODD_ND if nf == 2 else tmx.TMX_FIELD_ODD
    v = np.stack([synth.gaussian_cb_spinor(DIMS, 7, k, nf) for k in range(nrhs)])

    def make():
        ctx = tmx.Context(DIMS)
        ctx.set_params(tmx.Params(KAPPA, CSW, 0.01, MUBAR, EPSBAR, -1))
        ctx.load_gauge(U, 7.0)
        return ctx

    def apply(ctx):
        out = ctx.empty(kind, prec, nrhs)
        ctx.apply_mhat(out, ctx.pack(to_dev(v), kind, prec, nrhs), op, prec, 0, nrhs)
        return to_host(ctx.unpack(out, kind, prec, nrhs), v.shape)

    suffix = {0: "f64", 1: "f32", 2: "f16"}[prec] + ("_nd" if nf == 2 else "") + (f"_r{nrhs}" if nrhs > 1 else "")
    ctx = make()
    before = apply(ctx)
    assert not ctx.tuned_config("K1_" + suffix)["tuned"]
    ctx.tune(prec, op, nrhs)
    cfgs = {k: ctx.tuned_config(k + "_" + suffix) for k in ("K1", "K2")}
    for c in cfgs.values():
        assert c["tuned"] and c["block"] in (64, 128, 256) and c["xcd"] in (0, 1)
    after = apply(ctx)
    ctx.close()
    assert np.array_equal(before, after)
    o = Oracle(DIMS, U, KAPPA, CSW, mu=0.01, mubar=MUBAR, epsbar=EPSBAR)
    for k in range(nrhs):
        assert rel_l2(after[k], o.mhat(v[k], nf=nf)) < TOL[prec], k
    # a new context of the same volume starts from the cached choice
    ctx = make()
    for k, c in cfgs.items():
        assert ctx.tuned_config(k + "_" + suffix) == c
    again = apply(ctx)
    ctx.close()
    assert np.array_equal(before, again)
    lines = cache.read_text().split("\n")
    assert sum(("K1_" + suffix) in ln for ln in lines) >= 1 and sum(("K2_" + suffix) in ln for ln in lines) >= 1
