"""The autotuner: it picks a launch shape per kernel key (workgroup size, block
order, sites per thread, right-hand-side group size), the tuned operator
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


@pytest.mark.parametrize("prec,op,nrhs", [(0, 1, 1), (1, 2, 1), (2, 1, 3), (1, 2, 12)])
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
        assert c["spt"] in (1, 2) and nrhs % max(c["rg"], 1) == 0
    assert cfgs["K1"]["rg"] == cfgs["K2"]["rg"]  # the two halves share the group size
    print(f"[gpu tuner] chosen: {cfgs}", flush=True)
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


def test_every_group_size_gives_the_same_operator(monkeypatch, tmp_path):
    """Each right-hand-side group size the tuner can pick (K1 and K2 run per
    group), written into the tuning cache by hand, yields the oracle's
    operator on all 12 right-hand sides (two flavours, FP32)."""
    import paper_2212_06635_amd.tmx as tmx

    U = synth.gauge_links(DIMS, 0.3, 8)
    o = Oracle(DIMS, U, KAPPA, CSW, mu=0.01, mubar=MUBAR, epsbar=EPSBAR)
    v = np.stack([synth.gaussian_cb_spinor(DIMS, 8, k, 2) for k in range(12)])
    ref = np.stack([o.mhat(v[k], nf=2) for k in range(12)])
    kind = tmx.TMX_FIELD_ODD_ND
    dk = "x".join(map(str, DIMS))
    for rg in (1, 2, 3, 4, 6, 12):
        cache = tmp_path / f"tune{rg}.txt"
        cache.write_text(f"{dk} K1_f32_nd_r12 128 1 1 {rg} 1.0\n{dk} K2_f32_nd_r12 64 0 1 {rg} 1.0\n")
        monkeypatch.setenv("TMX_TUNE_CACHE", str(cache))
        ctx = tmx.Context(DIMS)
        assert ctx.tuned_config("K1_f32_nd_r12")["rg"] == rg
        ctx.set_params(tmx.Params(KAPPA, CSW, 0.01, MUBAR, EPSBAR, -1))
        ctx.load_gauge(U, 8.0)
        out = ctx.empty(kind, 1, 12)
        ctx.apply_mhat(out, ctx.pack(to_dev(v), kind, 1, 12), 2, 1, 0, 12)
        got = to_host(ctx.unpack(out, kind, 1, 12), v.shape)
        ctx.close()
        assert rel_l2(got, ref) < 1e-6, rg
