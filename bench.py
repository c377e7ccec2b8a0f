#!/usr/bin/env python3
"""Benchmark of the twisted-mass clover hot path on one MI355X.

One step = one pass over the hot path on a 32^3x64 synthetic gauge field
(kappa = 0.1394, csw = 1.69, mu = 0.00072; two-flavour mubar = 0.1246,
epsbar = 0.1315; links U = proj_SU3(exp(i 0.25 H)), seed 4):

  * Schur operator Mhat applied to a Gaussian source in FP64, FP32 and FP16
    storage (NAPPLY applications each), the normal operator N in FP64 and
    the two-flavour Mhat_h in FP32;
  * plain FP64 CG on N to a 1e-10 FP64 true residual;
  * mixed-precision CG (FP32 and FP16-storage inner iterations, FP64
    reliable updates) to the same FP64 true residual;
  * CG preconditioned by the learned network K K^dagger (FP16 inner, FP64
    reliable updates; the network is trained before the timed region on 256
    (source, solution) pairs from the plain solver on a 16^3x32 field, the
    best of three initialisations by preconditioned-CG iterations on a
    held-out source of that field), by its Hermitian form P = A^dagger A
    (A = L_2 L_1; one network application per iteration; trained the same way
    on pairs (b, N^{-1} b) with the energy-norm loss) and by the short form
    P_1 = L_1^dagger L_1 (the one-channel layers only, trained likewise);
  * CG and FP16 MP-CG on the mass-preconditioned What^dagger What (rho = 0.02);
  * a 12-shift multishift solve of the two-flavour normal operator (FP32
    multishift CG, then FP64-reliable refinement per shift) at the poles of
    Zolotarev's 12-pole approximation of N_h^(-1/2) on [1e-5, 1] lambda_max,
    and 12 Gaussian right-hand sides of the two-flavour operator advanced
    together (FP32 inner, FP64 reliable updates), each also with FP16-storage
    inner iterations.
After the timed steps, once: the rational approximation applied as a whole
(R(N_h) b with the same poles), its accuracy N_h R(N_h)^2 b = b, and the
exponent of its correction factor for one Gaussian eta; the force of that
rational monomial (the 12 solutions' hopping and clover forces summed on the
device); the hopping-term force kernel (link outer products of one shift)
and the clover-term force (sigma-plane insertions, then the staple sums).

The headline value is the FP64 Schur-operator bandwidth: model bytes of one
Mhat application (links, spinors and clover blocks each read once per
stencil pass) divided by its measured time (HIP events on the library's
stream), summed over all timed steps.  All inputs are resident in HBM before
the timed region.  Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Schur dslash GB/s (% HBM peak); CG time-to-1e-10, plain vs mixed+learned PC"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KAPPA, CSW, MU, MUBAR, EPSBAR = 0.1394, 1.69, 0.00072, 0.1246, 0.1315
# mass-preconditioning mass of What^pm(rho): about 28 x mu, within the 20-30 x
# range of the light-sector determinant ratios the paper discusses (Section 4.1)
RHO = 0.02
NAPPLY = 20
# the network's 8 -> 8 layer per site: factorised C_d (x) Gamma_d mixing
# (9 paths x (8*8*12 + 4*4*24) complex multiply-adds x 8 flops) and its
# algorithmic bytes (BF16 activations in and out, eight BF16 links)
NN_LAYER_FLOPS_PER_SITE = 9 * (8 * 8 * 12 + 4 * 4 * 24) * 8
NN_LAYER_BYTES_PER_SITE = 384 + 384 + 8 * 36

# algorithmic bytes per output site of one stencil launch (links, blocks and
# spinors each read once)
from paper_2212_06635_amd.counters import kernel_bytes_per_site, read_traffic  # noqa: E402

PROFILE = os.path.join(ROOT, "profiles", "dslash_schur_32x32x32x64_kernels.txt")


def mhat_bytes_per_site(prec: str, nf: int = 1) -> float:
    k = "_nd" if nf == 2 else ""
    return kernel_bytes_per_site(f"K1_{prec}{k}") + kernel_bytes_per_site(f"K2_{prec}{k}")


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(dims, U, b, napply):
    """The FP64 oracle timed on the host cores on a bounded sample."""
    from oracle import Oracle
    from oracle.oracle import num_threads

    t = time.perf_counter()
    o = Oracle(dims, U, KAPPA, CSW, mu=MU)
    log(f"oracle clover built in {time.perf_counter() - t:.1f}s")
    o.mhat(b)  # warm
    t = time.perf_counter()
    for _ in range(napply):
        o.mhat(b)
    dt = (time.perf_counter() - t) / napply
    Vh = o.Vh
    gbs = mhat_bytes_per_site("f64") * Vh / dt / 1e9
    return o, {"value": gbs, "unit": "GB/s", "cores": num_threads(), "kind": "oracle",
               "sample": f"{napply} FP64 Mhat applications at {'x'.join(map(str, dims))} "
                         f"({dt:.3f} s each, same model bytes as the GPU figure)"}


def cpu_solves(o, b, b2, shifts, gpu_cg_iters, gpu_shift_iters):
    """The oracle's plain FP64 CG to a 1e-10 true residual on the host cores:
    run to the end at 8^4 and 16^3x32 (same generator and parameters), and
    at the benchmark lattice `o` timed over a few iterations and extrapolated
    to the iteration count of the same solve; the two-flavour 12-shift solve
    as twelve sequential single-shift CG solves, extrapolated the same way."""
    from oracle import Oracle
    from oracle.oracle import num_threads
    from paper_2212_06635_amd import synth

    out = {"kind": "oracle", "cores": num_threads()}
    for dims, seed in (((8, 8, 8, 8), 1), ((16, 16, 16, 32), 2)):
        U = synth.gauge_links(dims, 0.25, seed)
        od = Oracle(dims, U, KAPPA, CSW, mu=MU)
        bs = synth.gaussian_cb_spinor(dims, seed, 0)
        t = time.perf_counter()
        _, it, rel = od.cg(bs, tol=1e-10)
        out["cg_f64_" + "x".join(map(str, dims))] = {"seconds": round(time.perf_counter() - t, 3), "iters": it,
                                                     "true_residual": rel, "measured": "whole solve"}
    k = 3
    t = time.perf_counter()
    o.cg(b, tol=1e-10, maxiter=k)
    per_it = (time.perf_counter() - t) / (k + 1)  # k iterations and the final residual check
    out["cg_f64_" + "x".join(map(str, o.dims))] = {
        "seconds": round(per_it * gpu_cg_iters, 2), "seconds_per_iteration": round(per_it, 4), "iters": gpu_cg_iters,
        "measured": f"extrapolated: {k} iterations timed, times the {gpu_cg_iters} iterations of the same solve on the GPU"}
    t = time.perf_counter()
    o.cg(b2, nf=2, shift=float(shifts[0]), tol=1e-10, maxiter=2)
    per_it = (time.perf_counter() - t) / 3
    total = int(sum(gpu_shift_iters))
    out["multishift_nd_12_sequential_cg"] = {
        "seconds": round(per_it * total, 1), "seconds_per_iteration": round(per_it, 4), "iters_total": total,
        "measured": "extrapolated: 2 two-flavour CG iterations timed, times the sum over the 12 shifts of the "
                    "iterations each shift took on the GPU (multishift stage plus refinement)"}
    return out


# the preconditioner forms: solver kind, training loss, training pairs
# (b, Mhat^{-1} b) or (b, N^{-1} b), label
PC_FORMS = {
    "kk": ("TMX_SOLVER_PCG_NN", "TMX_LOSS_RESIDUAL", "mhat", "K K^dagger"),
    "sym": ("TMX_SOLVER_PCG_NN_SYM", "TMX_LOSS_SYM", "normal", "P = A^dagger A, A = L_2 L_1"),
    "sym1": ("TMX_SOLVER_PCG_NN_SYM1", "TMX_LOSS_SYM1", "normal", "P_1 = L_1^dagger L_1"),
}


def train_networks(tmx, synth, npairs, epochs, forms=("kk", "sym", "sym1"), inits=3):
    """Train the preconditioner forms on a 16^3x32 field (seed 2).

    K is trained on pairs (b, Mhat^{-1} b) with the residual loss, the
    Hermitian forms on pairs (b, N^{-1} b) with the energy-norm loss.  The
    losses are averages over Gaussian sources and do not see how the network
    treats the lowest modes, which set the iteration count of preconditioned
    CG; training runs from `inits` random initialisations are therefore
    compared by that count on a held-out source of the same training field,
    and the best is kept.  Nothing of the benchmark field enters the choice.
    Returns {form: (weights, record)}.
    """
    import numpy as np
    import torch

    dims = (16, 16, 16, 32)
    U = synth.gauge_links(dims, 0.25, 2)
    tc = tmx.Context(dims)
    tc.set_params(tmx.Params(KAPPA, CSW, MU, 0.0, 0.0, -1))
    tc.load_gauge(U, 2.0)
    n1 = tc.Vh * 12
    bs = torch.from_numpy(np.stack([synth.gaussian_cb_spinor(dims, 2, k) for k in range(npairs)]).reshape(-1)).cuda()
    pairs, pair_seconds = {}, {}
    for kind in sorted({PC_FORMS[f][2] for f in forms}):
        t0 = time.perf_counter()
        xs = torch.zeros_like(bs)
        for k in range(npairs):
            xk = torch.zeros(n1, dtype=torch.complex128, device="cuda")
            if kind == "normal":
                tc.solve(xk, bs[k * n1:(k + 1) * n1], 1, kind=tmx.TMX_SOLVER_MPCG_F32, op=1, tol=1e-10)
            else:
                tc.solve_mhat(xk, bs[k * n1:(k + 1) * n1], dagger=0, op=1, tol=1e-10)
            xs[k * n1:(k + 1) * n1] = xk
        pairs[kind] = xs
        pair_seconds[kind] = round(time.perf_counter() - t0, 1)
    bval = torch.from_numpy(synth.gaussian_cb_spinor(dims, 2, 10 ** 6).reshape(-1)).cuda()
    x = torch.zeros_like(bval)
    rc, info = tc.solve(x, bval, 1, kind=tmx.TMX_SOLVER_MPCG_F16, op=1, tol=1e-10)
    val_cg = info[0]["iters"]
    out = {}
    for form in forms:
        skind, lkind, ptype, label = PC_FORMS[form]
        kind, loss_kind = getattr(tmx, skind), getattr(tmx, lkind)
        t1 = time.perf_counter()
        runs, best = [], None
        for init in range(inits):
            w0 = np.zeros(tc.pc_num_params(), dtype=np.float32)
            # identity on the d = 0 path of every layer, N(0, 1e-2) elsewhere
            from_oracle_free_init(w0, np.random.default_rng(3 + init))
            tc.pc_set_weights(w0)
            losses = tc.pc_train(bs, pairs[ptype], npairs, epochs=epochs, batch=8, lr=3e-3, seed=1,
                                 loss_kind=loss_kind)
            x = torch.zeros_like(bval)
            rc, info = tc.solve(x, bval, 1, kind=kind, op=1, tol=1e-10, inner_prec=2)
            it = info[0]["iters"] if rc == tmx.TMX_OK else 10 ** 9
            runs.append({"init": init, "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                         "val_pcg_iters": it})
            if best is None or it < best[0]:
                best = (it, tc.pc_get_weights())
        out[form] = (best[1], {"form": label, "pairs": npairs, "lattice": list(dims),
                               "pair_seconds": pair_seconds[ptype], "train_seconds": round(time.perf_counter() - t1, 1),
                               "epochs": epochs, "runs": runs, "val_cg_iters": val_cg})
    tc.close()
    return out


def learned_pc_other_volume(tmx, synth, wts, dims=(24, 24, 24, 48), seed=3):
    """The trained weights (translation invariant; wts: solver kind ->
    weights) used unchanged on a second volume: plain CG, MP-CG, CG
    preconditioned by K K^dagger and by the Hermitian forms, and flexible GCR
    with K, each to a 1e-10 FP64 true residual (one warm-up solve each, then
    the median of three)."""
    import numpy as np
    import torch

    U = synth.gauge_links(dims, 0.25, seed)
    ctx = tmx.Context(dims)
    ctx.set_params(tmx.Params(KAPPA, CSW, MU, 0.0, 0.0, -1))
    ctx.load_gauge(U, float(seed))
    b = torch.from_numpy(synth.gaussian_cb_spinor(dims, seed, 0).reshape(-1)).cuda()
    x = torch.zeros_like(b)
    out = {"lattice": list(dims), "seed": seed}
    for kind, name, ip in ((tmx.TMX_SOLVER_CG, "cg_f64", 1), (tmx.TMX_SOLVER_MPCG_F16, "mpcg_f16", 1),
                           (tmx.TMX_SOLVER_PCG_NN, "pcg_nn_f16", 2), (tmx.TMX_SOLVER_FGCR_NN, "fgcr_nn_f32", 1),
                           (tmx.TMX_SOLVER_PCG_NN_SYM, "pcg_nn_sym_f16", 2),
                           (tmx.TMX_SOLVER_PCG_NN_SYM1, "pcg_nn_sym1_f16", 2)):
        if kind in wts:
            ctx.pc_set_weights(wts[kind])
        elif kind == tmx.TMX_SOLVER_FGCR_NN:
            ctx.pc_set_weights(wts[tmx.TMX_SOLVER_PCG_NN])
        times = []
        for rep in range(4):
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, info = ctx.solve(x, b, 1, kind=kind, op=1, tol=1e-10, inner_prec=ip, restart=16)
            torch.cuda.synchronize()
            if rep:
                times.append(time.perf_counter() - t)
        out[name] = {"seconds": sorted(times)[1], "iters": info[0]["iters"], "rc": rc,
                     "true_residual": info[0]["true_residual"], "fallback": info[0]["fallback"]}
    ctx.close()
    return out


def large_volume(tmx, synth, w_p1, base=(16, 16, 16, 128), rep=(4, 4, 4), seed=5, napply=10):
    """The 64^3x128 configuration on one GPU: a 16^3x128 field (eps 0.25, seed
    5) repeated 4x in x, y and z (periodic space directions; the antiperiodic
    time extent kept), Gaussian sources drawn on the whole 64^3x128 lattice.
    FP64 Mhat bandwidth (HIP events), plain FP64 CG, FP16 MP-CG and CG
    preconditioned by P_1 (weights trained on 16^3x32, translation invariant)
    to a 1e-10 FP64 true residual, and the 12-shift two-flavour multishift
    solve (FP16 inner) at the poles of Zolotarev's approximation of
    N_h^(-1/2) on [1e-5, 1] lambda_max of this field (the recipe of the
    32^3x64 run).  Run before the 32^3x64 context exists, and the multishift
    solve (about 250 GB at its peak) first, its scratch given back
    (tmx_free_workspaces) before the one-flavour fields are built."""
    import gc

    import numpy as np
    import torch

    from paper_2212_06635_amd import zolotarev

    dims = tuple(base[i] * (rep[i] if i < 3 else 1) for i in range(4))
    U0 = synth.gauge_links(base, 0.25, seed)
    U = np.tile(U0, (1, rep[2], rep[1], rep[0], 1, 1, 1))
    ctx = tmx.Context(dims)
    ctx.set_params(tmx.Params(KAPPA, CSW, MU, MUBAR, EPSBAR, -1))
    ctx.load_gauge(U, float(seed))
    del U, U0
    gc.collect()
    out = {"lattice": list(dims), "field": f"{'x'.join(map(str, base))} (eps 0.25, seed {seed}) tiled "
                                          f"{'x'.join(map(str, rep))} in x, y, z; Gaussian sources on the whole lattice"}
    b2 = torch.from_numpy(synth.gaussian_cb_spinor(dims, seed, 1, 2).reshape(-1)).cuda()
    v = ctx.pack(b2, tmx.TMX_FIELD_ODD_ND, 1)
    w2 = ctx.empty(tmx.TMX_FIELD_ODD_ND, 1)
    lam = 0.0
    for _ in range(30):
        ctx.apply_mdagm(w2, v, 2, 1)
        wc = ctx.unpack(w2, tmx.TMX_FIELD_ODD_ND, 1)
        vc = ctx.unpack(v, tmx.TMX_FIELD_ODD_ND, 1)
        lam = float(torch.vdot(vc, wc).real / torch.vdot(vc, vc).real)
        v = ctx.pack(wc / wc.norm(), tmx.TMX_FIELD_ODD_ND, 1)
    del v, w2, wc, vc
    lam_max = 1.05 * lam
    shifts = zolotarev.for_spectrum(12, 1e-5 * lam_max, lam_max).shifts
    out["lambda_max_nd"] = round(lam, 5)
    xs = torch.zeros(len(shifts) * b2.numel(), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    rc, info = ctx.multishift_solve(xs, b2, shifts, op=2, tol=1e-10, inner_prec=2)
    torch.cuda.synchronize()
    out["multishift_nd_12_f16"] = {"seconds": round(time.perf_counter() - t, 3), "rc": rc,
                                   "iters": [i["iters"] for i in info],
                                   "max_true_residual": max(i["true_residual"] for i in info)}
    log(f"64^3x128 multishift: {time.perf_counter() - t:.2f}s")
    del xs, b2
    # the multishift solve's scratch (about 250 GB at its peak) goes back
    # before the one-flavour operator's fields and the network are built
    ctx.free_workspaces()
    gc.collect()
    torch.cuda.empty_cache()
    b = torch.from_numpy(synth.gaussian_cb_spinor(dims, seed, 0).reshape(-1)).cuda()
    src = ctx.pack(b, tmx.TMX_FIELD_ODD, 0)
    dst = ctx.empty(tmx.TMX_FIELD_ODD, 0)
    for _ in range(2):
        ctx.apply_mhat(dst, src, 1, 0)
    torch.cuda.synchronize()
    ctx.kstats_enable(True)
    for _ in range(napply):
        ctx.apply_mhat(dst, src, 1, 0)
    torch.cuda.synchronize()
    ks = ctx.kstats()
    ctx.kstats_enable(False)
    ms = sum(ks[k][1] for k in ("K1_f64", "K2_f64") if k in ks) / napply
    gbs = mhat_bytes_per_site("f64") * ctx.Vh / (ms * 1e-3) / 1e9
    out["mhat_f64"] = {"ms": round(ms, 3), "GBps": round(gbs, 1), "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 1)}
    del src, dst
    ctx.pc_set_weights(w_p1)
    x = torch.zeros_like(b)
    for kind, name, ip in ((tmx.TMX_SOLVER_MPCG_F16, "warm-up", 1), (tmx.TMX_SOLVER_CG, "cg_f64", 1),
                           (tmx.TMX_SOLVER_MPCG_F16, "mpcg_f16", 1), (tmx.TMX_SOLVER_PCG_NN_SYM1, "pcg_nn_sym1_f16", 2)):
        x.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, info = ctx.solve(x, b, 1, kind=kind, op=1, tol=1e-10, inner_prec=ip)
        torch.cuda.synchronize()
        if name != "warm-up":
            out[name] = {"seconds": round(time.perf_counter() - t, 4), "iters": info[0]["iters"], "rc": rc,
                         "true_residual": info[0]["true_residual"], "fallback": info[0]["fallback"]}
        log(f"64^3x128 {name}: {time.perf_counter() - t:.2f}s")
    del x, b
    ctx.close()
    gc.collect()
    torch.cuda.empty_cache()
    return out


def from_oracle_free_init(w, rng):
    """Identity initialisation of the network weights (layout of tmx_pc_set_weights)."""
    chans = [(1, 8), (8, 8), (8, 8), (8, 1)]
    k = 0
    for ci, co in chans:
        for d in range(9):
            n = 2 * (co * ci + 16)
            w[k:k + n] = rng.standard_normal(n) * 1e-2
            if d == 0:
                C = w[k:k + 2 * co * ci].reshape(co, ci, 2)
                C[:] = 0
                for i in range(min(co, ci)):
                    C[i, i, 0] = 1.0
                G = w[k + 2 * co * ci:k + n].reshape(4, 4, 2)
                G[:] = 0
                for i in range(4):
                    G[i, i, 0] = 1.0
            k += n
    assert k == w.size


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dims", default="32,32,32,64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-applies", type=int, default=3)
    ap.add_argument("--mode", default="full", choices=["full", "kernels", "nn", "force"],
                    help="kernels: only Mhat applies per precision and a copy of known size (for counters); "
                         "nn: only applications of the learned preconditioner (for counters)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuning of the stencil launch shapes (done before the timed region by default)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 64^3x128 configuration run after the timed steps")
    ap.add_argument("--train-pairs", type=int, default=256)
    ap.add_argument("--train-epochs", type=int, default=20)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one MI355X: the path is built and validated for a single GPU "
              "(multi-GPU sharding is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2212_06635_amd.tmx as tmx
    from paper_2212_06635_amd import synth, zolotarev

    dims = tuple(int(x) for x in args.dims.split(","))
    torch.cuda.set_device(0)
    large = None
    if args.mode == "full":
        # the networks first (their own 16^3x32 context), then the 64^3x128
        # configuration, each with the GPU to itself
        trained = train_networks(tmx, synth, args.train_pairs, args.train_epochs)
        if dims == (32, 32, 32, 64) and not args.no_large:
            log("the 64^3x128 configuration")
            large = large_volume(tmx, synth, trained["sym1"][0])
    log(f"generating {dims} gauge field")
    U = synth.gauge_links(dims, 0.25, 4)
    b = synth.gaussian_cb_spinor(dims, 4, 0)
    b2 = synth.gaussian_cb_spinor(dims, 4, 1, 2)
    ctx = tmx.Context(dims)
    ctx.set_params(tmx.Params(KAPPA, CSW, MU, MUBAR, EPSBAR, -1, rho=RHO))
    ctx.load_gauge(U, 4.0)
    Vh = ctx.Vh
    bd = torch.from_numpy(b.reshape(-1)).cuda()
    b2d = torch.from_numpy(b2.reshape(-1)).cuda()
    src = {p: ctx.pack(bd, tmx.TMX_FIELD_ODD, p) for p in (0, 1, 2)}
    dst = {p: ctx.empty(tmx.TMX_FIELD_ODD, p) for p in (0, 1, 2)}
    src_nd = ctx.pack(b2d, tmx.TMX_FIELD_ODD_ND, 1)
    dst_nd = ctx.empty(tmx.TMX_FIELD_ODD_ND, 1)
    x = torch.zeros_like(bd)
    names = {0: "f64", 1: "f32", 2: "f16"}
    tuned = {}
    if not args.no_tune and args.mode in ("full", "kernels"):
        # every stencil the timed steps use: one right-hand side in three
        # precisions, the two-flavour operator in FP32 / FP16 / FP64 (FP64 for
        # the reliable updates), and the 12 two-flavour right-hand sides.
        # With TMX_TUNE_CACHE set, the choices are appended to that file and a
        # later context of the same lattice (a profiled --no-tune run) starts
        # from them.
        t = time.perf_counter()
        for p in (0, 1, 2):
            ctx.tune(p, 1, 1)
            ctx.tune(p, 2, 1)
        ctx.tune(1, 2, 12)
        ctx.tune(2, 2, 12)
        ctx.tune(0, 2, 12)
        tuned = {k: ctx.tuned_config(k) for k in ("K1_f64", "K2_f64", "K1_f32", "K2_f32", "K1_f16", "K2_f16",
                                                   "K1_f32_nd", "K2_f32_nd", "K1_f32_nd_r12", "K2_f32_nd_r12",
                                                   "K1_f16_nd_r12", "K2_f16_nd_r12")}
        log(f"tuned in {time.perf_counter() - t:.1f}s: {tuned}")
    log("setup done")
    if args.mode == "nn":
        w0 = np.zeros(ctx.pc_num_params(), dtype=np.float32)
        from_oracle_free_init(w0, np.random.default_rng(3))
        ctx.pc_set_weights(w0)
        o = torch.zeros_like(bd)
        for mode in (0, 3):  # K, then the short Hermitian form P_1 through path channels
            for _ in range(5):
                ctx.pc_apply(o, bd, mode)
        # a device copy of 2 GiB, whose FETCH_SIZE / WRITE_SIZE calibrate the counters
        a = torch.empty(2 ** 28, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "nn", "lattice": list(dims), "applies": {"K": 5, "P_1": 5}}), flush=True)
        ctx.close()
        return
    if args.mode == "force":
        # 10 hopping-term force calls (two K1 launches and the force kernel
        # each), then the 2 GiB calibration copies
        fy = torch.from_numpy(synth.gaussian_cb_spinor(dims, 4, 1).reshape(-1)).cuda()
        fbuf = torch.zeros(Vh * 2 * 36, dtype=torch.complex128, device="cuda")
        for _ in range(10):
            ctx.hop_force(fbuf, bd, fy, op=1)
        for _ in range(10):
            ctx.clover_force(fbuf, bd, fy, op=1)
        a = torch.empty(2 ** 28, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "force", "lattice": list(dims), "calls": 10, "Vh": Vh}), flush=True)
        ctx.close()
        return
    if args.mode == "kernels":
        # a fixed number of applies per precision, then a device copy of
        # 2 GiB whose FETCH_SIZE / WRITE_SIZE calibrate the counters
        for p in (0, 1, 2):
            for _ in range(10):
                ctx.apply_mhat(dst[p], src[p], 1, p)
        a = torch.empty(2 ** 28, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "kernels", "lattice": list(dims), "applies_per_prec": 10,
                          "copy_bytes_each_way": a.numel() * 8, "copies": 3,
                          "kernel_bytes_per_site": {k: kernel_bytes_per_site(k) for k in
                                                    ("K1_f64", "K2_f64", "K1_f32", "K2_f32", "K1_f16", "K2_f16")},
                          "Vh": Vh}), flush=True)
        ctx.close()
        return

    wts = {getattr(tmx, PC_FORMS[f][0]): trained[f][0] for f in trained}
    ctx.pc_set_weights(trained["kk"][0])
    # largest eigenvalue of N_h by power iteration (FP32), for the shifts
    v = ctx.pack(b2d, tmx.TMX_FIELD_ODD_ND, 1)
    w2 = ctx.empty(tmx.TMX_FIELD_ODD_ND, 1)
    lam = 0.0
    for _ in range(30):
        ctx.apply_mdagm(w2, v, 2, 1)
        wc = ctx.unpack(w2, tmx.TMX_FIELD_ODD_ND, 1)
        vc = ctx.unpack(v, tmx.TMX_FIELD_ODD_ND, 1)
        lam = float(torch.vdot(vc, wc).real / torch.vdot(vc, vc).real)
        v = ctx.pack(wc / wc.norm(), tmx.TMX_FIELD_ODD_ND, 1)
    lam_max = 1.05 * lam
    # poles of Zolotarev's approximation of N_h^(-1/2) on [1e-5, 1] lambda_max
    zolo = zolotarev.for_spectrum(12, 1e-5 * lam_max, lam_max)
    shifts = zolo.shifts
    xs_ms = torch.zeros(12 * b2d.numel(), dtype=torch.complex128, device="cuda")
    b12 = torch.from_numpy(np.stack([synth.gaussian_cb_spinor(dims, 4, 100 + k, 2) for k in range(12)]).reshape(-1)).cuda()
    x12 = torch.zeros_like(b12)
    log(f"lambda_max(N_h) ~ {lam:.4f}; network trained ({ {f: trained[f][1]['runs'] for f in trained} })")

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        return e0, e1

    # solves whose kernels the library's per-kernel events record in the timed
    # steps: the FP64 CGs (the K1 launches of the roofline) and the K K^dagger
    # solve (the 8->8 layer's roofline); the other solves and the operator
    # loops run without them (two event records per launch cost 2 % of an
    # FP64 Mhat and 7 % of an FP16 one).  One further step with every solve
    # recorded gives the per-kernel table.
    recorded = {"cg_f64", "cg_w_f64", "pcg_nn_f16"}

    def step(record_all=False):
        ctx.kstats_enable(False)
        ev = {}
        for p in (0, 1, 2):
            ev[names[p]] = timed(lambda: [ctx.apply_mhat(dst[p], src[p], 1, p) for _ in range(NAPPLY)])
        ev["N_f64"] = timed(lambda: [ctx.apply_mdagm(dst[0], src[0], 1, 0) for _ in range(NAPPLY)])
        ev["nd_f32"] = timed(lambda: [ctx.apply_mhat(dst_nd, src_nd, 2, 1) for _ in range(NAPPLY)])
        step_ks = {}

        def record(on):
            # kstats_enable clears the library's table: fold it in first
            for name, (n, ms) in ctx.kstats().items():
                n0, ms0 = step_ks.get(name, (0, 0.0))
                step_ks[name] = (n0 + n, ms0 + ms)
            ctx.kstats_enable(on)

        solves = {}
        for kind, nm, ip, op in ((tmx.TMX_SOLVER_CG, "cg_f64", 1, 1), (tmx.TMX_SOLVER_MPCG_F32, "mpcg_f32", 1, 1),
                                 (tmx.TMX_SOLVER_MPCG_F16, "mpcg_f16", 1, 1), (tmx.TMX_SOLVER_PCG_NN, "pcg_nn_f16", 2, 1),
                                 (tmx.TMX_SOLVER_PCG_NN_SYM, "pcg_nn_sym_f16", 2, 1),
                                 (tmx.TMX_SOLVER_PCG_NN_SYM1, "pcg_nn_sym1_f16", 2, 1),
                                 # the mass-preconditioned normal operator What^dagger What
                                 (tmx.TMX_SOLVER_CG, "cg_w_f64", 1, tmx.TMX_OP_WPLUS),
                                 (tmx.TMX_SOLVER_MPCG_F16, "mpcg_w_f16", 1, tmx.TMX_OP_WPLUS)):
            if kind in wts:
                ctx.pc_set_weights(wts[kind])
            record(record_all or nm in recorded)
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, info = ctx.solve(x, bd, 1, kind=kind, op=op, tol=1e-10, inner_prec=ip)
            solves[nm] = {"seconds": time.perf_counter() - t, "iters": info[0]["iters"],
                          "reliable_updates": info[0]["reliable_updates"],
                          "true_residual": info[0]["true_residual"], "fallback": info[0]["fallback"], "rc": rc}
        record(record_all)
        xs_ms.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, info = ctx.multishift_solve(xs_ms, b2d, shifts, op=2, tol=1e-10, inner_prec=1)
        solves["multishift_nd_12"] = {"seconds": time.perf_counter() - t, "rc": rc,
                                      "iters": [i["iters"] for i in info],
                                      "max_true_residual": max(i["true_residual"] for i in info)}
        for kind, nm in ((tmx.TMX_SOLVER_MPCG_F32, "mrhs_nd_12_mpcg_f32"), (tmx.TMX_SOLVER_MPCG_F16, "mrhs_nd_12_mpcg_f16")):
            x12.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            rc, info = ctx.solve(x12, b12, 12, kind=kind, op=2, tol=1e-10)
            solves[nm] = {"seconds": time.perf_counter() - t, "rc": rc, "iters": max(i["iters"] for i in info),
                          "max_true_residual": max(i["true_residual"] for i in info)}
        # the same multishift with FP16-storage shift vectors
        xs_ms.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, info = ctx.multishift_solve(xs_ms, b2d, shifts, op=2, tol=1e-10, inner_prec=2)
        solves["multishift_nd_12_f16"] = {"seconds": time.perf_counter() - t, "rc": rc,
                                          "iters": [i["iters"] for i in info],
                                          "max_true_residual": max(i["true_residual"] for i in info)}
        record(False)
        return ev, solves, step_ks

    for w in range(args.warmup):
        step()
        log(f"warmup step {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs, last, ks = [], None, {}
    for k in range(args.steps):
        ev, last, step_ks = step()
        evs.append(ev)
        for name, (n, ms) in step_ks.items():  # per-kernel launches and time over the timed steps
            n0, ms0 = ks.get(name, (0, 0.0))
            ks[name] = (n0 + n, ms0 + ms)
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel times of every solve (outside the timed region)
    _, _, ks_all = step(record_all=True)

    def gbs(key, per_site):
        ms = sum(e[key][0].elapsed_time(e[key][1]) for e in evs)
        return per_site * Vh * NAPPLY * len(evs) / (ms * 1e-3) / 1e9, ms / (NAPPLY * len(evs))

    dslash = {}
    for p in ("f64", "f32", "f16"):
        g, ms = gbs(p, mhat_bytes_per_site(p))
        dslash[p] = {"GBps": round(g, 1), "pct_hbm_peak": round(100 * g / HBM_PEAK_GBS, 1), "ms": round(ms, 4)}
    g, ms = gbs("N_f64", 2 * mhat_bytes_per_site("f64"))
    dslash["N_f64"] = {"GBps": round(g, 1), "pct_hbm_peak": round(100 * g / HBM_PEAK_GBS, 1), "ms": round(ms, 4)}
    g, ms = gbs("nd_f32", mhat_bytes_per_site("f32", 2))
    dslash["nd_f32"] = {"GBps": round(g, 1), "pct_hbm_peak": round(100 * g / HBM_PEAK_GBS, 1), "ms": round(ms, 4)}

    # dominant kernel of the Schur dslash in the timed region: the stencil
    # kernel (K1/K2, degenerate, one right-hand side) with the largest summed time
    stencil = {k: v for k, v in ks.items() if k[:2] in ("K1", "K2") and "_nd" not in k and "_r" not in k}
    dom = max(stencil.items(), key=lambda kv: kv[1][1])
    dname, (dcount, dms) = dom
    per_launch_bytes = kernel_bytes_per_site(dname) * Vh
    avg_ms = dms / dcount
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    # HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary
    # (null unless it was taken at this size from the current kernel sources)
    traffic = read_traffic(PROFILE, dname) if dims == (32, 32, 32, 64) else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dname,
                "avg_launch_ms": round(avg_ms, 4), "launches": dcount,
                "bytes_per_launch": per_launch_bytes}

    # the learned preconditioner's 8->8 layer.  The method's work per site is
    # the factorised mixing (C_d (x) Gamma_d): per path 8x8 channel and 4x4 spin
    # complex products on 12 and 24 vectors, 1152 complex multiply-adds = 9216
    # flops, 82,944 over the nine paths; its algorithmic traffic is 1056 B
    # (8 channels in and out at 384 B in BF16, eight 36-B links).  At 78
    # flop/B, below the BF16 ridge of 312 flop/B, the layer is bound by HBM;
    # the dense real 64x64 form it runs on the matrix cores (221 kflop/site)
    # is reported beside it, labelled as such.
    nn_roof = None
    if "NN_8x8" in ks:
        n, ms_tot = ks["NN_8x8"]
        sec = ms_tot / n * 1e-3
        nbytes = NN_LAYER_BYTES_PER_SITE * 2 * Vh
        gb = nbytes / sec / 1e9
        tf = NN_LAYER_FLOPS_PER_SITE * 2 * Vh / sec / 1e12
        tf_dense = 2 * 64 * 64 * 27 * 2 * Vh / sec / 1e12
        nn_roof = {"bound": "hbm", "achieved": round(gb, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(gb / HBM_PEAK_GBS, 4), "kernel": "NN_8x8", "avg_launch_ms": round(ms_tot / n, 4),
                   "bytes_per_site": NN_LAYER_BYTES_PER_SITE, "flops_per_site": NN_LAYER_FLOPS_PER_SITE,
                   "tflops_method": round(tf, 2), "frac_bf16_mfma_method": round(tf / 2500.0, 5),
                   "tflops_dense_equivalent": round(tf_dense, 2),
                   "frac_bf16_mfma_dense_equivalent": round(tf_dense / 2500.0, 5)}

    out = {
        "metric": METRIC,
        "value": dslash["f64"]["GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((t1 - t0) * 1e3 / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "32^3x64 Wilson twisted-mass clover: Schur Mhat apply + CG / MP-CG to 1e-10"
                   if dims == (32, 32, 32, 64) else f"{'x'.join(map(str, dims))} twisted-mass clover",
                   "lattice": list(dims), "kappa": KAPPA, "csw": CSW, "mu": MU, "mubar": MUBAR,
                   "epsbar": EPSBAR, "rho": RHO, "link_eps": 0.25, "seed": 4, "t_bc": "antiperiodic"},
        "pct_hbm_peak": dslash["f64"]["pct_hbm_peak"],
        "dslash": dslash,
        "solves": last,
        "kernels_ms": {k: round(v[1] / v[0], 4) for k, v in ks_all.items()},
        "roofline": roofline,
        "roofline_nn_layer": nn_roof,
        "learned_pc_training": trained["kk"][1],
        "learned_pc_training_sym": trained["sym"][1],
        "learned_pc_training_sym1": trained["sym1"][1],
        "tuned_launch": tuned,
    }
    # the learned-preconditioner forms against plain FP64 CG (same source, same
    # 1e-10 target; the last timed step)
    forms = {"pcg_nn_f16": "P = K K^dagger", "pcg_nn_sym_f16": "P = L1^dagger L2^dagger L2 L1",
             "pcg_nn_sym1_f16": "P = L1^dagger L1"}
    t_cg = last["cg_f64"]["seconds"]
    out["learned_pc_vs_plain_cg"] = {
        "plain_cg_f64_seconds": round(t_cg, 4),
        "forms": {k: {"preconditioner": v, "seconds": round(last[k]["seconds"], 4), "iters": last[k]["iters"],
                      "speedup_vs_plain_cg": round(t_cg / last[k]["seconds"], 2)} for k, v in forms.items()},
        "fastest": min(forms, key=lambda k: last[k]["seconds"]),
    }
    # the rational approximation as a whole: R(N_h) b, then N_h R(N_h)^2 b = b
    log("rational approximation R(N_h) b (FP16 inner) and its accuracy")
    rb = torch.zeros_like(b2d)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rc, rinfo = ctx.rational_apply(rb, b2d, zolo.a0, zolo.a, zolo.shifts, op=2, tol=1e-10, inner_prec=2)
    torch.cuda.synchronize()
    t_rat = time.perf_counter() - t
    rrb = torch.zeros_like(b2d)
    ctx.rational_apply(rrb, rb, zolo.a0, zolo.a, zolo.shifts, op=2, tol=1e-10, inner_prec=2)
    v_in = ctx.pack(rrb, tmx.TMX_FIELD_ODD_ND, 0)
    v_out = ctx.empty(tmx.TMX_FIELD_ODD_ND, 0)
    ctx.apply_mdagm(v_out, v_in, 2, 0)
    back = ctx.unpack(v_out, tmx.TMX_FIELD_ODD_ND, 0)
    out["rational_nd_12_f16"] = {"seconds": round(t_rat, 4), "rc": rc, "poles": 12,
                                 "interval": [1e-5 * lam_max, lam_max], "delta": zolo.delta,
                                 "iters": [i["iters"] for i in rinfo],
                                 "check_N_R2_b": float((back - b2d).norm() / b2d.norm())}
    # the correction term of the approximation for one Gaussian eta (density exp(-|eta|^2))
    eta = torch.from_numpy(synth.gaussian_cb_spinor(dims, 4, 200, 2).reshape(-1) / np.sqrt(2.0)).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rc, e_corr, nterms = ctx.rational_correction(eta, zolo.a0, zolo.a, zolo.shifts, series_tol=1e-6, maxterms=6,
                                                 op=2, tol=1e-10, inner_prec=2)
    torch.cuda.synchronize()
    out["rational_correction_nd_12_f16"] = {"seconds": round(time.perf_counter() - t, 4), "rc": rc,
                                            "exponent": e_corr, "terms": nterms,
                                            "eta_norm2": float(eta.norm() ** 2)}
    # the heavy sector's rational force: the 12 multishift solutions of R(N_h)
    # phi, each shift's hopping and clover force -2 a_k F(x_k, Mhat_h x_k)
    # added on the device (Sections 4.2, 4.3)
    log("rational force of the two-flavour monomial (12 poles)")
    fnd = torch.zeros(Vh * 2 * 36, dtype=torch.complex128, device="cuda")
    ctx.rational_force(fnd, b2d, zolo.a, zolo.shifts, op=2, tol=1e-10, inner_prec=2)  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    rc, finfo = ctx.rational_force(fnd, b2d, zolo.a, zolo.shifts, op=2, tol=1e-10, inner_prec=2)
    torch.cuda.synchronize()
    out["rational_force_nd_12_f16"] = {"seconds": round(time.perf_counter() - t, 4), "rc": rc, "poles": 12,
                                       "max_true_residual": max(i["true_residual"] for i in finfo),
                                       "force_norm": float(fnd.norm())}
    del fnd
    # hopping-term force: the link outer products of one shift (Section 4.3)
    log("hopping-term force")
    fbuf = torch.zeros(Vh * 2 * 36, dtype=torch.complex128, device="cuda")
    ctx.hop_force(fbuf, x, bd, op=1)
    torch.cuda.synchronize()
    ctx.kstats_enable(True)
    for _ in range(5):
        ctx.hop_force(fbuf, x, bd, op=1)
    torch.cuda.synchronize()
    fks = ctx.kstats()
    ctx.kstats_enable(False)
    if "HOP_FORCE" in fks:
        n, ms_tot = fks["HOP_FORCE"]
        fbytes = 1344.0 * 2 * Vh  # a, b fields (2 x 192 B), 4 links (4 x 96 B), 4 outputs (4 x 144 B) per site
        out["hop_force_f64"] = {"kernel_ms": round(ms_tot / n, 4), "GBps": round(fbytes / (ms_tot / n * 1e-3) / 1e9, 1),
                                "bytes_per_site": 1344}
    # clover-term force: six sigma-plane insertions per site, the plaquette
    # loops with the insertion at every corner, then the link sums
    ctx.kstats_enable(True)
    for _ in range(5):
        ctx.clover_force(fbuf, x, bd, op=1)
    torch.cuda.synchronize()
    cks = ctx.kstats()
    ctx.kstats_enable(False)
    if "CLOVER_FORCE" in cks:
        n, ms_tot = cks["CLOVER_FORCE"]
        # a, b (384 B) + Hermitian insertions written and read (2 x 6 x 72 B) + 4 links (384 B) + 4 outputs
        # (576 B); the plaquette loops the link sums read back (6 x 144 B written and read) are not counted
        cbytes = 2208.0 * 2 * Vh
        out["clover_force_f64"] = {"kernel_ms": round(ms_tot / n, 4),
                                   "GBps": round(cbytes / (ms_tot / n * 1e-3) / 1e9, 1), "bytes_per_site": 2208}
    del fbuf
    if dims == (32, 32, 32, 64):
        log("learned preconditioner on a 24^3x48 field")
        out["learned_pc_24x24x24x48"] = learned_pc_other_volume(tmx, synth, wts)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        o, cb = cpu_baseline(dims, U, b, args.cpu_applies)
        out["cpu_baseline"] = cb
        # the plain-CG solution of the last step, checked by the oracle's operator
        x.zero_()
        ctx.solve(x, bd, 1, kind=tmx.TMX_SOLVER_MPCG_F16, op=1, tol=1e-10)
        out["solves"]["mpcg_f16"]["oracle_true_residual"] = o.residual(b, x.cpu().numpy().reshape(b.shape))
        log("timing the oracle's CG")
        o.mubar, o.epsbar = MUBAR, EPSBAR
        out["cpu_baseline_solves"] = cpu_solves(o, b, b2, shifts, out["solves"]["cg_f64"]["iters"],
                                                out["solves"]["multishift_nd_12"]["iters"])
    else:
        out["cpu_baseline"] = None
    ctx.close()
    if large is not None:
        out["large_64x64x64x128"] = large
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
