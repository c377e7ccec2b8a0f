"""GPU learned preconditioner against the FP64 network oracle.

The GPU network stages transported activations and weights in BF16 (8-bit
mantissa, relative rounding 2^-9) and accumulates in FP32, over four layers;
outputs are compared to the oracle to relative L2 <= 2e-2 and gradients by
relative L2 <= 5e-2 with cosine >= 0.999.
"""
import numpy as np
import pytest

from helpers import CSW, KAPPA, rel_l2, to_dev, to_host
from oracle import Oracle
from oracle import nn_oracle as nn
from paper_2212_06635_amd import synth

pytestmark = pytest.mark.gpu

DIMS = (8, 8, 4, 8)
MU0 = 0.01


@pytest.fixture(scope="module")
def S():
    import paper_2212_06635_amd.tmx as tmx

    print("\n[gpu nn] 8x8x4x8 eps=0.3", flush=True)
    U = synth.gauge_links(DIMS, 0.3, 31)
    ctx = tmx.Context(DIMS)
    ctx.set_params(tmx.Params(KAPPA, CSW, MU0, 0.0, 0.0, -1))
    ctx.load_gauge(U, 31.0)
    lat = nn.Lattice(DIMS, U, t_bc=-1)
    yield tmx, ctx, lat, U
    ctx.close()


def f32(w):
    return np.asarray(w, dtype=np.float32).astype(np.float64)


def test_param_count(S):
    tmx, ctx, lat, _ = S
    assert ctx.pc_num_params() == nn.num_params()


def test_identity_network(S):
    tmx, ctx, lat, _ = S
    w = nn.identity_init(None)
    ctx.pc_set_weights(w)
    b = synth.gaussian_cb_spinor(DIMS, 40, 0)
    out = to_dev(np.zeros_like(b))
    ctx.pc_apply(out, to_dev(b), 0)
    assert rel_l2(to_host(out, b.shape), b) < 1e-2
    assert np.allclose(ctx.pc_get_weights(), w.astype(np.float32))


@pytest.mark.parametrize("dagger", [0, 1])
def test_random_network_matches_oracle(S, dagger):
    tmx, ctx, lat, _ = S
    rng = np.random.default_rng(41)
    w = (rng.standard_normal(nn.num_params()) * 0.3).astype(np.float32)
    ctx.pc_set_weights(w)
    b = synth.gaussian_cb_spinor(DIMS, 41, 0)
    out = to_dev(np.zeros_like(b))
    ctx.pc_apply(out, to_dev(b), dagger)
    ref = (nn.adjoint if dagger else nn.forward)(lat, f32(w), b[:, 0])
    assert rel_l2(to_host(out, b.shape)[:, 0], ref) < 2e-2


@pytest.mark.parametrize("loss_kind,op", [(0, 1), (1, 1), (0, -1)])
def test_gradient_matches_oracle(S, loss_kind, op):
    """GPU loss and weight gradient (residual and solution losses; the residual
    loss also for Mhat(-mu), the operator of separately trained weights)
    against the oracle's."""
    tmx, ctx, lat, U = S
    rng = np.random.default_rng(42)
    w = (nn.identity_init(rng, 0.1)).astype(np.float32)
    ctx.pc_set_weights(w)
    bs = np.stack([synth.gaussian_cb_spinor(DIMS, 42, k) for k in range(2)])
    xs = np.stack([synth.gaussian_cb_spinor(DIMS, 43, k) for k in range(2)])
    loss, g = ctx.pc_loss_grad(to_dev(bs), to_dev(xs), 2, loss_kind, op)
    ops = ()
    if loss_kind == 0:
        o = Oracle(DIMS, U, KAPPA, CSW, mu=MU0)
        ops = (lambda v: o.mhat(v.reshape(-1, 1, 4, 3), sgn=op).reshape(-1, 4, 3),
               lambda v: o.mhat(v.reshape(-1, 1, 4, 3), sgn=op, dagger=True).reshape(-1, 4, 3))
    L, gref = nn.loss_and_grad(lat, f32(w), [b[:, 0] for b in bs], [x[:, 0] for x in xs], *ops)
    assert abs(loss - L) / L < 2e-2
    cos = float(np.dot(g, gref) / np.linalg.norm(g) / np.linalg.norm(gref))
    assert cos > 0.999, cos
    assert rel_l2(g, gref) < 5e-2


@pytest.fixture(scope="module")
def pairs(S):
    """(b, x = Mhat^{-1} b) from the plain solver on the same field."""
    tmx, ctx, lat, U = S
    n = 16
    bs = np.stack([synth.gaussian_cb_spinor(DIMS, 50, k) for k in range(n)])
    xd = to_dev(np.zeros_like(bs))
    for k in range(n):
        xk = to_dev(np.zeros_like(bs[k]))
        rc, info = ctx.solve_mhat(xk, to_dev(bs[k]), dagger=0, op=1, tol=1e-10)
        assert rc == tmx.TMX_OK
        xd[k * bs[k].size:(k + 1) * bs[k].size] = xk
    return bs, xd


@pytest.mark.parametrize("loss_kind", [1, 0])
def test_training_reduces_loss(S, pairs, loss_kind):
    tmx, ctx, lat, _ = S
    bs, xd = pairs
    ctx.pc_set_weights(nn.identity_init(np.random.default_rng(3), 1e-2))
    losses = ctx.pc_train(to_dev(bs), xd, len(bs), epochs=12, batch=4, lr=3e-3, seed=1, loss_kind=loss_kind)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.7 * losses[0], losses


def test_trained_network_beats_untrained(S, pairs):
    """What the trained network gains: preconditioned-CG iterations, trained vs identity network."""
    tmx, ctx, lat, _ = S
    bs, xd = pairs
    b = to_dev(synth.gaussian_cb_spinor(DIMS, 62, 0))
    ctx.pc_set_weights(nn.identity_init(None))
    x = b * 0
    rc0, info0 = ctx.solve(x, b, 1, kind=tmx.TMX_SOLVER_PCG_NN, op=1, tol=1e-10)
    ctx.pc_set_weights(nn.identity_init(np.random.default_rng(3), 1e-2))
    ctx.pc_train(to_dev(bs), xd, len(bs), epochs=30, batch=4, lr=3e-3, seed=2, loss_kind=0)
    x = b * 0
    rc1, info1 = ctx.solve(x, b, 1, kind=tmx.TMX_SOLVER_PCG_NN, op=1, tol=1e-10)
    print("PCG iterations identity / trained:", info0[0]["iters"], info1[0]["iters"])
    assert rc0 == tmx.TMX_OK and rc1 == tmx.TMX_OK
    # both on the preconditioned path itself (a fallback would add plain-CG iterations)
    assert info0[0]["fallback"] == 0 and info1[0]["fallback"] == 0, (info0, info1)
    assert info1[0]["iters"] < info0[0]["iters"], (info0, info1)


def test_fgcr_reaches_target(S, pairs):
    """FGCR with the trained network converges on its own (no CG fallback):
    FP64 true residual <= 1e-10 by the oracle operator."""
    tmx, ctx, lat, U = S
    bs, xd = pairs
    o = Oracle(DIMS, U, KAPPA, CSW, mu=MU0)
    ctx.pc_set_weights(nn.identity_init(np.random.default_rng(3), 1e-2))
    ctx.pc_train(to_dev(bs), xd, len(bs), epochs=30, batch=4, lr=3e-3, seed=2, loss_kind=0)
    b = synth.gaussian_cb_spinor(DIMS, 60, 0)
    x = to_dev(np.zeros_like(b))
    rc, info = ctx.solve(x, to_dev(b), 1, kind=tmx.TMX_SOLVER_FGCR_NN, op=1, tol=1e-10, restart=8)
    print("FGCR:", info[0])
    assert rc == tmx.TMX_OK, info
    assert info[0]["fallback"] == 0, info
    assert o.residual(b, to_host(x, b.shape)) <= 1e-10


def test_fgcr_fallback_with_garbage_network(S):
    """A useless network still yields a 1e-10 solution, through the CG fallback."""
    tmx, ctx, lat, U = S
    o = Oracle(DIMS, U, KAPPA, CSW, mu=MU0)
    rng = np.random.default_rng(9)
    ctx.pc_set_weights((rng.standard_normal(nn.num_params()) * 3.0).astype(np.float32))
    b = synth.gaussian_cb_spinor(DIMS, 61, 0)
    x = to_dev(np.zeros_like(b))
    rc, info = ctx.solve(x, to_dev(b), 1, kind=tmx.TMX_SOLVER_FGCR_NN, op=1, tol=1e-10, restart=8, maxiter=400)
    assert rc == tmx.TMX_OK
    assert info[0]["fallback"] == 1
    assert o.residual(b, to_host(x, b.shape)) <= 1e-10


def test_weights_validation(S):
    tmx, ctx, lat, _ = S
    with pytest.raises(tmx.TmxError):
        ctx.pc_set_weights(np.zeros(10, dtype=np.float32))
    bad = nn.identity_init(None).astype(np.float32)
    bad[5] = np.nan
    with pytest.raises(tmx.TmxError):
        ctx.pc_set_weights(bad)


def test_separately_trained_weights_for_minus_mu(S):
    """Weights trained for Mhat(-mu) on (b, Mhat(-mu)^{-1} b) pairs (the
    residual loss with Mhat(-mu)) precondition the Mhat(-mu) solve: fewer
    iterations than the identity network, solution accepted by the oracle."""
    tmx, ctx, lat, U = S
    o = Oracle(DIMS, U, KAPPA, CSW, mu=MU0)
    n = 16
    bs = np.stack([synth.gaussian_cb_spinor(DIMS, 70, k) for k in range(n)])
    xd = to_dev(np.zeros_like(bs))
    for k in range(n):
        xk = to_dev(np.zeros_like(bs[k]))
        rc, info = ctx.solve_mhat(xk, to_dev(bs[k]), dagger=0, op=-1, tol=1e-10)
        assert rc == tmx.TMX_OK
        xd[k * bs[k].size:(k + 1) * bs[k].size] = xk
    b = synth.gaussian_cb_spinor(DIMS, 71, 0)
    ctx.pc_set_weights(nn.identity_init(None))
    x = to_dev(np.zeros_like(b))
    rc0, info0 = ctx.solve(x, to_dev(b), 1, kind=tmx.TMX_SOLVER_PCG_NN, op=-1, tol=1e-10)
    ctx.pc_set_weights(nn.identity_init(np.random.default_rng(3), 1e-2))
    losses = ctx.pc_train(to_dev(bs), xd, n, epochs=30, batch=4, lr=3e-3, seed=2, loss_kind=0, op=-1)
    assert losses[-1] < 0.7 * losses[0], losses
    x = to_dev(np.zeros_like(b))
    rc1, info1 = ctx.solve(x, to_dev(b), 1, kind=tmx.TMX_SOLVER_PCG_NN, op=-1, tol=1e-10)
    print("PCG(-mu) iterations identity / trained for -mu:", info0[0]["iters"], info1[0]["iters"])
    assert rc0 == tmx.TMX_OK and rc1 == tmx.TMX_OK
    assert info1[0]["iters"] < info0[0]["iters"], (info0, info1)
    assert o.residual(b, to_host(x, b.shape), sgn=-1) <= 1e-10
    with pytest.raises(tmx.TmxError):
        ctx.pc_train(to_dev(bs), xd, n, epochs=1, op=2)


def test_multishift_refinement_with_learned_pc(S, pairs):
    """The multishift solve with the learned network preconditioning each
    shift's FP64 refinement: every shift accepted by the oracle's residual of
    (N + sigma), the network path taken (preconditioner applications counted),
    and the solutions those of the plain refinement."""
    tmx, ctx, lat, U = S
    bs, xd = pairs
    o = Oracle(DIMS, U, KAPPA, CSW, mu=MU0)
    ctx.pc_set_weights(nn.identity_init(np.random.default_rng(3), 1e-2))
    ctx.pc_train(to_dev(bs), xd, len(bs), epochs=12, batch=4, lr=3e-3, seed=1, loss_kind=1)
    b = synth.gaussian_cb_spinor(DIMS, 72, 0)
    shifts = [0.0, 1e-3, 1e-2, 1e-1]
    n = b.size
    for inner in (tmx.TMX_F32, tmx.TMX_F16):
        x = to_dev(np.zeros(len(shifts) * n, dtype=np.complex128))
        # the library's own FP64 residual and the oracle's differ in rounding:
        # ask for 0.9e-10 so that the oracle's check can hold at 1e-10
        rc, info = ctx.multishift_solve(x, to_dev(b), shifts, kind=tmx.TMX_SOLVER_PCG_NN, op=1, tol=0.9e-10,
                                        inner_prec=inner)
        assert rc == tmx.TMX_OK
        xp = to_dev(np.zeros(len(shifts) * n, dtype=np.complex128))
        rcp, _ = ctx.multishift_solve(xp, to_dev(b), shifts, op=1, tol=1e-10, inner_prec=inner)
        assert rcp == tmx.TMX_OK
        for k, s in enumerate(shifts):
            xk = to_host(x[k * n:(k + 1) * n], b.shape)
            res = rel_l2(o.mdagm(xk) + s * xk, b)
            print(f"inner {inner} shift {s:g}: {info[k]['iters']} iterations, "
                  f"{info[k]['restarts']} network applications, oracle residual {res:.2e}")
            assert res <= 1e-10
            assert info[k]["restarts"] >= 1
            assert rel_l2(xk, to_host(xp[k * n:(k + 1) * n], b.shape)) < 1e-8
    with pytest.raises(tmx.TmxError):
        ctx.multishift_solve(to_dev(np.zeros(2 * n, dtype=np.complex128)), to_dev(b), [0.0, 0.1],
                             kind=tmx.TMX_SOLVER_PCG_NN, op=tmx.TMX_OP_WPLUS)


def test_adam_step_matches_oracle(S):
    """Four Adam steps of the library (FP32, on caller-given gradients) against
    the oracle's FP64 Adam from the same FP32 weights, gradients and
    hyper-parameters; setting the weights restarts the step count."""
    tmx, ctx, lat, _ = S
    rng = np.random.default_rng(47)
    n = nn.num_params()
    w0 = nn.identity_init(rng, 0.1).astype(np.float32)
    grads = [(rng.standard_normal(n) * 10.0 ** rng.uniform(-4, 1, n)).astype(np.float32) for _ in range(4)]
    hp = {"lr": 2e-3, "beta1": 0.85, "beta2": 0.995, "eps": 1e-7}
    hp64 = {k: float(np.float32(v)) for k, v in hp.items()}  # what the FP32 configuration holds
    ctx.pc_set_weights(w0)
    for g in grads:
        ctx.pc_adam_step(g, **hp)
    got = ctx.pc_get_weights().astype(np.float64)
    w, m, v = w0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        w, m, v = nn.adam_step(w, m, v, t, g.astype(np.float64), **hp64)
    err = np.abs(got - w).max()
    print(f"Adam: max |w_gpu - w_oracle| = {err:.2e} after 4 steps of size ~{hp['lr']}")
    assert err <= 2e-6
    ctx.pc_set_weights(w0)
    ctx.pc_adam_step(grads[1], **hp)
    w1, _, _ = nn.adam_step(w0.astype(np.float64), np.zeros(n), np.zeros(n), 1, grads[1].astype(np.float64), **hp64)
    assert np.abs(ctx.pc_get_weights() - w1).max() <= 1e-6
    with pytest.raises(tmx.TmxError):
        ctx.pc_adam_step(grads[0][:10], **hp)
    bad = grads[0].copy()
    bad[3] = np.inf
    with pytest.raises(tmx.TmxError):
        ctx.pc_adam_step(bad, **hp)


@pytest.mark.parametrize("mode,depth", [(2, 2), (3, 1)])
def test_hermitian_form_matches_oracle(S, mode, depth):
    """P = L_1^dagger L_2^dagger L_2 L_1 (tmx_pc_apply mode 2) and the short
    form P_1 = L_1^dagger L_1 (mode 3) against the network oracle, random
    weights; Hermitian to the BF16 staging error."""
    tmx, ctx, lat, _ = S
    rng = np.random.default_rng(45)
    w = (rng.standard_normal(nn.num_params()) * 0.3).astype(np.float32)
    ctx.pc_set_weights(w)
    u = synth.gaussian_cb_spinor(DIMS, 45, 0)
    v = synth.gaussian_cb_spinor(DIMS, 45, 1)
    Pu, Pv = to_dev(np.zeros_like(u)), to_dev(np.zeros_like(v))
    ctx.pc_apply(Pu, to_dev(u), mode)
    ctx.pc_apply(Pv, to_dev(v), mode)
    ref = nn.sym_forward(lat, f32(w), v[:, 0], depth=depth)
    with pytest.raises(tmx.TmxError):
        ctx.pc_apply(Pu, to_dev(u), 4)  # no such mode
    got = to_host(Pv, v.shape)[:, 0]
    assert rel_l2(got, ref) < 2e-2
    a = np.vdot(u.reshape(-1), to_host(Pv, v.shape).reshape(-1))
    b = np.vdot(to_host(Pu, u.shape).reshape(-1), v.reshape(-1))
    assert abs(a - b) <= 2e-2 * abs(a)


@pytest.mark.parametrize("depth", [2, 1])
def test_hermitian_form_gradient_matches_oracle(S, depth):
    """Energy-norm loss of the Hermitian form and its gradient (layers 1 and
    2, or layer 1 for the short form; the others zero) against the oracle's."""
    tmx, ctx, lat, U = S
    rng = np.random.default_rng(46)
    w = nn.identity_init(rng, 0.1).astype(np.float32)
    ctx.pc_set_weights(w)
    bs = np.stack([synth.gaussian_cb_spinor(DIMS, 46, k) for k in range(2)])
    xs = np.stack([synth.gaussian_cb_spinor(DIMS, 47, k) for k in range(2)])
    kind = tmx.TMX_LOSS_SYM if depth == 2 else tmx.TMX_LOSS_SYM1
    loss, g = ctx.pc_loss_grad(to_dev(bs), to_dev(xs), 2, kind, 1)
    o = Oracle(DIMS, U, KAPPA, CSW, mu=MU0)
    mh = lambda v: o.mhat(v.reshape(-1, 1, 4, 3)).reshape(-1, 4, 3)
    mhd = lambda v: o.mhat(v.reshape(-1, 1, 4, 3), dagger=True).reshape(-1, 4, 3)
    L, gref = nn.sym_loss_and_grad(lat, f32(w), [b[:, 0] for b in bs], [x[:, 0] for x in xs], mh, mhd, depth=depth)
    assert abs(loss - L) / L < 2e-2
    n1 = 2 * 9 * (8 + 16)
    nused = n1 if depth == 1 else n1 + 2 * 9 * (64 + 16)
    assert np.all(g[nused:] == 0)
    cos = float(np.dot(g, gref) / np.linalg.norm(g) / np.linalg.norm(gref))
    assert cos > 0.999, cos
    assert rel_l2(g, gref) < 5e-2


@pytest.mark.parametrize("depth", [2, 1])
def test_trained_hermitian_form_preconditions_cg(S, depth):
    """Trained on pairs (b, N^{-1} b) of the field, the Hermitian form (or
    its short form) cuts the iterations of the preconditioned CG (one network
    application per iteration) below the identity network's, without falling
    back; the solution is accepted by the oracle."""
    tmx, ctx, lat, U = S
    kind = tmx.TMX_SOLVER_PCG_NN_SYM if depth == 2 else tmx.TMX_SOLVER_PCG_NN_SYM1
    loss_kind = tmx.TMX_LOSS_SYM if depth == 2 else tmx.TMX_LOSS_SYM1
    o = Oracle(DIMS, U, KAPPA, CSW, mu=MU0)
    n = 16
    bs = np.stack([synth.gaussian_cb_spinor(DIMS, 73, k) for k in range(n)])
    xd = to_dev(np.zeros_like(bs))
    for k in range(n):
        xk = to_dev(np.zeros_like(bs[k]))
        rc, info = ctx.solve(xk, to_dev(bs[k]), 1, kind=tmx.TMX_SOLVER_CG, op=1, tol=1e-10)
        assert rc == tmx.TMX_OK
        xd[k * bs[k].size:(k + 1) * bs[k].size] = xk
    b = synth.gaussian_cb_spinor(DIMS, 74, 0)
    ctx.pc_set_weights(nn.identity_init(None))
    x = to_dev(np.zeros_like(b))
    rc0, info0 = ctx.solve(x, to_dev(b), 1, kind=kind, op=1, tol=1e-10)
    ctx.pc_set_weights(nn.identity_init(np.random.default_rng(3), 1e-2))
    losses = ctx.pc_train(to_dev(bs), xd, n, epochs=30, batch=4, lr=3e-3, seed=2, loss_kind=loss_kind)
    assert losses[-1] < 0.7 * losses[0], losses
    x = to_dev(np.zeros_like(b))
    rc1, info1 = ctx.solve(x, to_dev(b), 1, kind=kind, op=1, tol=0.9e-10, inner_prec=2)
    print(f"PCG (Hermitian form, depth {depth}) iterations identity / trained:", info0[0]["iters"],
          info1[0]["iters"], "network applications", info1[0]["restarts"])
    assert rc0 == tmx.TMX_OK and rc1 == tmx.TMX_OK
    assert info0[0]["fallback"] == 0 and info1[0]["fallback"] == 0
    assert info1[0]["iters"] < info0[0]["iters"]
    assert o.residual(b, to_host(x, b.shape)) <= 1e-10
