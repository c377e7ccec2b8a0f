"""Pins of the learned-preconditioner oracle (network definition: linear,
gauge-equivariant parallel-transport layers with C_d (x) Gamma_d weights)."""
import numpy as np
import pytest

from oracle import nn_oracle as nn
from paper_2212_06635_amd import synth

DIMS = (4, 4, 2, 4)


@pytest.fixture(scope="module")
def lat():
    U = synth.gauge_links(DIMS, 0.4, 17)
    return nn.Lattice(DIMS, U, t_bc=-1), U


def rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(nn.num_params()) * scale


def test_param_count_and_roundtrip():
    assert nn.num_params() == 2 * 9 * (8 + 16 + 64 + 16 + 64 + 16 + 8 + 16)
    w = rand_params(1)
    assert np.array_equal(nn.flatten(nn.unflatten(w)), w)


def test_identity_init_is_identity(lat):
    L, _ = lat
    w = nn.identity_init(None)
    b = synth.gaussian_cb_spinor(DIMS, 3, 0)[:, 0]
    assert np.array_equal(nn.forward(L, w, b), b)


def test_two_hop_path_is_pure_transport(lat):
    """Only +x in layer 3 and +y in layer 4: (K b)(x) = U_y(x) U_x(x+y) b(x+y+x)."""
    L, U = lat
    params = nn.unflatten(nn.identity_init(None))
    C3, G3 = params[2]
    C3[0] = 0
    G3[0] = 0
    C3[1] = np.eye(8)
    G3[1] = np.eye(4)  # d = 1: +x
    C4, G4 = params[3]
    C4[0] = 0
    G4[0] = 0
    C4[3] = np.eye(1, 8)
    G4[3] = np.eye(4)  # d = 3: +y
    w = nn.flatten(params)
    b = synth.gaussian_cb_spinor(DIMS, 3, 1)[:, 0]
    out = nn.forward(L, w, b)
    lx, ly, lz, lt = DIMS
    full = np.zeros((lx * ly * lz * lt, 4, 3), dtype=complex)
    full[synth.odd_sites(DIMS, 1)] = b
    Ul = U.reshape(-1, 4, 3, 3)
    odd = synth.odd_sites(DIMS, 1)
    for k in range(0, len(odd), 7):
        i = odd[k]
        x, y, z, t = i % lx, (i // lx) % ly, (i // (lx * ly)) % lz, i // (lx * ly * lz)
        j = x + lx * ((y + 1) % ly + ly * (z + lz * t))  # x + y-hat
        m = (x + 1) % lx + lx * ((y + 1) % ly + ly * (z + lz * t))  # x + y-hat + x-hat
        expect = (Ul[i, 1] @ Ul[j, 0] @ full[m].T).T
        assert np.allclose(out[k], expect, atol=1e-14)


def test_gauge_covariance(lat):
    L, U = lat
    G = synth.random_gauge_transform(DIMS, 5)
    Lp = nn.Lattice(DIMS, synth.gauge_transform_links(U, G), t_bc=-1)
    w = rand_params(2)
    b = synth.gaussian_cb_spinor(DIMS, 3, 2)[:, 0]
    Go = G.reshape(-1, 3, 3)[synth.odd_sites(DIMS, 1)]
    gb = np.einsum("xab,xsb->xsa", Go, b)
    assert np.allclose(nn.forward(Lp, w, gb), np.einsum("xab,xsb->xsa", Go, nn.forward(L, w, b)), atol=1e-12)


def test_adjoint(lat):
    L, _ = lat
    w = rand_params(3)
    u = synth.gaussian_cb_spinor(DIMS, 3, 3)[:, 0]
    v = synth.gaussian_cb_spinor(DIMS, 3, 4)[:, 0]
    a = np.vdot(u, nn.forward(L, w, v))
    b = np.vdot(nn.adjoint(L, w, u), v)
    assert abs(a - b) / abs(a) < 1e-13


def test_gradient_matches_finite_differences(lat):
    L, _ = lat
    w = rand_params(4, 0.2)
    bs = [synth.gaussian_cb_spinor(DIMS, 3, 10 + i)[:, 0] for i in range(2)]
    xs = [synth.gaussian_cb_spinor(DIMS, 3, 20 + i)[:, 0] for i in range(2)]
    loss, g = nn.loss_and_grad(L, w, bs, xs)
    rng = np.random.default_rng(7)
    idx = rng.choice(w.size, 40, replace=False)
    h = 1e-5
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        lp = nn.loss_and_grad(L, wp, bs, xs)[0]
        lm = nn.loss_and_grad(L, wm, bs, xs)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_residual_loss_gradient_matches_finite_differences(lat):
    """Residual loss |Mhat (K b - x)|^2 / |b|^2 with the FP64 Schur operator of the C oracle."""
    from oracle import Oracle

    L, U = lat
    o = Oracle(DIMS, U, 0.1394, 1.69, mu=0.01)
    mh = lambda v: o.mhat(v.reshape(-1, 1, 4, 3)).reshape(-1, 4, 3)
    mhd = lambda v: o.mhat(v.reshape(-1, 1, 4, 3), dagger=True).reshape(-1, 4, 3)
    w = rand_params(5, 0.2)
    bs = [synth.gaussian_cb_spinor(DIMS, 3, 30 + i)[:, 0] for i in range(2)]
    xs = [synth.gaussian_cb_spinor(DIMS, 3, 40 + i)[:, 0] for i in range(2)]
    loss, g = nn.loss_and_grad(L, w, bs, xs, mh, mhd)
    # the loss itself: |Mhat K b - Mhat x|^2/|b|^2
    direct = sum(np.linalg.norm(mh(nn.forward(L, w, b) - x)) ** 2 / np.linalg.norm(b) ** 2 for b, x in zip(bs, xs)) / 2
    assert abs(loss - direct) / direct < 1e-13
    rng = np.random.default_rng(8)
    h = 1e-5
    for k in rng.choice(w.size, 25, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (nn.loss_and_grad(L, wp, bs, xs, mh, mhd)[0] - nn.loss_and_grad(L, wm, bs, xs, mh, mhd)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9, (k, fd, g[k])


def _adam_run(w0, grads, **kw):
    w, m, v = np.array(w0, dtype=np.float64), np.zeros(len(w0)), np.zeros(len(w0))
    out = []
    for t, g in enumerate(grads, start=1):
        w, m, v = nn.adam_step(w, m, v, t, g, **kw)
        out.append(w.copy())
    return out


def test_adam_hand_computed_two_steps():
    """Worked by hand from the moment recurrences (beta1 = 0.9,
    beta2 = 0.999, lr = 0.1, eps = 0, w0 = 0.5, g = 1 then -2):
    m1 = 0.1, v1 = 0.001, bias-corrected 1 and 1, step 0.1;
    m2 = -0.11, v2 = 0.004999, bias-corrected -0.11/0.19 and
    0.004999/0.001999, step -0.0366103527035845565..."""
    w1, w2 = _adam_run([0.5], [[1.0], [-2.0]], lr=0.1, beta1=0.9, beta2=0.999, eps=0.0)
    assert abs(w1[0] - 0.4) < 1e-15
    assert abs(w2[0] - 0.43661035270358455653) < 1e-15


def test_adam_first_step_and_constant_gradient():
    """Bias correction makes the estimates exact for a constant gradient:
    every step (the first one included) moves w by lr g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 2, 50)
    w0 = rng.standard_normal(50)
    lr, eps = 3e-3, 1e-8
    ws = _adam_run(w0, [g] * 6, lr=lr, eps=eps)
    step = lr * g / (np.abs(g) + eps)
    for t, w in enumerate(ws, start=1):
        assert np.allclose(w, w0 - t * step, rtol=0, atol=1e-13)


def test_adam_scale_invariance():
    """With eps = 0 the update depends on the gradients only through their
    ratio to their running scale: multiplying every gradient by c > 0 leaves
    the trajectory unchanged, c < 0 mirrors it."""
    rng = np.random.default_rng(6)
    w0 = rng.standard_normal(20)
    grads = [rng.standard_normal(20) for _ in range(5)]
    ref = _adam_run(w0, grads, lr=1e-2, eps=0.0)
    for c in (1e-4, 37.0):
        got = _adam_run(w0, [c * g for g in grads], lr=1e-2, eps=0.0)
        assert all(np.allclose(a, b, rtol=0, atol=1e-13) for a, b in zip(got, ref))
    neg = _adam_run(w0, [-g for g in grads], lr=1e-2, eps=0.0)
    assert all(np.allclose(a - w0, -(b - w0), rtol=0, atol=1e-13) for a, b in zip(neg, ref))


@pytest.mark.parametrize("depth", [2, 1])
def test_hermitian_form_is_hermitian_and_positive(lat, depth):
    """P = A^dagger A (A = L_2 L_1, or L_1 for the short form): <u, P v> =
    <P u, v>, <v, P v> = |A v|^2 >= 0 with A applied directly, and the
    identity initialisation gives P = 1 (the layers the identity path)."""
    L, _ = lat
    w = rand_params(8, 0.3)
    u = synth.gaussian_cb_spinor(DIMS, 5, 0)[:, 0]
    v = synth.gaussian_cb_spinor(DIMS, 5, 1)[:, 0]
    Pu, Pv = nn.sym_forward(L, w, u, depth=depth), nn.sym_forward(L, w, v, depth=depth)
    assert abs(np.vdot(u, Pv) - np.vdot(Pu, v)) < 1e-12 * abs(np.vdot(u, Pv))
    (C1, G1), (C2, G2) = nn.unflatten(w)[:2]
    Av = nn.layer_forward(L, C1, G1, L.embed_odd(v))
    if depth == 2:
        Av = nn.layer_forward(L, C2, G2, Av)
    # only the odd sites of P v are kept, so <v, P v> = |A E_odd v|^2 exactly
    assert abs(np.vdot(v, Pv).real - np.vdot(Av, Av).real) < 1e-12 * np.vdot(Av, Av).real
    assert abs(np.vdot(v, Pv).imag) < 1e-12 * abs(np.vdot(v, Pv))
    assert np.allclose(nn.sym_forward(L, nn.identity_init(None), v, depth=depth), v, rtol=0, atol=1e-15)


def test_short_form_through_path_channels(lat):
    """The library applies P_1 = L_1^dagger L_1 without the 8-channel
    intermediate: with h_d = Gamma_d T_d b and M[d'][d] = sum_c
    conj(C_{rev d'}[c]) C_d[c] (the adjoint's channel contraction met by the
    first layer's channel spread), P_1 b = sum_d' Gamma_{rev d'}^H T_d'
    z_d', z_d' = sum_d M[d'][d] h_d.  That rewriting against the layer-by-layer
    form."""
    L, _ = lat
    w = rand_params(12, 0.3)
    b = synth.gaussian_cb_spinor(DIMS, 12, 0)[:, 0]
    C, G = nn.unflatten(w)[0]
    x = L.embed_odd(b)
    h = [np.einsum("st,ovtc->ovsc", G[d], L.transport(x, d)) for d in range(nn.NPATH)]
    M = np.array([[np.sum(np.conj(C[nn.reverse_path(dp)][:, 0]) * C[d][:, 0]) for d in range(nn.NPATH)]
                  for dp in range(nn.NPATH)])
    out = np.zeros_like(x)
    for dp in range(nn.NPATH):
        z = sum(M[dp, d] * h[d] for d in range(nn.NPATH))
        Gp = np.conj(G[nn.reverse_path(dp)]).T
        out += L.transport(np.einsum("st,ovtc->ovsc", Gp, z), dp)
    ref = nn.sym_forward(L, w, b, depth=1)
    assert np.allclose(L.restrict_odd(out), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("depth", [2, 1])
def test_hermitian_form_gradient_matches_finite_differences(lat, depth):
    """Energy-norm loss of P = A^dagger A with the C oracle's Schur operator:
    the gradient (each layer used forward and as an adjoint) against central
    differences; the layers past A do not enter."""
    from oracle import Oracle

    L, U = lat
    o = Oracle(DIMS, U, 0.1394, 1.69, mu=0.01)
    mh = lambda v: o.mhat(v.reshape(-1, 1, 4, 3)).reshape(-1, 4, 3)
    mhd = lambda v: o.mhat(v.reshape(-1, 1, 4, 3), dagger=True).reshape(-1, 4, 3)
    w = rand_params(9, 0.2)
    bs = [synth.gaussian_cb_spinor(DIMS, 3, 50 + i)[:, 0] for i in range(2)]
    xs = [synth.gaussian_cb_spinor(DIMS, 3, 60 + i)[:, 0] for i in range(2)]
    loss, g = nn.sym_loss_and_grad(L, w, bs, xs, mh, mhd, depth=depth)
    n1 = 2 * 9 * (8 + 16)
    nused = n1 if depth == 1 else n1 + 2 * 9 * (64 + 16)
    assert np.all(g[nused:] == 0)
    assert np.any(g[:n1] != 0)
    rng = np.random.default_rng(11)
    idx = rng.choice(n1, 12, replace=False)
    if depth == 2:
        idx = np.concatenate([idx, n1 + rng.choice(2 * 9 * 80, 16, replace=False)])
    h = 1e-5
    for k in idx:
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (nn.sym_loss_and_grad(L, wp, bs, xs, mh, mhd, depth=depth)[0]
              - nn.sym_loss_and_grad(L, wm, bs, xs, mh, mhd, depth=depth)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9, (k, fd, g[k])
