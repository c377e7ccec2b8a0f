"""Fermion-force building blocks on the GPU against the oracle: the link
derivative of Re<Y, Mhat X> through the hopping terms and through the clover
term, as traceless anti-Hermitian 3x3 matrices in the canonical link layout;
the oracle's forms are pinned by finite differences."""
import numpy as np
import pytest

from helpers import CSW, EPSBAR, KAPPA, MUBAR, rel_l2, to_dev, to_host
from oracle import Oracle
from paper_2212_06635_amd import synth

pytestmark = pytest.mark.gpu

CASES = [((4, 4, 2, 6), 0.3, 11), ((6, 4, 2, 10), 0.3, 3), ((8, 8, 8, 8), 0.3, 1)]
MU0 = 0.05


@pytest.fixture(scope="module", params=CASES, ids=lambda c: "x".join(map(str, c[0])))
def S(request):
    import paper_2212_06635_amd.tmx as tmx

    dims, eps, seed = request.param
    print(f"\n[gpu force] lattice {dims} eps={eps} seed={seed}", flush=True)
    U = synth.gauge_links(dims, eps, seed)
    o = Oracle(dims, U, KAPPA, CSW, mu=MU0, mubar=MUBAR, epsbar=EPSBAR)
    ctx = tmx.Context(dims)
    ctx.set_params(tmx.Params(KAPPA, CSW, MU0, MUBAR, EPSBAR, -1))
    ctx.load_gauge(U, float(seed))
    yield tmx, o, ctx, dims
    ctx.close()


@pytest.mark.parametrize("sgn", [1, -1])
def test_hop_force(S, sgn):
    import torch

    tmx, o, ctx, dims = S
    X = synth.gaussian_cb_spinor(dims, 41, 0)
    Y = synth.gaussian_cb_spinor(dims, 41, 1)
    ref = o.hop_force(X, Y, sgn)
    F = torch.zeros(ref.size, dtype=torch.complex128, device="cuda")
    ctx.hop_force(F, to_dev(X), to_dev(Y), op=sgn)
    got = to_host(F, ref.shape)
    assert rel_l2(got, ref) < 1e-13


def test_hop_force_accumulates(S):
    import torch

    tmx, o, ctx, dims = S
    X1, Y1 = synth.gaussian_cb_spinor(dims, 42, 0), synth.gaussian_cb_spinor(dims, 42, 1)
    X2, Y2 = synth.gaussian_cb_spinor(dims, 42, 2), synth.gaussian_cb_spinor(dims, 42, 3)
    ref = 0.5 * o.hop_force(X1, Y1, 1) + 2.0 * o.hop_force(X2, Y2, 1)
    F = torch.full((ref.size,), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    ctx.hop_force(F, to_dev(X1), to_dev(Y1), op=1, coeff=0.5)  # overwrites (NaN never read)
    ctx.hop_force(F, to_dev(X2), to_dev(Y2), op=1, coeff=2.0, accumulate=1)
    assert rel_l2(to_host(F, ref.shape), ref) < 1e-13


def test_hop_force_rejects_other_operators(S):
    import torch

    tmx, o, ctx, dims = S
    X = to_dev(synth.gaussian_cb_spinor(dims, 43, 0))
    F = torch.zeros(int(np.prod(dims)) * 36, dtype=torch.complex128, device="cuda")
    with pytest.raises(tmx.TmxError):
        ctx.hop_force(F, X, X, op=tmx.TMX_OP_WPLUS)
    with pytest.raises(ValueError):
        ctx.hop_force(F[:10], X, X, op=1)  # too small an output: refused before any launch
    with pytest.raises(ValueError):
        ctx.hop_force(F, X, X, op=tmx.TMX_OP_ND)  # one-flavour fields for the two-flavour operator


@pytest.mark.parametrize("sgn", [1, -1])
def test_clover_force(S, sgn):
    """The clover-term part of the link derivative (both parities' site blocks)."""
    import torch

    tmx, o, ctx, dims = S
    X = synth.gaussian_cb_spinor(dims, 44, 0)
    Y = synth.gaussian_cb_spinor(dims, 44, 1)
    ref = o.clover_force(X, Y, sgn)
    F = torch.zeros(ref.size, dtype=torch.complex128, device="cuda")
    ctx.clover_force(F, to_dev(X), to_dev(Y), op=sgn)
    assert rel_l2(to_host(F, ref.shape), ref) < 1e-13


def test_full_force_accumulated(S):
    """hop_force then clover_force accumulating: the whole derivative of
    Re<Y, Mhat X>, the sum that the oracle's finite-difference pin checks."""
    import torch

    tmx, o, ctx, dims = S
    X = synth.gaussian_cb_spinor(dims, 45, 0)
    Y = synth.gaussian_cb_spinor(dims, 45, 1)
    ref = 0.75 * (o.hop_force(X, Y, 1) + o.clover_force(X, Y, 1))
    F = torch.full((ref.size,), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    ctx.hop_force(F, to_dev(X), to_dev(Y), op=1, coeff=0.75)
    ctx.clover_force(F, to_dev(X), to_dev(Y), op=1, coeff=0.75, accumulate=1)
    assert rel_l2(to_host(F, ref.shape), ref) < 1e-13


def test_clover_force_rejects_other_operators(S):
    import torch

    tmx, o, ctx, dims = S
    X = to_dev(synth.gaussian_cb_spinor(dims, 46, 0))
    F = torch.zeros(int(np.prod(dims)) * 36, dtype=torch.complex128, device="cuda")
    with pytest.raises(tmx.TmxError):
        ctx.clover_force(F, X, X, op=tmx.TMX_OP_WPLUS)
    with pytest.raises(ValueError):
        ctx.clover_force(F, X[:10], X, op=1)
    # a clover term loaded from the host has no links to differentiate
    ctx.load_clover(ctx.get_clover())
    try:
        with pytest.raises(tmx.TmxError):
            ctx.clover_force(F, X, X, op=1)
    finally:
        ctx.load_clover(None)  # back to the term built from the links
    ctx.clover_force(F, X, X, op=1)


def test_two_flavour_force(S):
    """The two-flavour operator (eq. Q-hat_h): hopping and clover forces of
    Re<Y, Mhat_h X> against the oracle's flavour-summed forms, written and
    accumulated."""
    import torch

    tmx, o, ctx, dims = S
    X = synth.gaussian_cb_spinor(dims, 47, 0, 2)
    Y = synth.gaussian_cb_spinor(dims, 47, 1, 2)
    rh, rc = o.hop_force(X, Y, 1, nf=2), o.clover_force(X, Y, 1, nf=2)
    F = torch.full((rh.size,), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    ctx.hop_force(F, to_dev(X), to_dev(Y), op=tmx.TMX_OP_ND)
    assert rel_l2(to_host(F, rh.shape), rh) < 1e-13
    ctx.clover_force(F, to_dev(X), to_dev(Y), op=tmx.TMX_OP_ND)
    assert rel_l2(to_host(F, rc.shape), rc) < 1e-13
    ctx.hop_force(F, to_dev(X), to_dev(Y), op=tmx.TMX_OP_ND, coeff=-1.5, accumulate=1)
    assert rel_l2(to_host(F, rc.shape), rc - 1.5 * rh) < 1e-13


@pytest.mark.parametrize("op", [2, 1])
def test_rational_force(S, op):
    """The rational monomial's force on the device -- multishift solves, then
    -2 a_k (hop + clover force)(x_k, Mhat x_k) added shift by shift -- against
    the oracle's (its own CG solves, forces pinned by finite differences).
    Two-flavour: the 12 poles of Zolotarev's approximation of N_h^(-1/2) on
    [1e-5, 1] x 2.2 (above the largest eigenvalue of N_h here), the heavy
    sector's rational monomial; degenerate: four shifts.  The solves differ
    by their 1e-11 tolerances, so the forces agree to ~cond(N) 1e-11."""
    import torch

    from paper_2212_06635_amd import zolotarev

    tmx, o, ctx, dims = S
    nf = 2 if op == 2 else 1
    phi = synth.gaussian_cb_spinor(dims, 48, 0, nf)
    if op == 2:
        z = zolotarev.for_spectrum(12, 2.2e-5, 2.2)
        coeffs, shifts = list(z.a), list(z.shifts)
    else:
        coeffs, shifts = [0.02, 0.1, 0.3, 0.5], [1e-3, 1e-2, 0.1, 1.0]
    ref = o.rational_force(phi, coeffs, shifts, nf=nf, sgn=1)
    F = torch.zeros(ref.size, dtype=torch.complex128, device="cuda")
    rc, info = ctx.rational_force(F, to_dev(phi), coeffs, shifts, op=op, tol=1e-11, inner_prec=1)
    assert rc == tmx.TMX_OK, info
    err = rel_l2(to_host(F, ref.shape), ref)
    print(f"[gpu force] rational force nf={nf}: rel L2 {err:.2e}", flush=True)
    assert err < 1e-8
    # accumulating onto a prior force adds
    G = F.clone()
    ctx.rational_force(G, to_dev(phi), coeffs, shifts, accumulate=1, op=op, tol=1e-11, inner_prec=1)
    assert rel_l2(to_host(G, ref.shape), 2 * ref) < 1e-8
