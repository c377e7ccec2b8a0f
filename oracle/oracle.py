"""Plain FP64 CPU oracle (test infrastructure only: the tests, the smoke
check and the benchmark's CPU baseline use it; the GPU library never does).

The operator arithmetic -- hopping term, clover term, site blocks, D, the
Schur operator and its normal form, CG -- lives in ``tmx_oracle.c`` (plain
loops, FP64, OpenMP over sites), called here through ctypes; the learned
preconditioner is in ``nn_oracle.py``.  The forms built on top of the
operator are written here in numpy, each in the order its definition states:
the mass-preconditioned operators (Section 2), the rational function and its
correction series (Section 4.2), and the link derivatives of Re<Y, Mhat X>
through the hopping and the clover terms (Section 4.3).  Every function is
pinned by tests that do not reuse it (closed forms, brute force, finite
differences, spectral forms); none is parity unpinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tmx_oracle.c")
_LIB = os.path.join(_HERE, "libtmx_oracle.so")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_oracle(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    L = ctypes.c_long
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = I
    lib.orc_gammas.argtypes = [P, P]
    lib.orc_hop.argtypes = [P, I, P, P, P, I, I]
    lib.orc_clover.argtypes = [P, P, D, D, P]
    lib.orc_site_block.argtypes = [P, L, D, D, D, D, I, P]
    lib.orc_apply_D.argtypes = [P, I, P, P, D, D, D, D, I, P, P]
    lib.orc_mhat.argtypes = [P, I, P, P, D, D, D, D, I, I, P, P]
    lib.orc_mhat.restype = I
    lib.orc_mhat_dag.argtypes = [P, I, P, P, D, D, D, D, I, I, P, P]
    lib.orc_mhat_dag.restype = I
    lib.orc_mdagm.argtypes = [P, I, P, P, D, D, D, D, I, I, D, P, P]
    lib.orc_mdagm.restype = I
    lib.orc_cg.argtypes = [P, I, P, P, D, D, D, D, I, I, D, P, P, D, I, ctypes.POINTER(D)]
    lib.orc_cg.restype = I
    lib.orc_residual.argtypes = [P, I, P, P, D, D, D, D, I, I, D, P, P]
    lib.orc_residual.restype = D
    lib.orc_residual_mhat.argtypes = [P, I, P, P, D, D, D, D, I, I, I, P, P]
    lib.orc_residual_mhat.restype = D
    _lib = lib
    return lib


def num_threads() -> int:
    return int(load_library().orc_num_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


class Oracle:
    """FP64 oracle of one gauge field and parameter set.

    dims = (Lx, Ly, Lz, Lt); U in the layout of ``synth.gauge_links``.
    Parameters are the bare ones (kappa, csw, mu, mubar, epsbar); the hopping
    normalisation factors 2*kappa are applied inside the oracle.
    """

    def __init__(self, dims, U, kappa, csw, mu=0.0, mubar=0.0, epsbar=0.0, t_bc=-1, T=None):
        self.lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.L = np.asarray(self.dims, dtype=np.int32)
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        self.U = _c(U).reshape(self.V, 4, 3, 3)
        self.kappa, self.csw = float(kappa), float(csw)
        self.mu, self.mubar, self.epsbar = float(mu), float(mubar), float(epsbar)
        self.t_bc = int(t_bc)
        if T is None:
            T = np.empty((self.V, 12, 12), dtype=np.complex128)
            self.lib.orc_clover(_ptr(self.L), _ptr(self.U), self.kappa, self.csw, _ptr(T))
        self.T = _c(T).reshape(self.V, 12, 12)

    # -- pieces --------------------------------------------------------
    @staticmethod
    def gammas():
        lib = load_library()
        g = np.empty((5, 4, 4), dtype=np.complex128)
        s = np.empty((4, 4, 4, 4), dtype=np.complex128)
        lib.orc_gammas(_ptr(g), _ptr(s))
        return g, s

    def hop(self, psi, out_parity=-1):
        psi = _c(psi)
        nf = psi.size // (12 * self.V)
        out = np.empty_like(psi)
        self.lib.orc_hop(_ptr(self.L), self.t_bc, _ptr(self.U), _ptr(psi), _ptr(out), nf, out_parity)
        return out

    def site_block(self, lex, nf=1, sgn=1):
        n = 12 * nf
        B = np.empty((n, n), dtype=np.complex128)
        self.lib.orc_site_block(_ptr(self.T), int(lex), self.kappa, sgn * self.mu, sgn * self.mubar,
                                self.epsbar, nf, _ptr(B))
        return B

    # -- operators -----------------------------------------------------
    def D(self, psi, nf=1, sgn=1):
        psi = _c(psi)
        out = np.empty_like(psi)
        self.lib.orc_apply_D(_ptr(self.L), self.t_bc, _ptr(self.U), _ptr(self.T), self.kappa, sgn * self.mu,
                             sgn * self.mubar, self.epsbar, nf, _ptr(psi), _ptr(out))
        return out

    def mhat(self, v, nf=1, sgn=1, dagger=False):
        v = _c(v)
        out = np.empty_like(v)
        fn = self.lib.orc_mhat_dag if dagger else self.lib.orc_mhat
        bad = fn(_ptr(self.L), self.t_bc, _ptr(self.U), _ptr(self.T), self.kappa, self.mu, self.mubar,
                 self.epsbar, nf, sgn, _ptr(v), _ptr(out))
        if bad:
            raise FloatingPointError("singular site block")
        return out

    def mdagm(self, v, nf=1, sgn=1, shift=0.0):
        v = _c(v)
        out = np.empty_like(v)
        bad = self.lib.orc_mdagm(_ptr(self.L), self.t_bc, _ptr(self.U), _ptr(self.T), self.kappa, self.mu,
                                 self.mubar, self.epsbar, nf, sgn, float(shift), _ptr(v), _ptr(out))
        if bad:
            raise FloatingPointError("singular site block")
        return out

    def cg(self, b, nf=1, sgn=1, shift=0.0, tol=1e-10, maxiter=10000):
        b = _c(b)
        x = np.empty_like(b)
        rel = ctypes.c_double(0)
        it = self.lib.orc_cg(_ptr(self.L), self.t_bc, _ptr(self.U), _ptr(self.T), self.kappa, self.mu,
                             self.mubar, self.epsbar, nf, sgn, float(shift), _ptr(b), _ptr(x), float(tol),
                             int(maxiter), ctypes.byref(rel))
        return x, it, rel.value

    def residual(self, b, x, nf=1, sgn=1, shift=0.0):
        b, x = _c(b), _c(x)
        return self.lib.orc_residual(_ptr(self.L), self.t_bc, _ptr(self.U), _ptr(self.T), self.kappa, self.mu,
                                     self.mubar, self.epsbar, nf, sgn, float(shift), _ptr(b), _ptr(x))

    # -- mass preconditioning (Section 2, eq. for W^pm(rho)) ----------------
    # Q^pm = g5 D(pm mu) (full lattice) and Qhat^pm = g5 Mhat(pm mu) (odd
    # sites); W^pm(rho) = Q^pm pm i rho with rho in the normalisation of the
    # operator, rho~ = 2 kappa rho (as nu = 2 kappa mu).  One helper adds the
    # i rho term to both, so the paper's identity on the full operator pins
    # the convention used for the Schur one.
    @staticmethod
    def g5(v):
        """gamma5 = diag(1, 1, -1, -1) on the spin index (components 6..11 of a site)."""
        w = np.array(v, dtype=np.complex128, copy=True)
        w.reshape(-1, 12)[:, 6:] *= -1
        return w

    def _w(self, qv, v, sgn, rho, dagger):
        # (Q + i s rho~) v, or its adjoint (Q^dagger - i s rho~) v given qv = Q^dagger v
        rt = 2.0 * self.kappa * rho
        return qv + (-1j if dagger else 1j) * sgn * rt * _c(v)

    def q_full(self, psi, sgn=1):
        return self.g5(self.D(psi, 1, sgn))

    def w_full(self, psi, sgn=1, rho=0.0):
        return self._w(self.q_full(psi, sgn), psi, sgn, rho, False)

    def q_hat(self, v, sgn=1, dagger=False):
        # Qhat = g5 Mhat ; Qhat^dagger = Mhat^dagger g5
        if dagger:
            return self.mhat(self.g5(v), 1, sgn, dagger=True)
        return self.g5(self.mhat(v, 1, sgn))

    def w_hat(self, v, sgn=1, rho=0.0, dagger=False):
        return self._w(self.q_hat(v, sgn, dagger), v, sgn, rho, dagger)

    def w_normal(self, v, sgn=1, rho=0.0):
        """W^dagger W v for W = What^sgn(rho) (Hermitian positive definite)."""
        return self.w_hat(self.w_hat(v, sgn, rho), sgn, rho, dagger=True)

    def residual_w(self, b, x, sgn=1, rho=0.0):
        """|b - W^dagger W x| / |b| for W = What^sgn(rho)."""
        b = _c(b)
        return float(np.linalg.norm(b - self.w_normal(x, sgn, rho)) / np.linalg.norm(b))

    # -- hopping-term force ---------------------------------------------------
    def hop_force(self, X, Y, sgn=1, nf=1):
        """Link derivative of S = Re<Y, Mhat(sgn) X> through the hopping terms
        (clover and twist blocks held fixed), for U_mu(x) -> exp(i eps T) U_mu(x):
        dS/d eps = Re Tr[i T F_mu(x)], F = TA(Q) the traceless anti-Hermitian
        part of Q_mu(x) = -kappa^2 bc U_mu(x) [sum_s ((1 - g_mu) b(x+mu))_s a(x)_s^dagger
        + sum_s ((1 + g_mu) a(x+mu))_s b(x)_s^dagger], with full-lattice fields
        b = X (odd) | u = B_ee(sgn)^-1 H_eo X (even) and
        a = Y (odd) | w = B_ee(-sgn)^-1 g5 H_eo g5 Y (even).  Shape (V, 4, 3, 3).
        Two flavours (nf = 2, the operator of eq. Q-hat_h): the hopping term
        is flavour diagonal and the site blocks B_ee(+-) mix the flavours, so
        a and b are two-flavour fields and the outer products are summed over
        the flavour index."""
        g, _ = self.gammas()
        a, b, co, _ = self._force_fields(X, Y, sgn, nf)
        V = self.V
        lx, ly, lz, lt = self.dims
        F = np.zeros((V, 4, 3, 3), dtype=np.complex128)
        eye4 = np.eye(4)
        L = (lx, ly, lz, lt)
        for mu in range(4):
            c2 = co.copy()
            c2[:, mu] = (c2[:, mu] + 1) % L[mu]
            y = c2[:, 0] + lx * (c2[:, 1] + ly * (c2[:, 2] + lz * c2[:, 3]))
            bc = np.where((mu == 3) & (co[:, 3] == lt - 1), float(self.t_bc), 1.0)
            pb = np.einsum("st,xftc->xfsc", eye4 - g[mu], b[y])
            pa = np.einsum("st,xftc->xfsc", eye4 + g[mu], a[y])
            M = np.einsum("xfsc,xfsd->xcd", pb, a.conj()) + np.einsum("xfsc,xfsd->xcd", pa, b.conj())
            Q = -(self.kappa ** 2) * bc[:, None, None] * np.einsum("xij,xjk->xik", self.U[:, mu], M)
            A = 0.5 * (Q - np.conj(np.swapaxes(Q, 1, 2)))
            F[:, mu] = A - (np.trace(A, axis1=1, axis2=2) / 3.0)[:, None, None] * np.eye(3)
        return F

    def _force_fields(self, X, Y, sgn, nf=1):
        """Full-lattice a (Y | B_ee(-sgn)^-1 g5 H_eo g5 Y) and b (X | B_ee(sgn)^-1 H_eo X),
        shape (V, nf, 4, 3), the lexicographic coordinates and the parity of every site."""
        g, _ = self.gammas()
        lx, ly, lz, lt = self.dims
        V = self.V
        lex = np.arange(V)
        co = np.stack([lex % lx, (lex // lx) % ly, (lex // (lx * ly)) % lz, lex // (lx * ly * lz)], axis=1)
        par = co.sum(axis=1) % 2
        odd, even = np.nonzero(par == 1)[0], np.nonzero(par == 0)[0]
        g5 = lambda f: np.einsum("st,xftc->xfsc", g[4], f)
        hop_even = lambda f: self.hop(f, out_parity=0)

        def full(v_odd):
            f = np.zeros((V, nf, 4, 3), dtype=np.complex128)
            f[odd] = _c(v_odd).reshape(-1, nf, 4, 3)
            return f

        def block_solve(f, s):
            out = np.zeros_like(f)
            for x in even:
                out[x] = np.linalg.solve(self.site_block(int(x), nf, s), f[x].reshape(12 * nf)).reshape(nf, 4, 3)
            return out

        b, a = full(X), full(Y)
        b[even] = block_solve(hop_even(b), sgn)[even]
        a[even] = block_solve(g5(hop_even(g5(a))), -sgn)[even]
        return a, b, co, par

    def clover_force(self, X, Y, sgn=1, nf=1):
        """Link derivative of S = Re<Y, Mhat(sgn) X> through the clover term
        T = i kappa csw sum_{mu<nu} sigma_mu,nu F_mu,nu (F = (Q - Q^dagger)/8, Q the
        four leaves), hopping matrices held fixed, in the convention of hop_force:
        dS/d eps = Re Tr[i T F_rho(y)] for U_rho(y) -> exp(i eps T) U_rho(y).
        With Lambda = c b a^dagger (c = 1 odd, kappa^2 even; a, b as in hop_force),
        G_rn(z) = c sum_s (sigma_rn b)_s a_s^dagger, H = G + G^dagger, and for
        every plane (rho, nu) the plaquettes through U_rho(y) oriented rho -> nu
        with H inserted at each corner:
        F = TA[(i kappa csw / 8) sum_nu (U C_up - E_low U^dagger)].  Shape (V, 4, 3, 3).
        Two flavours (nf = 2): the clover term enters both flavours alike, so G
        sums over the flavour index."""
        _, sig = self.gammas()
        a, b, co, par = self._force_fields(X, Y, sgn, nf)
        V = self.V
        L = self.dims
        c = np.where(par == 1, 1.0, self.kappa ** 2)
        U = self.U
        dag = lambda m: np.conj(np.swapaxes(m, -1, -2))
        mm = lambda *ms: ms[0] if len(ms) == 1 else np.einsum("xij,xjk->xik", ms[0], mm(*ms[1:]))

        def sh(idx, mu, d):
            cc = co[idx].copy()
            cc[:, mu] = (cc[:, mu] + d) % L[mu]
            return cc[:, 0] + L[0] * (cc[:, 1] + L[1] * (cc[:, 2] + L[2] * cc[:, 3]))

        H = {}
        for r in range(4):
            for n in range(4):
                if r != n:
                    sb = np.einsum("st,xftc->xfsc", sig[r, n], b)
                    G = c[:, None, None] * np.einsum("xfsi,xfsj->xij", sb, np.conj(a))
                    H[r, n] = G + dag(G)
        F = np.zeros((V, 4, 3, 3), dtype=np.complex128)
        y = np.arange(V)
        for r in range(4):
            Z = np.zeros((V, 3, 3), dtype=np.complex128)
            Ur = U[:, r]
            for n in range(4):
                if n == r:
                    continue
                h = H[r, n]
                yr, yn = sh(y, r, 1), sh(y, n, 1)
                yrn = sh(yr, n, 1)
                ymn = sh(y, n, -1)
                ymnr = sh(ymn, r, 1)
                # upper plaquette y -> y+r -> y+r+n -> y+n -> y
                a1, a2, a3 = U[yr, n], dag(U[yn, r]), dag(U[y, n])
                B = mm(a1, a2, a3)
                Cup = (mm(B, h[y]) + mm(h[yr], B) + mm(a1, h[yrn], a2, a3) + mm(a1, a2, h[yn], a3))
                # lower plaquette y-n -> y-n+r -> y+r -> y -> y-n, through U_r(y)^dagger
                d1, d2, d3 = dag(U[ymn, n]), U[ymn, r], U[ymnr, n]
                D = mm(d1, d2, d3)
                Elow = (mm(D, h[yr]) + mm(h[y], D) + mm(d1, h[ymn], d2, d3) + mm(d1, d2, h[ymnr], d3))
                Z += mm(Ur, Cup) - mm(Elow, dag(Ur))
            Z *= 1j * self.kappa * self.csw / 8.0
            A = 0.5 * (Z - dag(Z))
            F[:, r] = A - (np.trace(A, axis1=1, axis2=2) / 3.0)[:, None, None] * np.eye(3)
        return F

    # -- rational approximation (Section 4.2) --------------------------------
    def rational(self, b, a0, coeffs, shifts, nf=1, sgn=1, tol=1e-13):
        """a0 b + sum_k coeffs[k] (N + shifts[k])^{-1} b, each solve by the oracle's CG."""
        out = a0 * _c(b)
        for a, s in zip(coeffs, shifts):
            x, _, _ = self.cg(b, nf=nf, sgn=sgn, shift=float(s), tol=tol)
            out = out + a * x
        return out

    def rational_force(self, phi, coeffs, shifts, nf=1, sgn=1, tol=1e-13):
        """Link derivative of S_R = <phi, R(N) phi>, R(N) = a0 + sum_k coeffs[k]
        (N + shifts[k])^{-1}, the action of a rational monomial (Sections 4.2,
        4.3), in the convention of hop_force: with x_k = (N + shifts[k])^{-1} phi,
        dS_R = -sum_k coeffs[k] <x_k, dN x_k> and <x, dN x> = 2 Re<Mhat x, dMhat x>,
        so F_R = -2 sum_k coeffs[k] (hop_force + clover_force)(x_k, Mhat x_k)."""
        F = 0.0
        for a, s in zip(coeffs, shifts):
            x, _, _ = self.cg(phi, nf=nf, sgn=sgn, shift=float(s), tol=tol)
            y = self.mhat(x, nf=nf, sgn=sgn)
            F = F - 2.0 * a * (self.hop_force(x, y, sgn, nf) + self.clover_force(x, y, sgn, nf))
        return F

    def rational_correction(self, eta, a0, coeffs, shifts, nf=1, sgn=1, terms=6):
        """Partial sums of sum_k binom(-1/2, k) <eta, Z^k eta>, Z = N R(N)^2 - 1,
        for k = 1 .. terms (the exponent of the correction factor
        det(1 + Z)^(1/2) = < exp(-eta^dagger [(1 + Z)^(-1/2) - 1] eta) >)."""
        eta = _c(eta)
        v, e, coef, sums = eta, 0.0, 1.0, []
        for k in range(1, terms + 1):
            r2 = self.rational(self.rational(v, a0, coeffs, shifts, nf, sgn), a0, coeffs, shifts, nf, sgn)
            v = self.mdagm(r2, nf=nf, sgn=sgn) - v
            coef *= (-0.5 - (k - 1)) / k
            e += coef * float(np.vdot(eta.reshape(-1), v.reshape(-1)).real)
            sums.append(e)
        return sums

    def residual_mhat(self, b, x, nf=1, sgn=1, dagger=False):
        b, x = _c(b), _c(x)
        return self.lib.orc_residual_mhat(_ptr(self.L), self.t_bc, _ptr(self.U), _ptr(self.T), self.kappa,
                                          self.mu, self.mubar, self.epsbar, nf, sgn, int(bool(dagger)),
                                          _ptr(b), _ptr(x))
