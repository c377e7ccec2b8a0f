"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module draws random numbers and builds gauge fields, sources and gauge
transformations.  It holds none of the Dirac-operator or solver arithmetic:
everything it returns is an *input* to the method.

Layouts (all numpy, complex128):

* gauge links ``U``: ``[t][z][y][x][mu][3][3]`` (row-major SU(3) matrices),
  ``mu`` = 0,1,2,3 <-> x,y,z,t.  The flat site index is the lexicographic
  ``lex = x + Lx*(y + Ly*(z + Lz*t))``.
* full-lattice spinors: ``[lex][flavour][spin 4][colour 3]``.
* one-parity ("checkerboard") spinors: ``[cb][flavour][spin][colour]`` where
  ``cb = lex // 2`` over the sites of that parity (parity = (x+y+z+t) mod 2,
  0 = even); valid because Lx is even.

Link generator (the recipe of the synthetic ensembles): for each direction
``mu`` and time slice ``t`` a generator ``numpy.random.default_rng([seed, mu,
t])`` draws 8 standard normals per site, ``H = sum_a w_a lambda_a / 2`` with the
Gell-Mann matrices, ``U = exp(i eps H)`` through the eigen-decomposition of
``H``, then rows 0 and 1 are Gram-Schmidt orthonormalised and row 2 is set to
``conj(row0 x row1)`` so the link is in SU(3) to rounding.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "gauge_links",
    "unit_links",
    "abelian_flux_links",
    "random_su3",
    "random_gauge_transform",
    "gauge_transform_links",
    "gaussian_spinor",
    "gaussian_cb_spinor",
    "odd_sites",
    "parity_of_lex",
    "cb_to_full",
    "full_to_cb",
]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _project_rows(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt rows 0,1; row 2 = conj(row0 x row1).  u: (..., 3, 3)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def _exp_i_eps_h(w: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for H = sum_a w_a lambda_a/2, w: (..., 8)."""
    lam = gell_mann()
    h = np.einsum("...a,aij->...ij", w, lam) * 0.5
    ev, vec = np.linalg.eigh(h)
    ph = np.exp(1j * eps * ev)
    return np.einsum("...ij,...j,...kj->...ik", vec, ph, np.conj(vec))


def gauge_links(dims, eps: float, seed: int) -> np.ndarray:
    """Seeded SU(3) links U = proj_SU3(exp(i eps H)), shape (Lt,Lz,Ly,Lx,4,3,3).

    dims = (Lx, Ly, Lz, Lt).  Each (direction, time slice) chunk has its own
    generator so the field does not depend on how it is chunked.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    out = np.empty((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        for t in range(lt):
            rng = np.random.default_rng([int(seed), mu, t])
            w = rng.standard_normal((lz, ly, lx, 8))
            out[t, :, :, :, mu] = _project_rows(_exp_i_eps_h(w, eps))
    return out


def unit_links(dims) -> np.ndarray:
    """The free field U = 1."""
    lx, ly, lz, lt = (int(d) for d in dims)
    out = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    out[..., 0, 0] = out[..., 1, 1] = out[..., 2, 2] = 1
    return out


def abelian_flux_links(dims, n: int, q=(1.0, -1.0, 0.0)) -> np.ndarray:
    """Constant abelian magnetic flux through every (x,y) plaquette.

    U_y(x) = diag(exp(i q_c phi x)), U_x(x) = diag(exp(-i q_c phi Lx y)) on the
    last x slice (else 1), all other links 1, phi = 2 pi n / (Lx Ly).  Every
    (x,y) plaquette then equals diag(exp(i q_c phi)) and all other plaquettes
    are 1.  (The charges sum to zero so the links are in SU(3).)
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    out = unit_links(dims)
    phi = 2 * np.pi * n / (lx * ly)
    q = np.asarray(q, dtype=np.float64)
    xs = np.arange(lx)
    ys = np.arange(ly)
    for c in range(3):
        out[:, :, :, :, 1, c, c] = np.exp(1j * q[c] * phi * xs)[None, None, None, :]
        ux = np.ones((ly, lx), dtype=np.complex128)
        ux[:, lx - 1] = np.exp(-1j * q[c] * phi * lx * ys)
        out[:, :, :, :, 0, c, c] = ux[None, None, :, :]
    return out


def random_su3(rng: np.random.Generator, shape) -> np.ndarray:
    """Haar-like random SU(3) matrices of the given leading shape."""
    z = rng.standard_normal(tuple(shape) + (3, 3)) + 1j * rng.standard_normal(tuple(shape) + (3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[..., None, None]
    return _project_rows(q)


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """G(x) in SU(3) per site, shape (Lt,Lz,Ly,Lx,3,3)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng([int(seed), 7777])
    return random_su3(rng, (lt, lz, ly, lx))


def gauge_transform_links(U: np.ndarray, G: np.ndarray) -> np.ndarray:
    """U'_mu(x) = G(x) U_mu(x) G(x+mu)^dagger (periodic shifts)."""
    out = np.empty_like(U)
    # array axes (t,z,y,x) <-> mu (3,2,1,0)
    for mu in range(4):
        ax = 3 - mu
        gshift = np.roll(G, -1, axis=ax)
        out[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(gshift, -1, -2))
    return out


def parity_of_lex(dims) -> np.ndarray:
    """Parity (0 even, 1 odd) of every lexicographic site."""
    lx, ly, lz, lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return ((x + y + z + t) & 1).reshape(-1)


def odd_sites(dims, parity: int = 1) -> np.ndarray:
    """Lexicographic indices of the sites of one parity, in checkerboard order."""
    p = parity_of_lex(dims)
    return np.nonzero(p == parity)[0]


def gaussian_spinor(n_sites: int, seed: int, k: int = 0, nflav: int = 1) -> np.ndarray:
    """Complex Gaussian spinor (Re, Im ~ N(0,1)), shape (n_sites, nflav, 4, 3)."""
    rng = np.random.default_rng([int(seed), 1000 + int(k)])
    a = rng.standard_normal((n_sites, nflav, 4, 3, 2))
    return a[..., 0] + 1j * a[..., 1]


def gaussian_cb_spinor(dims, seed: int, k: int = 0, nflav: int = 1) -> np.ndarray:
    """Gaussian source on the sites of one parity: shape (V/2, nflav, 4, 3)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    return gaussian_spinor(lx * ly * lz * lt // 2, seed, k, nflav)


def cb_to_full(v_cb: np.ndarray, dims, parity: int = 1) -> np.ndarray:
    """Embed a one-parity spinor into a full-lattice one (zeros elsewhere)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    V = lx * ly * lz * lt
    out = np.zeros((V,) + v_cb.shape[1:], dtype=v_cb.dtype)
    out[odd_sites(dims, parity)] = v_cb
    return out


def full_to_cb(v: np.ndarray, dims, parity: int = 1) -> np.ndarray:
    """Restrict a full-lattice spinor to the sites of one parity."""
    return np.ascontiguousarray(v[odd_sites(dims, parity)])
