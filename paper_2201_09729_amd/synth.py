"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module holds no arithmetic of the method (no Dirac operator, clover term,
Laplacian, solver, projector or contraction).  It only draws random inputs:

* gauge fields U = exp(i eps H) with H a random traceless Hermitian 3x3 matrix
  per link (the synthetic stand-in for the paper's CLS ensembles E5/A5, Table 1,
  whose configurations are not available);
* real Z2 noise on one timeslice (the paper's stochastic wall sources, Sec. 2);
* Gaussian start vectors for the Laplacian eigensolver;
* random SU(3) gauge transformations and a constant abelian flux field, used as
  test inputs.

Canonical layouts (complex128, x fastest, dims = (T, Z, Y, X)):
  gauge  [T][Z][Y][X][mu][a][b]   mu = 0:t, 1:x, 2:y, 3:z
  spinor [nrhs][T][Z][Y][X][s][c]
  colour [nt][nvec][Z][Y][X][c]
"""
from __future__ import annotations

import numpy as np


def _random_traceless_hermitian(rng: np.random.Generator, shape) -> np.ndarray:
    """H = (A + A^dag)/2 - tr(H)/3, with A_ij ~ N(0,1) + i N(0,1)."""
    a = rng.standard_normal(shape + (3, 3)) + 1j * rng.standard_normal(shape + (3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real
    h = h - (tr / 3.0)[..., None, None] * np.eye(3)
    return h


def _expi(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for Hermitian H via its eigendecomposition (batched)."""
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, np.conj(v))


def gauge_field(dims, eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """Random SU(3) links U = exp(i eps H), one draw per link, in canonical layout.

    dims = (T, Z, Y, X).  Deterministic given (dims, eps, seed).  Generated in
    chunks of links so that large lattices do not need the full temporary of the
    eigendecomposition at once; the random stream is consumed in canonical order.
    """
    T, Z, Y, X = (int(d) for d in dims)
    nlink = T * Z * Y * X * 4
    rng = np.random.default_rng(seed)
    out = np.empty((nlink, 3, 3), dtype=np.complex128)
    for s in range(0, nlink, chunk):
        e = min(nlink, s + chunk)
        h = _random_traceless_hermitian(rng, (e - s,))
        out[s:e] = _expi(h, eps)
    return out.reshape(T, Z, Y, X, 4, 3, 3)


def unit_gauge(dims) -> np.ndarray:
    """Free field: every link is the identity."""
    T, Z, Y, X = (int(d) for d in dims)
    u = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = 1.0
    u[..., 1, 1] = 1.0
    u[..., 2, 2] = 1.0
    return u


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-ish random SU(3) matrices (QR of a complex Gaussian, phase fixed)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(a)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return q


def gauge_transform(dims, seed: int) -> np.ndarray:
    """A random gauge transformation g(x) in SU(3), shape [T][Z][Y][X][3][3]."""
    T, Z, Y, X = (int(d) for d in dims)
    return random_su3(T * Z * Y * X, seed).reshape(T, Z, Y, X, 3, 3)


def abelian_flux_gauge(dims, plane=(1, 2), n: int = 1) -> np.ndarray:
    """Constant abelian flux phi = 2 pi n / (L_mu L_nu) through every plaquette
    of the (mu, nu) plane, embedded in SU(3) as diag(e^{i th}, e^{-i th}, 1).

    Directions: mu = 0:t, 1:x, 2:y, 3:z.  Periodic in all directions.
    """
    T, Z, Y, X = (int(d) for d in dims)
    ext = {0: T, 1: X, 2: Y, 3: Z}
    axis = {0: 0, 1: 3, 2: 2, 3: 1}  # direction -> array axis in [T][Z][Y][X]
    mu, nu = plane
    Lmu, Lnu = ext[mu], ext[nu]
    phi = 2.0 * np.pi * n / (Lmu * Lnu)
    coords = np.indices((T, Z, Y, X))
    xm = coords[axis[mu]]
    xn = coords[axis[nu]]
    # U_nu(x) = exp(i phi x_mu);  U_mu(x) = exp(-i phi L_mu x_nu) on the last mu slice.
    th_nu = phi * xm
    th_mu = np.where(xm == Lmu - 1, -phi * Lmu * xn, 0.0)
    u = unit_gauge(dims)
    for d, th in ((mu, th_mu), (nu, th_nu)):
        u[..., d, 0, 0] = np.exp(1j * th)
        u[..., d, 1, 1] = np.exp(-1j * th)
    return u, phi


def z2_noise(dims, t0: int, nnoise: int, seed: int, complex_noise: bool = False) -> np.ndarray:
    """Z2 noise per (spatial site, colour) on timeslice t0: [nnoise][Z][Y][X][3].

    Real Z2: float64 values +-1.  Complex Z2: complex128 values (+-1 +- i)/sqrt(2),
    real and imaginary signs drawn independently.  Both have unit modulus, so
    E[xi xi^dag] = 1.
    """
    T, Z, Y, X = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, size=(nnoise, Z, Y, X, 3))
    re = (1.0 - 2.0 * bits).astype(np.float64)
    if not complex_noise:
        return re
    im = 1.0 - 2.0 * rng.integers(0, 2, size=(nnoise, Z, Y, X, 3))
    return (re + 1j * im) / np.sqrt(2.0)


def gaussian_start(dims, nt: int, seed: int) -> np.ndarray:
    """Normalised complex Gaussian start vectors, one per timeslice: [nt][Z][Y][X][3]."""
    T, Z, Y, X = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((nt, Z, Y, X, 3)) + 1j * rng.standard_normal((nt, Z, Y, X, 3))
    nrm = np.sqrt(np.sum(np.abs(v) ** 2, axis=(1, 2, 3, 4)))
    return v / nrm[:, None, None, None, None]


def random_spinor(dims, nrhs: int, seed: int) -> np.ndarray:
    """Complex Gaussian spinor fields [nrhs][T][Z][Y][X][4][3]."""
    T, Z, Y, X = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    shp = (nrhs, T, Z, Y, X, 4, 3)
    return rng.standard_normal(shp) + 1j * rng.standard_normal(shp)


def point_source(dims, site=(0, 0, 0, 0), spin: int = 0, colour: int = 0) -> np.ndarray:
    """A unit point source at site (t, z, y, x), one spin and colour: [1][T][Z][Y][X][4][3]."""
    T, Z, Y, X = (int(d) for d in dims)
    b = np.zeros((1, T, Z, Y, X, 4, 3), dtype=np.complex128)
    b[(0,) + tuple(site) + (spin, colour)] = 1.0
    return b

