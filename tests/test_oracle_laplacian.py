"""CPU pins of the oracle's spatial Laplacian (paper eq. 1), Lanczos eigensolver,
distillation projector and sources."""
import numpy as np
import pytest

from paper_2201_09729_amd import synth
from tests import _dense as D


def dense_lap(orc, U, t):
    shp = tuple(U.shape[1:4]) + (3,)
    n = int(np.prod(shp))

    def ap(cols):
        k = cols.shape[0]
        return orc.laplacian(U, t, cols.reshape((k,) + shp)).reshape(k, n)

    return D.dense_operator(ap, n)


def test_free_laplacian_spectrum(orc):
    """U = 1: eigenvalues -6 + 2 sum_j cos(2 pi n_j / L_j), each with colour multiplicity 3."""
    dims = (2, 4, 6, 4)
    U = synth.unit_gauge(dims)
    L = dense_lap(orc, U, 1)
    assert np.max(np.abs(L - np.conj(L.T))) < 1e-15
    ev = np.sort(np.linalg.eigvalsh(L))
    _, Z, Y, X = dims
    nz, ny, nx = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    lam = -6 + 2 * (np.cos(2 * np.pi * nz / Z) + np.cos(2 * np.pi * ny / Y) + np.cos(2 * np.pi * nx / X))
    ref = np.sort(np.repeat(lam.ravel(), 3))
    assert np.max(np.abs(ev - ref)) < 1e-13


def test_laplacian_plane_wave_axes(orc):
    """Each spatial axis enters with its own extent: lap e^{ip.m} c = (-6 + 2 sum cos p_j) e^{ip.m} c."""
    dims = (3, 4, 6, 8)
    U = synth.unit_gauge(dims)
    _, Z, Y, X = dims
    z, y, x = np.indices((Z, Y, X))
    p = (2 * np.pi * 1 / Z, 2 * np.pi * 2 / Y, 2 * np.pi * 3 / X)
    c = np.array([1.0, 2.0 - 1j, 0.5j])
    v = (np.exp(1j * (p[0] * z + p[1] * y + p[2] * x))[..., None] * c)[None]
    got = orc.laplacian(U, 2, v)
    lam = -6 + 2 * sum(np.cos(q) for q in p)
    assert np.linalg.norm(got - lam * v) / np.linalg.norm(v) < 1e-14


def test_laplacian_gauge_covariance(orc):
    dims = (4, 4, 6, 8)
    U = synth.gauge_field(dims, 0.3, 4)
    g = synth.gauge_transform(dims, 9)
    Ug = D.gauge_transform_links(U, g)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((2, 4, 6, 8, 3)) + 1j * rng.standard_normal((2, 4, 6, 8, 3))
    t = 3
    gt = g[t]
    lhs = orc.laplacian(Ug, t, np.einsum("zyxab,nzyxb->nzyxa", gt, v))
    rhs = np.einsum("zyxab,nzyxb->nzyxa", gt, orc.laplacian(U, t, v))
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs) < 1e-14


def test_laplacian_uses_only_its_timeslice(orc):
    """lap(t) depends only on the spatial links of timeslice t."""
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 4)
    U2 = U.copy()
    U2[1] = synth.gauge_field(dims, 0.5, 99)[1]  # change timeslice 1 only
    U2[:, :, :, :, 0] = synth.gauge_field(dims, 0.5, 98)[:, :, :, :, 0]  # and all temporal links
    v = synth.gaussian_start(dims, 1, 3)
    assert np.array_equal(orc.laplacian(U, 2, v), orc.laplacian(U2, 2, v))
    assert not np.allclose(orc.laplacian(U, 1, v), orc.laplacian(U2, 1, v))


@pytest.mark.parametrize("dims,nev,seed", [((4, 4, 4, 4), 4, 1), ((2, 8, 8, 8), 16, 2)])
def test_lanczos_vs_dense_eigh(orc, dims, nev, seed):
    U = synth.gauge_field(dims, 0.3, seed)
    t = dims[0] - 1
    v0 = synth.gaussian_start(dims, 1, 100 + seed)[0]
    ev, V = orc.lap_eigs(U, t, nev, v0, tol=1e-12)
    L = dense_lap(orc, U, t)
    w, Wd = np.linalg.eigh(-L)
    assert np.max(np.abs(-ev - w[:nev])) < 1e-11
    assert np.all(np.diff(ev) <= 0) and np.all(ev <= 0)
    Vm = V.reshape(nev, -1)
    assert np.max(np.abs(Vm.conj() @ Vm.T - np.eye(nev))) < 1e-12
    res = np.linalg.norm(Vm @ L.T - ev[:, None] * Vm, axis=1)
    assert res.max() < 1e-9
    gap = w[nev] - w[nev - 1]
    Pl = Vm.T @ Vm.conj()
    Pd = Wd[:, :nev] @ np.conj(Wd[:, :nev].T)
    assert np.linalg.norm(Pl - Pd, 2) < 1e-9 / gap
    # phase convention: largest component real positive
    for k in range(nev):
        i = np.argmax(np.abs(Vm[k]))
        assert abs(Vm[k, i].imag) < 1e-14 and Vm[k, i].real > 0


def test_projector_algebra(orc):
    dims = (4, 4, 4, 6)
    U = synth.gauge_field(dims, 0.3, 5)
    nev = 5
    t = 2
    ev, Vt = orc.lap_eigs(U, t, nev, synth.gaussian_start(dims, 1, 5)[0], tol=1e-12)
    T = dims[0]
    L3 = int(np.prod(dims[1:]))
    n = L3 * 12
    cols = np.zeros((n, T) + tuple(dims[1:]) + (4, 3), complex)
    cols.reshape(n, T, n)[np.arange(n), t, np.arange(n)] = 1.0
    P = orc.project(Vt, cols, t, 0)[:, t].reshape(n, n).T
    Q = orc.project(Vt, cols, t, 1)[:, t].reshape(n, n).T
    assert np.max(np.abs(P @ P - P)) < 1e-13
    assert np.max(np.abs(P - np.conj(P.T))) < 1e-14
    assert abs(np.trace(P) - 4 * nev) < 1e-12
    assert np.max(np.abs(P + Q - np.eye(n))) < 1e-14
    src = orc.dist_sources(Vt, T, t)
    assert np.max(np.abs(orc.project(Vt, src, t, 1))) < 1e-13
    assert np.max(np.abs(orc.project(Vt, src, t, 0) - src)) < 1e-13
    # zero off the timeslice
    x = synth.random_spinor(dims, 1, 2)
    out = orc.project(Vt, x, t, 1)
    assert np.all(out[0, :t] == 0) and np.all(out[0, t + 1:] == 0)


def test_sources_layout(orc):
    dims = (4, 2, 2, 4)
    T = dims[0]
    xi = synth.z2_noise(dims, 1, 2, 7)
    src = orc.noise_sources(xi, T, 1)
    assert src.shape == (8, T, 2, 2, 4, 4, 3)
    for r in range(2):
        for s in range(4):
            blk = src[r * 4 + s]
            assert np.array_equal(blk[1, ..., s, :], xi[r])
            mask = np.ones(blk.shape, bool)
            mask[1, ..., s, :] = False
            assert np.all(blk[mask] == 0)
    assert set(np.unique(xi)) == {-1.0, 1.0}
