"""CPU pins of the oracle's Wilson-clover operator, clover term and solver.

Each test checks the oracle against something other than itself: closed forms
(free field in momentum space, constant abelian flux), invariants
(gamma5-hermiticity, gauge covariance) and library routines (dense LU).
"""
import numpy as np
import pytest

from paper_2201_09729_amd import synth
from tests import _dense as D


def test_gamma_convention(orc):
    g = orc.gammas()
    ref = D.gammas_convention()
    assert np.array_equal(g, ref)
    for a in range(4):
        assert np.allclose(g[a], np.conj(g[a].T))
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2.0 * (a == b) * np.eye(4), atol=0)
    assert np.allclose(g[0] @ g[1] @ g[2] @ g[3], g[4], atol=0)


def _plane_wave(dims, n, u):
    """psi(x) = exp(i p.x) u with p_mu = 2 pi n_mu / L_mu."""
    T, Z, Y, X = dims
    t, z, y, x = np.indices(dims)
    L = {0: T, 1: X, 2: Y, 3: Z}
    coord = {0: t, 1: x, 2: y, 3: z}
    p = np.array([2 * np.pi * n[mu] / L[mu] for mu in range(4)])
    ph = np.exp(1j * sum(p[mu] * coord[mu] for mu in range(4)))
    return (ph[..., None, None] * u[None, None, None, None])[None], p


@pytest.mark.parametrize("n", [(1, 0, 0, 0), (0, 1, 2, 3), (2, 3, 1, 1), (5, 1, 0, 2)])
def test_free_field_plane_wave(orc, n):
    """D e^{ipx} u = e^{ipx} [m0 + sum(1 - cos p) + i sum gamma_mu sin p_mu] u."""
    dims = (6, 4, 8, 10)
    kappa = 0.12
    m0 = 1.0 / (2 * kappa) - 4
    U = synth.unit_gauge(dims)
    A = orc.clover(U, kappa, 1.0)
    rng = np.random.default_rng(0)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi, p = _plane_wave(dims, n, u)
    g = D.gammas_convention()
    Mp = (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4))
    ph = psi[0][..., 0, 0] / u[0, 0]
    expect = ph[..., None, None] * (Mp @ u)[None, None, None, None]
    got = orc.dirac(U, A, psi)[0]
    err = np.linalg.norm(got - expect) / np.linalg.norm(expect)
    assert err < 1e-13


def test_free_propagator_fft(orc):
    """Free S(x,0) = (1/V) sum_p e^{ipx} (m(p) - i sum g sin p)/(m(p)^2 + sum sin^2 p)."""
    dims = (8, 4, 6, 4)
    kappa = 0.12
    m0 = 1.0 / (2 * kappa) - 4
    U = synth.unit_gauge(dims)
    A = orc.clover(U, kappa, 1.3)
    g = D.gammas_convention()
    tol = 1e-12
    T, Z, Y, X = dims
    kt, kz, ky, kx = np.meshgrid(*(2 * np.pi * np.fft.fftfreq(L) for L in dims), indexing="ij")
    pm = {0: kt, 1: kx, 2: ky, 3: kz}
    mp = m0 + sum(1 - np.cos(pm[mu]) for mu in range(4))
    den = mp ** 2 + sum(np.sin(pm[mu]) ** 2 for mu in range(4))
    Sp = (mp[..., None, None] * np.eye(4) - 1j * sum(np.sin(pm[mu])[..., None, None] * g[mu] for mu in range(4))) / den[..., None, None]
    # S(x, 0) = (1/V) sum_p e^{ipx} S(p) = ifftn over the lattice axes
    Sx = np.fft.ifftn(Sp, axes=(0, 1, 2, 3))
    for spin, col in [(0, 0), (2, 1), (3, 2)]:
        b = synth.point_source(dims, (0, 0, 0, 0), spin, col)
        x, its, res, conv = orc.solve(U, A, b, tol=tol)
        assert conv[0] and res[0] <= tol
        expect = np.zeros(dims + (4, 3), complex)
        expect[..., :, col] = Sx[..., :, spin]
        err = np.linalg.norm(x[0] - expect) / np.linalg.norm(expect)
        assert err < 50 * tol, err


@pytest.fixture(scope="module")
def small_system(orc):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 1)
    A = orc.clover(U, 0.120, 1.0)
    Dd = D.dense_dirac(orc, U, A)
    return dims, U, A, Dd


def test_gamma5_hermiticity_dense(small_system):
    dims, U, A, Dd = small_system
    V = int(np.prod(dims))
    g5 = np.kron(np.eye(V), np.kron(D.G5, np.eye(3)))
    lhs = g5 @ Dd @ g5
    assert np.max(np.abs(lhs - np.conj(Dd.T))) < 1e-14


def test_dagger_matches_adjoint(orc, small_system):
    dims, U, A, Dd = small_system
    psi = synth.random_spinor(dims, 2, 7)
    got = orc.dirac(U, A, psi, dagger=True).reshape(2, -1)
    ref = (np.conj(Dd.T) @ psi.reshape(2, -1).T).T
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-14


def test_solver_vs_dense_lu(orc, small_system):
    dims, U, A, Dd = small_system
    b = synth.random_spinor(dims, 3, 11)
    x, its, res, conv = orc.solve(U, A, b, tol=1e-12)
    assert conv.all() and (res <= 1e-12).all()
    xref = np.linalg.solve(Dd, b.reshape(3, -1).T).T
    err = np.linalg.norm(x.reshape(3, -1) - xref, axis=1) / np.linalg.norm(xref, axis=1)
    cond = np.linalg.cond(Dd)
    assert (err <= cond * 1e-12 * 2).all(), (err, cond)


def test_gauge_covariance(orc):
    """D[U^g] (g psi) = g (D[U] psi) and A[U^g](x) = g(x) A[U](x) g(x)^dag."""
    dims = (4, 6, 4, 8)
    U = synth.gauge_field(dims, 0.4, 5)
    g = synth.gauge_transform(dims, 6)
    Ug = D.gauge_transform_links(U, g)
    A = orc.clover(U, 0.121, 1.2)
    Ag = orc.clover(Ug, 0.121, 1.2)
    psi = synth.random_spinor(dims, 1, 8)
    gpsi = np.einsum("tzyxab,ntzyxsb->ntzyxsa", g, psi)
    lhs = orc.dirac(Ug, Ag, gpsi)
    rhs = np.einsum("tzyxab,ntzyxsb->ntzyxsa", g, orc.dirac(U, A, psi))
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs) < 1e-13
    gv = g.reshape(-1, 3, 3)
    Gx = np.einsum("st,vab->vsatb", np.eye(4), gv).reshape(-1, 12, 12)
    Arot = Gx @ A @ np.conj(np.swapaxes(Gx, 1, 2))
    assert np.max(np.abs(Ag - Arot)) < 1e-13


def test_clover_structure(orc):
    dims = (4, 4, 6, 4)
    U = synth.gauge_field(dims, 0.3, 2)
    kappa, csw = 0.121, 1.2
    m0 = 1.0 / (2 * kappa) - 4
    A = orc.clover(U, kappa, csw)
    # Hermitian
    assert np.max(np.abs(A - np.conj(np.swapaxes(A, 1, 2)))) < 1e-15
    # commutes with gamma5: block diagonal in chirality (spins 0,1 vs 2,3)
    Ab = A.reshape(-1, 4, 3, 4, 3)
    assert np.max(np.abs(Ab[:, 0:2, :, 2:4, :])) < 1e-16
    assert np.max(np.abs(Ab[:, 2:4, :, 0:2, :])) < 1e-16
    # vanishes (apart from the mass) for the free field
    A0 = orc.clover(synth.unit_gauge(dims), kappa, csw)
    assert np.max(np.abs(A0 - (4 + m0) * np.eye(12)[None])) < 1e-15
    # non-trivial for the random field
    assert np.max(np.abs(A - (4 + m0) * np.eye(12)[None])) > 1e-2


@pytest.mark.parametrize("plane,n", [((1, 2), 1), ((0, 3), 2), ((2, 3), 1), ((0, 1), 3)])
def test_clover_abelian_flux(orc, plane, n):
    """Constant flux phi in the (mu,nu) plane, colour embedding diag(e^{i th}, e^{-i th}, 1):
    Fhat_{mu nu} = i sin(phi) diag(1, -1, 0), all other planes zero, and
    A = (4+m0) + csw (i/2) sigma_{mu nu} x Fhat_{mu nu}."""
    dims = (6, 4, 6, 8)
    U, phi = synth.abelian_flux_gauge(dims, plane, n)
    F = orc.field_strength(U)
    planes = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    pi = planes.index(plane)
    expect = 1j * np.sin(phi) * np.diag([1.0, -1.0, 0.0])
    for q in range(6):
        ref = expect if q == pi else np.zeros((3, 3))
        assert np.max(np.abs(F[:, q] - ref[None])) < 1e-14
    kappa, csw = 0.12, 1.7
    m0 = 1.0 / (2 * kappa) - 4
    g = D.gammas_convention()
    mu, nu = plane
    sig = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
    Aref = (4 + m0) * np.eye(12) + csw * 0.5j * np.kron(sig, expect)
    A = orc.clover(U, kappa, csw)
    assert np.max(np.abs(A - Aref[None])) < 1e-14


def test_mass_enters_as_identity(orc):
    """D(m0') - D(m0) = (m0' - m0) 1, hence dS/dm0 = -S^2."""
    dims = (4, 4, 4, 6)
    U = synth.gauge_field(dims, 0.3, 3)
    psi = synth.random_spinor(dims, 1, 9)
    k1, k2 = 0.120, 0.1215
    d1 = orc.dirac(U, orc.clover(U, k1, 1.0), psi)
    d2 = orc.dirac(U, orc.clover(U, k2, 1.0), psi)
    dm = (1 / (2 * k2) - 4) - (1 / (2 * k1) - 4)
    assert np.linalg.norm(d2 - d1 - dm * psi) / np.linalg.norm(psi) < 1e-14


def test_mass_derivative_of_solution(orc, small_system):
    """Central finite difference of x(m0) = D(m0)^-1 b against the closed form -S^2 b."""
    dims, U, A, Dd = small_system
    b = synth.random_spinor(dims, 1, 12)
    kappa = 0.120
    m0 = 1 / (2 * kappa) - 4
    h = 1e-4
    kp = 1.0 / (2 * (m0 + h) + 8)
    km = 1.0 / (2 * (m0 - h) + 8)
    xp = orc.solve(U, orc.clover(U, kp, 1.0), b, tol=1e-13)[0]
    xm = orc.solve(U, orc.clover(U, km, 1.0), b, tol=1e-13)[0]
    fd = (xp - xm).reshape(-1) / (2 * h)
    S = np.linalg.inv(Dd)
    ref = -(S @ (S @ b.reshape(-1)))
    assert np.linalg.norm(fd - ref) / np.linalg.norm(ref) < 1e-6


def test_true_residual_vs_dense(orc, small_system):
    """The residual every solve test asserts on: |b - D x|_2 / |b|_2 per right-hand side, in
    FP64 and not squared (the reading of the 1e-10 residual), against the dense 4^4
    operator.  Right-hand sides of very different norms, so that a reduction over the
    wrong axes, a normalisation by |x| or a missing square root fails."""
    dims, U, A, Dd = small_system
    n = 4
    scale = np.array([1.0, 1e-3, 50.0, 7.0])
    b = synth.random_spinor(dims, n, 21) * scale[:, None, None, None, None, None, None]
    bm = b.reshape(n, -1)
    bn = np.linalg.norm(bm, axis=1)
    xlu = np.linalg.solve(Dd, bm.T).T
    # x = 0: residual 1 exactly
    assert np.allclose(orc.true_residual(U, A, np.zeros_like(b), b), 1.0, rtol=0, atol=1e-15)
    # x = c x_lu: residual |1 - c| per right-hand side (complex c, one per RHS)
    c = np.array([0.5 + 0.5j, 2.0, -1.0, 1j])
    xc = (c[:, None] * xlu).reshape(b.shape)
    got = orc.true_residual(U, A, xc, b)
    assert np.allclose(got, np.abs(1 - c), rtol=1e-12, atol=0), (got, np.abs(1 - c))
    # x = x_lu + delta: residual |D delta| / |b|, delta of a different size per RHS
    rng = np.random.default_rng(22)
    eps = np.array([1e-3, 0.0, 0.3, 1e-6])
    delta = (rng.normal(size=bm.shape) + 1j * rng.normal(size=bm.shape)) * (eps * bn)[:, None] / np.sqrt(bm.shape[1])
    got = orc.true_residual(U, A, (xlu + delta).reshape(b.shape), b)
    ref = np.linalg.norm(delta @ Dd.T, axis=1) / bn
    assert got[1] < 1e-13, got
    nz = eps > 0
    assert np.allclose(got[nz], ref[nz], rtol=1e-8, atol=0), (got, ref)


def test_cgls_fixed_is_the_krylov_minimiser(orc, small_system):
    """The timed CGLS run: k iterations from x = 0 give the minimiser of |b - D x|_2 over
    the Krylov space K_k(D^dag D, D^dag b) (the defining property of CG on the normal
    equations), computed here by a dense least-squares problem in an orthonormal basis
    of that space; its returned residual is |b - D x_k| / |b|."""
    dims, U, A, Dd = small_system
    b = synth.random_spinor(dims, 1, 23)
    bv = b.reshape(-1)
    Dh = np.conj(Dd.T)
    w = Dh @ bv
    basis = []
    for k in range(1, 6):
        basis.append(w)
        Q, _ = np.linalg.qr(np.stack(basis, axis=1))
        y, *_ = np.linalg.lstsq(Dd @ Q, bv, rcond=None)
        xref = Q @ y
        x, res = orc.cgls_fixed(U, A, b[0], k)
        err = np.linalg.norm(x.reshape(-1) - xref) / np.linalg.norm(xref)
        assert err < 1e-10, (k, err)
        rref = np.linalg.norm(bv - Dd @ x.reshape(-1)) / np.linalg.norm(bv)
        assert abs(res - rref) <= 1e-12 * rref, (k, res, rref)
        w = Dh @ (Dd @ w)
    # many iterations converge to the dense solution
    x, res = orc.cgls_fixed(U, A, b[0], 160)
    xlu = np.linalg.solve(Dd, bv)
    assert np.linalg.norm(x.reshape(-1) - xlu) / np.linalg.norm(xlu) < 1e-11
    assert res < 1e-12
