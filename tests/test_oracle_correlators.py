"""CPU pins of the oracle's correlator pieces (paper eq. 2-4) against dense traces.

On a 4^4 lattice the full propagator S = D^-1 is formed densely (LAPACK inverse of
the dense operator), and every trace tr[g5 G X_t S(t,t0) Y_t0 G g5 S(t,t0)^dag] is
evaluated directly as a matrix product (tests/_dense.py), independently of the
oracle's perambulator and estimator code.
"""
import numpy as np
import pytest

from paper_2201_09729_amd import synth
from tests import _dense as D

GAM = {"PS": [D.G5], "V": [D.G[1], D.G[2], D.G[3]]}


@pytest.fixture(scope="module")
def sys44(orc):
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.3, 1)
    kappa, csw = 0.120, 1.0
    A = orc.clover(U, kappa, csw)
    Dd = D.dense_dirac(orc, U, A)
    S = np.linalg.inv(Dd)
    nev = 3
    T = dims[0]
    Vall = np.stack([orc.lap_eigs(U, t, nev, synth.gaussian_start(dims, 1, 50 + t)[0], tol=1e-12)[1]
                     for t in range(T)])
    return dims, U, A, S, Vall, nev


def dense_parts(S, dims, Vall, t0, name):
    T = dims[0]
    out = {}
    for X in "1PQ":
        for Y in "1PQ":
            c = np.zeros(T, complex)
            for d in range(T):
                t = (t0 + d) % T
                c[d] = np.mean([D.dense_trace(S, dims, Vall, t, t0, G, X, Y) for G in GAM[name]])
            out[X + Y] = c
    return out


def apply_S(S, src):
    n = src.shape[0]
    return (S @ src.reshape(n, -1).T).T.reshape(src.shape)


@pytest.mark.parametrize("name", ["PS", "V"])
def test_exact_parts_vs_dense(orc, sys44, name):
    dims, U, A, S, Vall, nev = sys44
    T = dims[0]
    t0 = 1
    ref = dense_parts(S, dims, Vall, t0, name)
    src = orc.dist_sources(Vall[t0], T, t0)
    phid = apply_S(S, src).reshape((nev, 4) + src.shape[1:])
    cd = orc.c_dist_exact(Vall, t0, phid, name)
    cqp = orc.c_qp_exact(Vall, t0, phid, name)
    scale = np.max(np.abs(ref["11"]))
    assert np.max(np.abs(cd - ref["PP"])) < 1e-12 * scale
    assert np.max(np.abs(cqp - ref["QP"])) < 1e-12 * scale
    # split of the full correlator is exact per configuration (both mixed orders)
    tot = ref["QQ"] + ref["PQ"] + ref["QP"] + ref["PP"]
    assert np.max(np.abs(tot - ref["11"])) < 1e-12 * scale
    # traces are real, and positive at distance 1 with this sign convention
    assert np.max(np.abs(ref["11"].imag)) < 1e-12 * scale
    assert ref["11"][1].real > 0


@pytest.mark.parametrize("name", ["PS", "V"])
def test_full_dilution_estimator_is_exact(orc, sys44, name):
    """With xi running over all unit vectors of the timeslice (sum instead of mean),
    the one-end estimator of eq. (3) equals the exact trace for every X, Y."""
    dims, U, A, S, Vall, nev = sys44
    T = dims[0]
    t0 = 2
    L3 = int(np.prod(dims[1:]))
    xi = np.eye(L3 * 3).reshape((L3 * 3,) + tuple(dims[1:]) + (3,))
    eta = orc.noise_sources(xi, T, t0)
    etab = orc.project(Vall[t0], eta, t0, 1)
    phi = apply_S(S, eta)
    phib = apply_S(S, etab)
    src = orc.dist_sources(Vall[t0], T, t0)
    phid = apply_S(S, src)
    got = orc.correlators(Vall, t0, phid, phi, phib, names=(name,))[name]
    ref = dense_parts(S, dims, Vall, t0, name)
    Nr = L3 * 3
    scale = np.max(np.abs(ref["11"]))
    for part, key in (("QQ_est", "QQ"), ("PQ_est", "PQ"), ("QP_est", "QP"), ("PP_est", "PP"), ("11_est", "11")):
        assert np.max(np.abs(Nr * got[part] - ref[key])) < 1e-11 * scale, part
    assert np.max(np.abs(got["PP_exact"] - ref["PP"])) < 1e-12 * scale
    assert np.max(np.abs(got["QP_exact"] - ref["QP"])) < 1e-12 * scale


def test_source_sink_swap_identity(sys44):
    """C_QP(t; t0) = C_PQ(t0; t): the exact form behind the paper's time-reversal
    combination of the two mixed terms (eq. 2)."""
    dims, U, A, S, Vall, nev = sys44
    for name in ("PS", "V"):
        for t0, t in ((0, 1), (1, 3), (2, 0)):
            a = np.mean([D.dense_trace(S, dims, Vall, t, t0, G, "Q", "P") for G in GAM[name]])
            b = np.mean([D.dense_trace(S, dims, Vall, t0, t, G, "P", "Q") for G in GAM[name]])
            assert abs(a - b) < 1e-12 * abs(a)


def test_z2_estimator_statistics_and_linearity(orc, sys44):
    """Real Z2 noise: the sample mean converges to the exact trace (within 4 standard
    errors), and per sample QQ + PQ + QP + PP = 11 exactly (linearity)."""
    dims, U, A, S, Vall, nev = sys44
    T = dims[0]
    t0 = 0
    nn = 48
    xi = synth.z2_noise(dims, t0, nn, 1234)
    eta = orc.noise_sources(xi, T, t0)
    etab = orc.project(Vall[t0], eta, t0, 1)
    phi = apply_S(S, eta)
    phib = apply_S(S, etab)
    src = orc.dist_sources(Vall[t0], T, t0)
    phid = apply_S(S, src)
    ref = dense_parts(S, dims, Vall, t0, "PS")
    samples = []
    for r in range(nn):
        sl = slice(4 * r, 4 * r + 4)
        c = orc.correlators(Vall, t0, phid, phi[sl], phib[sl], names=("PS",))["PS"]
        tot = c["QQ_est"] + c["PQ_est"] + c["QP_est"] + c["PP_est"]
        assert np.max(np.abs(tot - c["11_est"])) < 1e-12 * np.max(np.abs(c["11_est"]))
        samples.append([c["11_est"], c["QQ_est"], c["PQ_est"]])
    samples = np.array(samples)  # [nn][3][T]
    mean = samples.mean(axis=0)
    err = samples.std(axis=0, ddof=1) / np.sqrt(nn)
    for i, key in enumerate(("11", "QQ", "PQ")):
        dev = np.abs(mean[i] - ref[key])
        assert np.all(dev <= 4 * np.abs(err[i]) + 1e-12 * np.max(np.abs(ref["11"]))), key


@pytest.mark.parametrize("dilution,ncol,npar", [("spin", 1, 1), ("spin-colour", 3, 1), ("spin-eo", 1, 2),
                                                ("spin-colour-eo", 3, 2)])
@pytest.mark.parametrize("complex_noise", [False, True])
def test_diluted_estimator_matches_dense_noise_trace(orc, sys44, dilution, ncol, npar, complex_noise):
    """One noise vector split into colour and/or even-odd components, each spin-diluted:
    the oracle's estimator equals the dense trace with the wall identity replaced by
    sum_d P_d xi xi^dag P_d, for every X, Y (eq. 3 with dilution)."""
    dims, U, A, S, Vall, nev = sys44
    T = dims[0]
    t0 = 3
    xi = synth.z2_noise(dims, t0, 1, 77, complex_noise=complex_noise)
    assert orc.dilution_size(dilution) == ncol * npar
    eta = orc.noise_sources(xi, T, t0, dilution)
    assert eta.shape[0] == 4 * ncol * npar
    etab = orc.project(Vall[t0], eta, t0, 1)
    phi = apply_S(S, eta)
    phib = apply_S(S, etab)
    phid = apply_S(S, orc.dist_sources(Vall[t0], T, t0))
    N = D.wall_noise_matrix(xi[0], dims, t0, ncol, npar)
    for name in ("PS", "V"):
        got = orc.correlators(Vall, t0, phid, phi, phib, names=(name,), ndil=ncol * npar)[name]
        scale = None
        for part, (X, Y) in (("QQ_est", "QQ"), ("PQ_est", "PQ"), ("QP_est", "QP"), ("PP_est", "PP"), ("11_est", "11")):
            ref = np.array([np.mean([D.dense_trace_noise(S, dims, Vall, (t0 + d) % T, t0, G, X, Y, N)
                                     for G in GAM[name]]) for d in range(T)])
            if scale is None:
                scale = np.max(np.abs(ref))
            assert np.max(np.abs(got[part] - ref)) < 1e-11 * scale, (name, part)


def test_dilution_components_partition_the_noise(orc):
    """The diluted components of a noise vector add back up to it, and components of
    different d do not overlap (they split colour and wall parity)."""
    dims = (4, 4, 6, 8)
    T = dims[0]
    xi = synth.z2_noise(dims, 1, 2, 5, complex_noise=True)
    for dil in ("spin", "spin-colour", "spin-eo", "spin-colour-eo"):
        nd = orc.dilution_size(dil)
        eta = orc.noise_sources(xi, T, 1, dil).reshape((2, nd, 4) + (T,) + dims[1:] + (4, 3))
        for r in range(2):
            tot = eta[r].sum(axis=0)  # [4][T][Z][Y][X][4][3]
            for s in range(4):
                assert np.array_equal(tot[s, 1, ..., s, :], xi[r])
                support = np.abs(eta[r, :, s]) > 0
                assert np.all(support.sum(axis=0) <= 1)


def test_complex_z2_noise():
    xi = synth.z2_noise((4, 4, 4, 4), 0, 3, 9, complex_noise=True)
    assert np.allclose(np.abs(xi), 1.0)
    assert set(np.unique(np.round(xi.real * np.sqrt(2)))) == {-1.0, 1.0}
    assert set(np.unique(np.round(xi.imag * np.sqrt(2)))) == {-1.0, 1.0}
    # real Z2 draws are unchanged by the option
    assert np.array_equal(synth.z2_noise((4, 4, 4, 4), 0, 3, 9), np.sign(xi.real) * 1.0)


@pytest.mark.parametrize("ndil", [1, 2])
def test_correlator_vjp_is_the_derivative_of_the_contraction(orc, ndil):
    """The backward of the contractions against the forward: every piece is a Hermitian
    quadratic form in the solution fields u = (phi_dist, phi, phibar), so
    [C(u + d) - C(u - d)] / 2 is its exact directional derivative.  For random weights G
    and directions d, Re sum conj(G) [C(u + d) - C(u - d)] / 2 must equal
    Re <grad, d> from correlators_vjp, to rounding.  Also with fewer distillation solution
    groups than modes (the pieces are sums over source groups)."""
    dims = (4, 4, 2, 4)
    T = dims[0]
    rng = np.random.default_rng(31)
    nev, ndist, ng, t0 = 3, 2, 2 * ndil, 1
    U = synth.gauge_field(dims, 0.3, 2)
    Vall = np.stack([orc.lap_eigs(U, t, nev, synth.gaussian_start(dims, 1, 70 + t)[0], tol=1e-12)[1] for t in range(T)])

    def rnd(n):
        return rng.normal(size=(n,) + dims + (4, 3)) + 1j * rng.normal(size=(n,) + dims + (4, 3))

    u = [rnd(4 * ndist), rnd(4 * ng), rnd(4 * ng)]
    d = [rnd(4 * ndist), rnd(4 * ng), rnd(4 * ng)]
    G = {name: {p: rng.normal(size=T) + 1j * rng.normal(size=T) for p in orc.PARTS} for name in ("PS", "V")}
    cp = orc.correlators(Vall, t0, *[a + b for a, b in zip(u, d)], ndil=ndil)
    cm = orc.correlators(Vall, t0, *[a - b for a, b in zip(u, d)], ndil=ndil)
    lhs = sum(np.sum(np.conj(G[n][p]) * (cp[n][p] - cm[n][p]) / 2).real for n in G for p in orc.PARTS)
    grads = orc.correlators_vjp(Vall, t0, *u, G, ndil=ndil)
    rhs = sum(np.vdot(gf, df).real for gf, df in zip(grads, d))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + sum(np.abs(gf).sum() * np.abs(df).max() for gf, df in zip(grads, d))), (lhs, rhs)
    # and piece by piece for one (Gamma, piece, Delta) at a time: the weights act where they should
    for n, p, dl in (("PS", "PP_exact", 2), ("V", "QQ_est", 0), ("PS", "11_est", 3)):
        G1 = {n: {p: np.eye(T)[dl]}}
        g1 = orc.correlators_vjp(Vall, t0, *u, G1, ndil=ndil)
        lhs1 = ((cp[n][p][dl] - cm[n][p][dl]) / 2).real
        rhs1 = sum(np.vdot(gf, df).real for gf, df in zip(g1, d))
        assert abs(lhs1 - rhs1) <= 1e-12 * max(1.0, abs(lhs1)) * 1e2, (n, p, lhs1, rhs1)
        # the gradient lives on the sink timeslice t0 + Delta only
        tt = (t0 + dl) % T
        for gf in g1:
            mask = np.ones(T, bool)
            mask[tt] = False
            assert np.max(np.abs(gf[:, mask])) == 0.0
