"""GPU parity at the full sizes of the workload configurations.

  * 8^3 x 16, FP64 single-RHS even-odd CG: the whole chain (Laplacian modes from the
    oracle, 64 distillation + 16 stochastic solves, contractions) against the oracle's
    own solves and contractions;
  * 16^3 x 32, 128 distillation right-hand sides in one FP16 multi-RHS solve;
  * the uneven batch 3 x 12^3x24 + 2 x 16^3x32 + 1 x 24^3x48 in one BF16 solve;
  * 24^3 x 48 in the benchmark's launch configuration (192 RHS, 2 per thread);
  * 32^3 x 64 FP64 solves with the adjoint-solve gradient d/dm0 against finite differences.

At these sizes the oracle checks what it can compute one item at a time: its own
solves of sampled right-hand sides whose inputs come from the seeded generators,
the FP64 true residual |b - D x| / |b| of sampled GPU solutions under the oracle's
operator, and the eigen-residual |lap v - lambda v| of the GPU's Laplacian modes
under the oracle's Laplacian.  The exact split C_11 = C_QQ + C_PQ + C_QP + C_PP
holds at any size and is checked on the GPU correlators.
"""
import numpy as np
import pytest

from paper_2201_09729_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10
RES_SLACK = 1.0 + 1e-4  # the GPU and the oracle sum the FP64 residual in different orders


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_09729_amd import dlma
    dlma.load_library()
    return dlma


@pytest.fixture(autouse=True)
def _release():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def oracle_relres(orc, U, A, x, b):
    """|b - D x| / |b| under the oracle's operator for one right-hand side [T][Z][Y][X][4][3]."""
    return float(orc.true_residual(U, A, x[None], b[None])[0])


def check_modes(orc, U, t, V, ev, tol):
    """GPU Laplacian modes of timeslice t under the oracle's Laplacian: eigen-residual,
    orthonormality, ascending order of -lap."""
    V = V.cpu().numpy()
    nev = V.shape[0]
    G = V.reshape(nev, -1).conj() @ V.reshape(nev, -1).T
    assert np.max(np.abs(G - np.eye(nev))) < 1e-11
    r = orc.laplacian(U, t, V) - ev[:, None, None, None, None] * V
    res = np.linalg.norm(r.reshape(nev, -1), axis=1)
    assert np.all(res <= 12.0 * tol * 1.01), res
    assert np.all(np.diff(ev) <= 1e-12)  # lap eigenvalues descending (-lap ascending)


def test_pipeline_8x16_fp64_single_rhs(D, orc):
    """8^3 x 16, N = 16 modes (64 distillation sources), 2 Z2 vectors spin-diluted
    (8 eta + 8 (1 - box) eta = 16 stochastic solves), FP64 single-RHS even-odd CG to
    1e-10: every correlator part against the oracle's own chain."""
    dims = (16, 8, 8, 8)
    kappa, csw, nev, t0, nn = 0.120, 1.0, 16, 0, 2
    T = dims[0]
    U = synth.gauge_field(dims, 0.3, 2)
    A = orc.clover(U, kappa, csw)
    v0 = synth.gaussian_start(dims, T, 502)
    Vall = np.stack([orc.lap_eigs(U, t, nev, v0[t], tol=1e-12)[1] for t in range(T)])
    xi = synth.z2_noise(dims, t0, nn, 1002)
    src = orc.dist_sources(Vall[t0], T, t0)
    eta = orc.noise_sources(xi, T, t0)
    etab = orc.project(Vall[t0], eta, t0, 1)
    phid = orc.solve(U, A, src, tol=1e-12)[0]
    phi = orc.solve(U, A, eta, tol=1e-12)[0]
    phib = orc.solve(U, A, etab, tol=1e-12)[0]
    ref = orc.correlators(Vall, t0, phid, phi, phib)

    g = D.dlma_load_gauge(cu(U), kappa, csw)
    opts = D.default_opts(tol=TOL, prec="fp64", rhs_block=1)
    (pd, p1, pb), st = D.dlma_solve([g, g, g], [cu(src), cu(eta), cu(etab)], opts=opts)
    assert all(s["converged"] and s["relres"] <= TOL for s in st)
    # solutions: relative error bounded by cond(D) * (1e-10 + 1e-12)
    for got, want in ((pd, phid), (p1, phi), (pb, phib)):
        gn = got.cpu().numpy()
        err = np.linalg.norm((gn - want).reshape(len(want), -1), axis=1) / np.linalg.norm(want.reshape(len(want), -1), axis=1)
        assert np.max(err) < 1e-8, np.max(err)
    got = D.dlma_correlators(g, t0, cu(Vall), pd, p1, pb)
    for name in ("PS", "V"):
        scale = np.max(np.abs(ref[name]["11_est"]))
        for part in orc.PARTS:
            err = np.max(np.abs(got[name][part] - ref[name][part]))
            assert err < 5e-8 * scale, (name, part, err / scale)
        s = sum(got[name][p] for p in ("QQ_est", "PQ_est", "QP_est", "PP_est"))
        assert np.max(np.abs(s - got[name]["11_est"])) < 1e-12 * scale


def test_fp16_multi_rhs_16x32(D, orc):
    """16^3 x 32, eps 0.25, kappa 0.121, c_sw 1.2: 128 distillation sources (N = 32 x 4
    spins) plus 4 Z2 wall sources in one mixed FP16 solve to 1e-10."""
    dims = (32, 16, 16, 16)
    kappa, csw, nev, t0 = 0.121, 1.2, 32, 0
    T = dims[0]
    U = synth.gauge_field(dims, 0.25, 3)
    g = D.dlma_load_gauge(cu(U), kappa, csw)
    V, ev = D.dlma_lap_eigs(g, nev, t0, 1, cu(synth.gaussian_start(dims, 1, 603)))
    check_modes(orc, U, t0, V[0], ev[0], 1e-10)
    xi = synth.z2_noise(dims, t0, 1, 1003)
    eta = orc.noise_sources(xi, T, t0)  # inputs from the seeded generators only
    b = torch.cat([D.dist_sources(V[0], T, t0), cu(eta)])
    opts = D.default_opts(tol=TOL, prec="mix_fp16")
    (x,), st = D.dlma_solve([g], [b], opts=opts)
    assert len(st) == 4 * nev + 4
    assert all(s["converged"] and s["relres"] <= TOL for s in st)
    A = orc.clover(U, kappa, csw)
    for i in (0, 1, 77, 4 * nev - 1):
        assert oracle_relres(orc, U, A, x[i].cpu().numpy(), b[i].cpu().numpy()) <= TOL * RES_SLACK
    # the oracle's own solve of one noise source, element by element
    want = orc.solve(U, A, eta[:1], tol=1e-12)[0][0]
    got = x[4 * nev].cpu().numpy()
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-8


def test_uneven_batch_bf16(D, orc):
    """3 x 12^3x24 (seeds 1-3), 2 x 16^3x32 (seeds 4, 5), 1 x 24^3x48 (seed 6), kappa
    cycling 0.119, 0.120, 0.121, c_sw 1.2, eps 0.25; 64 right-hand sides each
    (32 distillation from N = 8 modes + 32 Z2 wall sources) in one BF16 solve."""
    shapes = [(24, 12, 12, 12)] * 3 + [(32, 16, 16, 16)] * 2 + [(48, 24, 24, 24)]
    kappas = [0.119, 0.120, 0.121, 0.119, 0.120, 0.121]
    nev, t0, nn = 8, 0, 8
    gs, bs, Us = [], [], []
    for i, dims in enumerate(shapes):
        seed = i + 1
        U = synth.gauge_field(dims, 0.25, seed)
        g = D.dlma_load_gauge(cu(U), kappas[i], 1.2)
        V, ev = D.dlma_lap_eigs(g, nev, t0, 1, cu(synth.gaussian_start(dims, 1, 600 + seed)))
        eta = D.noise_sources(cu(synth.z2_noise(dims, t0, nn, 1000 + seed)), dims[0], t0)
        bs.append(torch.cat([D.dist_sources(V[0], dims[0], t0), eta]))
        gs.append(g)
        Us.append(U)
    opts = D.default_opts(tol=TOL, prec="mix_bf16")
    xs, st = D.dlma_solve(gs, bs, opts=opts)
    assert len(st) == 64 * len(shapes)
    assert all(s["converged"] and s["relres"] <= TOL for s in st)
    for i, (U, b, x) in enumerate(zip(Us, bs, xs)):
        A = orc.clover(U, kappas[i], 1.2)
        for r in (0, 4 * nev):
            assert oracle_relres(orc, U, A, x[r].cpu().numpy(), b[r].cpu().numpy()) <= TOL * RES_SLACK, (i, r)


def test_headline_launch_configuration(D, orc):
    """24^3 x 48, eps 0.25, seed 6, kappa 0.121, c_sw 1.2, t' = 0: 128 distillation +
    32 eta + 32 (1 - box) eta, mixed FP16, 2 right-hand sides per thread (the
    benchmark's configuration); sampled solutions under the oracle's operator."""
    dims = (48, 24, 24, 24)
    kappa, csw, nev, t0, nn = 0.121, 1.2, 32, 0, 8
    T = dims[0]
    U = synth.gauge_field(dims, 0.25, 6)
    g = D.dlma_load_gauge(cu(U), kappa, csw)
    v0 = cu(synth.gaussian_start(dims, 1, 606))
    VL, evL = D.dlma_lap_eigs(g, nev, t0, 1, v0)
    check_modes(orc, U, t0, VL[0], evL[0], 1e-10)
    # the benchmark takes the modes with the block variant: same eigenvalues, and the
    # same vectors where an eigenvalue is isolated (phase rule), else the same space
    V, ev = D.dlma_lap_eigs(g, nev, t0, 1, v0, block_size=min(64, nev + 24))
    check_modes(orc, U, t0, V[0], ev[0], 1e-10)
    assert np.max(np.abs(ev - evL)) < 1e-11
    O = (VL[0].reshape(nev, -1).conj() @ V[0].reshape(nev, -1).T).cpu().numpy()  # overlaps of the two bases
    assert np.max(np.abs(O.conj().T @ O - np.eye(nev))) < 1e-8  # unitary: the same space
    del VL
    eta = D.noise_sources(cu(synth.z2_noise(dims, t0, nn, 1006)), T, t0)
    b = torch.cat([D.dist_sources(V[0], T, t0), eta, D.dlma_project(g, t0, V[0], eta, 1)])
    del eta
    # one defect-correction pass brings every right-hand side to the inner tolerance's
    # level (2e-3): a corrupted store in the solution update of some RHS shows as
    # several times worse residuals there and extra passes.  CGNE's passes are uniform
    # (1.4e-3 .. 3.6e-3 measured); BiCGStab's spread more (up to 1.1e-2 measured).
    for solver, bound in ((0, 5e-3), (1, 3e-2)):
        opts1 = D.default_opts(tol=TOL, prec="mix_fp16", rhs_block=2, max_outer=1, inner_solver=solver)
        _, st1 = D.dlma_solve([g], [b], opts=opts1, allow_notconv=True)
        worst = max(s["relres"] for s in st1)
        print("one pass, inner solver %d: worst relres %.3e" % (solver, worst), flush=True)
        assert worst <= bound, (solver, worst)
    opts = D.default_opts(tol=TOL, prec="mix_fp16", rhs_block=2)
    (x,), st = D.dlma_solve([g], [b], opts=opts)
    assert len(st) == 192
    assert all(s["converged"] and s["relres"] <= TOL for s in st)
    assert max(s["outer"] for s in st) <= 5, sorted(set(s["outer"] for s in st))
    A = orc.clover(U, kappa, csw)
    for i in (0, 63, 127, 128, 159, 160, 191):
        assert oracle_relres(orc, U, A, x[i].cpu().numpy(), b[i].cpu().numpy()) <= TOL * RES_SLACK, i
    # the projected sources carry no component along V(t')
    P = D.dlma_project(g, t0, V[0], b[160:164], 0)
    assert float(P.abs().max()) < 1e-12


def test_grad_32x64_fp64(D, orc):
    """32^3 x 64, eps 0.2, kappa 0.1215, c_sw 1.3, FP64: d/dm0 of a weighted
    pseudoscalar sink sum of one spin-diluted wall source, by the adjoint solve,
    against central finite differences (dm0 = 1e-4, solves to 1e-12)."""
    dims = (64, 32, 32, 32)
    kappa, csw = 0.1215, 1.3
    T = dims[0]
    U = synth.gauge_field(dims, 0.2, 5)
    g = D.dlma_load_gauge(cu(U), kappa, csw)
    b = D.noise_sources(cu(synth.z2_noise(dims, 0, 1, 1005)), T, 0)[:1].contiguous()
    m0v = 1 / (2 * kappa) - 4
    m0 = torch.tensor(m0v, dtype=torch.float64, requires_grad=True)
    opts = D.default_opts(tol=1e-12, prec="fp64")
    w = torch.linspace(0.5, 1.5, T, dtype=torch.float64, device="cuda")

    def corr(x):
        return (x.abs() ** 2).reshape(x.shape[0], T, -1).sum(dim=(0, 2))

    x = D.dirac_solve(b, m0, g, opts)
    L = (w * corr(x)).sum()
    L.backward()
    A = orc.clover(U, kappa, csw)
    assert oracle_relres(orc, U, A, x[0].detach().cpu().numpy(), b[0].cpu().numpy()) <= 1e-12 * RES_SLACK
    h = 1e-4

    def loss(mv):
        with torch.no_grad():
            xx = D.dirac_solve(b, torch.tensor(mv, dtype=torch.float64), g, opts)
            return float((w * corr(xx)).sum())

    fd = (loss(m0v + h) - loss(m0v - h)) / (2 * h)
    assert abs(m0.grad.item() - fd) <= 1e-6 * abs(fd), (m0.grad.item(), fd)
