"""GPU parity of the solver's inner operator against the oracle.

dlma_apply_schur runs the solver's own stencil kernels (K1: y = A_oo^-1 D_oe x,
K2: A_ee x - D_eo y) in each storage precision and launch shape.  The oracle's
even-odd reduced operator is computed in FP64 from the full operator.

Tolerance, in units u of roundoff of the storage precision: 4u relative per
right-hand side, and 8u site by site relative to the largest site.  Each output
component sums terms that carry a few independent storage roundings in series:
- the input x or the intermediate y;
- a link or clover entry;
- the FP16 spin projection;
- the final store.
Accumulation is FP32.  Independent roundings add in quadrature, to about 2u,
plus mild cancellation between A_ee x and the hopping term.  Measured on these
cases: 0.8u (FP16, BF16) and 1.4u (FP32) relative, at most 2.6u per site.
FP64 storage: 1e-14, for summation order only.

Launch shapes with the same right-hand sides per thread run the same kernel, so
their results must agree bit for bit:
- every super-group order;
- the FP16 stencils with and without their LDS window of neighbours.
"""
import numpy as np
import pytest

from paper_2201_09729_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"fp64": 1e-14, "mix_fp32": 4 * 2.0**-24, "mix_fp16": 4 * 2.0**-11, "mix_bf16": 4 * 2.0**-8}

# (dims, eps, seed, kappa, csw)
LATTICES = [
    # 360 sites per timeslice and parity: two full 128-site blocks and a ragged one; X/2 = 6
    ((4, 6, 10, 12), 0.25, 11, 0.121, 1.2),
    # 32 sites per timeslice: one block whose second wave has no site
    ((8, 4, 4, 4), 0.3, 12, 0.120, 1.0),
    # X/2 = 10, five full blocks per timeslice
    ((4, 8, 8, 20), 0.25, 13, 0.121, 1.2),
]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def D():
    _need_gpu()
    from paper_2201_09729_amd import dlma
    dlma.load_library()
    return dlma


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _errors(y, ref):
    n = y.shape[0]
    d = (y - ref).reshape(n, -1)
    r = ref.reshape(n, -1)
    rel = np.linalg.norm(d, axis=1) / np.linalg.norm(r, axis=1)
    ds = np.linalg.norm((y - ref).reshape(n, -1, 12), axis=2)
    rs = np.linalg.norm(ref.reshape(n, -1, 12), axis=2)
    site = ds.max(axis=1) / rs.max(axis=1)
    return rel.max(), site.max()


@pytest.mark.parametrize("dagger", [False, True])
@pytest.mark.parametrize("case", LATTICES, ids=["4x6x10x12", "8x4x4x4", "4x8x8x20"])
def test_schur_operator_matches_oracle(D, orc, case, dagger):
    dims, eps, seed, kappa, csw = case
    nrhs = 5  # ragged for 2, 3 and 4 right-hand sides per thread
    U = synth.gauge_field(dims, eps, seed)
    x = synth.random_spinor(dims, nrhs, seed + 50)
    ref = orc.schur(U, orc.clover(U, kappa, csw), x, dagger=dagger)
    odd = orc.even_mask(dims) == 0
    g = D.dlma_load_gauge(cu(U), kappa, csw)
    xd = cu(x)
    for prec, tol in TOL.items():
        outs = {}
        for nb in (1, 2, 3, 4):
            for sg in (0, 1, 2):
                for win in ((True, False) if prec == "mix_fp16" else (True,)):
                    print("schur", dims, "dagger", dagger, prec, "nb", nb, "sg", sg, "window", win, flush=True)
                    y = D.dlma_apply_schur(g, xd, dagger, prec, nb, sg, win).cpu().numpy()
                    rel, site = _errors(y, ref)
                    print("   rel %.3e  site %.3e" % (rel, site), flush=True)
                    assert rel <= tol and site <= 2 * tol, (prec, nb, sg, win, rel, site)
                    assert not np.any(y[:, odd])
                    outs[(nb, sg, win)] = y
        for (nb, sg, win), y in outs.items():
            assert np.array_equal(y, outs[(nb, 0, True)]), (prec, nb, sg, win)
        print("schur", dims, "dagger", dagger, prec, "tuned", flush=True)
        y = D.dlma_apply_schur(g, xd, dagger, prec, 0).cpu().numpy()
        rel, site = _errors(y, ref)
        assert rel <= tol and site <= 2 * tol, (prec, "tuned", rel, site)
    g.close()


def test_schur_fullsize_fp16_window(D, orc):
    """24^3x48 at the solver's 192-RHS launch shape (2 per thread, 8 groups per
    super-group) with and without the LDS window: bit-identical results.  The oracle
    checks sampled right-hand sides through Dhat's definition on the full lattice."""
    dims = (48, 24, 24, 24)
    U = synth.gauge_field(dims, 0.25, 6)
    g = D.dlma_load_gauge(cu(U), 0.121, 1.2)
    nrhs = 192
    xd = torch.empty((nrhs,) + dims + (4, 3), dtype=torch.complex128, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(3)
    xd.real.normal_(generator=gen)
    xd.imag.normal_(generator=gen)
    print("schur fullsize window on", flush=True)
    y1 = D.dlma_apply_schur(g, xd, False, "mix_fp16", 2, 8, True)
    print("schur fullsize window off", flush=True)
    y0 = D.dlma_apply_schur(g, xd, False, "mix_fp16", 2, 8, False)
    assert torch.equal(y0, y1)
    del y0
    pick = [0, 101, 191]
    ref = orc.schur(U, orc.clover(U, 0.121, 1.2), xd[pick].cpu().numpy())
    rel, site = _errors(y1[pick].cpu().numpy(), ref)
    print("   rhs %s rel %.3e site %.3e" % (pick, rel, site), flush=True)
    assert rel <= TOL["mix_fp16"] and site <= 2 * TOL["mix_fp16"]
    g.close()
