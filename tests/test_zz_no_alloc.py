"""The allocation-free projector (dlma_project_noalloc) against dlma_project and the
oracle: bit-identical to the allocating entry point, which shares its kernels, on
two calls in a row (the second smaller, in place), including a call whose
right-hand sides pass through the fixed coefficient array in several chunks."""
import ctypes

import numpy as np
import pytest

from paper_2201_09729_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_09729_amd import dlma
    dlma.load_library()
    return dlma


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_project_noalloc_matches_project(D, orc):
    dims = (6, 4, 4, 8)
    U = synth.gauge_field(dims, 0.3, 3)
    g = D.dlma_load_gauge(cu(U), 0.120, 1.0)
    v0 = synth.gaussian_start(dims, 2, 9)
    _, V5 = orc.lap_eigs(U, 4, 5, v0[0], tol=1e-12)
    _, V3 = orc.lap_eigs(U, 1, 3, v0[1], tol=1e-12)

    # first call: nev = 5 gives 3276 right-hand sides per pass through the 65536-entry
    # coefficient array, so 3300 right-hand sides take two passes
    nr1 = 3300
    print("noalloc call 1: nev 5, nrhs", nr1, flush=True)
    gen = torch.Generator(device="cuda").manual_seed(41)
    x1 = torch.randn(nr1, *dims, 4, 3, dtype=torch.complex128, device="cuda", generator=gen)
    out1 = torch.empty_like(x1)
    D.dlma_project_noalloc(g, 4, cu(V5), x1, 1, out1)
    torch.cuda.synchronize()
    ref1 = D.dlma_project(g, 4, cu(V5), x1, 1)
    assert torch.equal(out1, ref1)
    for r in (0, 3275, 3276, nr1 - 1):  # both sides of the chunk boundary
        xr = x1[r:r + 1].cpu().numpy()
        o = orc.project(V5, xr, 4, 1)
        assert np.max(np.abs(out1[r:r + 1].cpu().numpy() - o)) < 1e-13 * np.max(np.abs(xr))

    # second call, smaller: nev = 3, 2 right-hand sides, mode 0, in place
    print("noalloc call 2: nev 3, nrhs 2, in place", flush=True)
    x2 = synth.random_spinor(dims, 2, 4)
    xt = cu(x2)
    D.dlma_project_noalloc(g, 1, cu(V3), xt, 0, xt)
    torch.cuda.synchronize()
    ref2 = D.dlma_project(g, 1, cu(V3), cu(x2), 0)
    assert torch.equal(xt, ref2)
    o2 = orc.project(V3, x2, 1, 0)
    assert np.max(np.abs(xt.cpu().numpy() - o2)) < 1e-13 * np.max(np.abs(x2))


def test_project_noalloc_rejects_oversize(D):
    """nev beyond the coefficient array's limit is an argument error, before any work."""
    dims = (4, 4, 4, 4)
    g = D.dlma_load_gauge(cu(synth.gauge_field(dims, 0.3, 1)), 0.120, 1.0)
    lib = D.load_library()
    x = torch.zeros(1, *dims, 4, 3, dtype=torch.complex128, device="cuda")
    p = ctypes.c_void_p(x.data_ptr())
    rc = lib.dlma_project_noalloc(g.h, 0, 16385, p, p, p, 1, 0, D._stream())
    assert rc == D.DLMA_EINVAL
    assert b"16384" in lib.dlma_last_error()
