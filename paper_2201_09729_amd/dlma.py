"""Python binding of libdlma.so (argument marshalling only).

Every function has the name of the C entry point it calls (include/dlma.h) and
takes torch tensors that live on the GPU; device pointers and torch's current
HIP stream are passed through ctypes.  All computation happens in the library's
HIP kernels.  There is no fallback: if the library is missing or fails to load,
every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdlma.so")

DLMA_OK = 0
DLMA_EINVAL = -1
DLMA_ENOMEM = -2
DLMA_EHIP = -3
DLMA_ENOTCONV = -4
DLMA_ENAN = -5
DLMA_EUNSUPPORTED = -6

PREC = {"fp64": 0, "mix_fp32": 1, "mix_fp16": 2, "mix_bf16": 3}
NPARTS = 7
PART_NAMES = ("QQ_est", "PQ_est", "QP_est", "PP_est", "11_est", "PP_exact", "QP_exact")
GAMMA_NAMES = ("PS", "V")


class DlmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("dlma error %d: %s" % (code, msg))
        self.code = code


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("max_outer", ctypes.c_int),
                ("prec", ctypes.c_int), ("inner_tol", ctypes.c_double), ("rhs_block", ctypes.c_int),
                ("use_x0", ctypes.c_int), ("graph_iters", ctypes.c_int), ("check_every", ctypes.c_int),
                ("dagger", ctypes.c_int), ("lds_window", ctypes.c_int), ("inner_solver", ctypes.c_int)]


class SolveStat(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int), ("inner_iters", ctypes.c_int), ("relres", ctypes.c_double),
                ("converged", ctypes.c_int)]


class RhsSet(ctypes.Structure):
    _fields_ = [("b", ctypes.c_void_p), ("x", ctypes.c_void_p), ("nrhs", ctypes.c_int)]


class EigOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_basis", ctypes.c_int), ("check_every", ctypes.c_int),
                ("cheb_degree", ctypes.c_int), ("restart_basis", ctypes.c_int), ("restart_keep", ctypes.c_int),
                ("max_restarts", ctypes.c_int), ("block_size", ctypes.c_int), ("block_iters", ctypes.c_int)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdlma.so once; raises if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libdlma.so not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "dlma_version": ([], ctypes.c_char_p),
        "dlma_release_cache": ([], I),
        "dlma_last_error": ([], ctypes.c_char_p),
        "dlma_load_gauge": ([P, P, D, D, P, P], I),
        "dlma_set_mass": ([P, D, P], I),
        "dlma_free_gauge": ([P], I),
        "dlma_gauge_info": ([P, P, P, P], I),
        "dlma_apply_dw": ([P, P, P, I, I, P], I),
        "dlma_apply_schur": ([P, P, P, I, I, I, I, I, I, P], I),
        "dlma_solve_opts_default": ([P], None),
        "dlma_solve": ([P, I, P, P, P, P], I),
        "dlma_lap_eigs": ([P, I, I, I, P, P, P, P, P], I),
        "dlma_project": ([P, I, I, P, P, P, I, I, P], I),
        "dlma_project_noalloc": ([P, I, I, P, P, P, I, I, P], I),
        "dlma_correlators": ([P, I, I, P, P, I, I, I, P, P, P, P], I),
        "dlma_correlators_grad": ([P, I, I, P, P, I, I, I, P, P, P, P, P, P, P], I),
        "dlma_dot": ([P, P, ctypes.c_long, P, P], I),
        "dlma_profile_enable": ([I], I),
        "dlma_profile_reset": ([], I),
        "dlma_profile_read": ([I, P, P, P], I),
        "dlma_bench_schur": ([P, I, I, I, I, P, P, P], I),
        "dlma_bench_copy": ([ctypes.c_long, I, P, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc, allow=()):
    if rc != DLMA_OK and rc not in allow:
        msg = load_library().dlma_last_error()
        raise DlmaError(rc, msg.decode() if msg else "")
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype=torch.complex128) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if t.dtype != dtype:
        raise ValueError("tensor must be %s" % dtype)
    return t.contiguous()


def dlma_release_cache() -> None:
    """Free the device memory the library caches between calls (synchronises the device)."""
    _check(load_library().dlma_release_cache())


def dlma_version() -> str:
    return load_library().dlma_version().decode()


class Gauge:
    """Owns a dlma_gauge_t handle (freed with dlma_free_gauge)."""

    def __init__(self, handle, dims, kappa, csw):
        self.h = ctypes.c_void_p(handle)
        self.dims = tuple(dims)
        self.kappa = kappa
        self.csw = csw

    def close(self):
        if self.h is not None and self.h.value:
            load_library().dlma_free_gauge(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dlma_load_gauge(U: torch.Tensor, kappa: float, csw: float) -> Gauge:
    """U: complex128 [T][Z][Y][X][4][3][3] on the GPU."""
    U = _dev(U)
    if U.dim() != 7 or tuple(U.shape[4:]) != (4, 3, 3):
        raise ValueError("gauge must have shape [T,Z,Y,X,4,3,3]")
    dims = (ctypes.c_int * 4)(*[int(d) for d in U.shape[:4]])
    h = ctypes.c_void_p()
    _check(load_library().dlma_load_gauge(dims, ctypes.c_void_p(U.data_ptr()), float(kappa), float(csw),
                                          _stream(), ctypes.byref(h)))
    return Gauge(h.value, U.shape[:4], kappa, csw)


def dlma_set_mass(g: Gauge, kappa: float) -> None:
    _check(load_library().dlma_set_mass(g.h, float(kappa), _stream()))
    g.kappa = kappa


def dlma_apply_dw(g: Gauge, x: torch.Tensor, dagger: bool = False) -> torch.Tensor:
    """D x or D^dag x for x of shape [n][T][Z][Y][X][4][3] (complex128, GPU)."""
    x = _dev(x)
    out = torch.empty_like(x)
    n = x.shape[0]
    _check(load_library().dlma_apply_dw(g.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        int(n), int(bool(dagger)), _stream()))
    return out


def dlma_apply_schur(g: Gauge, x: torch.Tensor, dagger: bool = False, prec="mix_fp16", rhs_block: int = 0,
                     super_group: int = 0, lds_window: bool = True) -> torch.Tensor:
    """Dhat x_e (or Dhat^dag x_e) through the solver's inner stencils of precision prec,
    x of shape [n][T][Z][Y][X][4][3] (complex128, GPU); odd sites of the result are 0."""
    x = _dev(x)
    out = torch.empty_like(x)
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    _check(load_library().dlma_apply_schur(g.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           int(x.shape[0]), int(bool(dagger)), p, int(rhs_block), int(super_group),
                                           int(bool(lds_window)), _stream()))
    return out


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load_library().dlma_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PREC[v]
        setattr(o, k, v)
    return o


def dlma_solve(gauges, bs, xs=None, opts: SolveOpts | None = None, allow_notconv: bool = False):
    """Solve D x = b for lists of gauges and source tensors [n][T][Z][Y][X][4][3].

    Returns (list of solution tensors, list of per-RHS stat dicts)."""
    if isinstance(gauges, Gauge):
        gauges, bs = [gauges], [bs]
        if xs is not None:
            xs = [xs]
    opts = opts or default_opts()
    bs = [_dev(b) for b in bs]
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    else:
        xs = [_dev(x) for x in xs]
    ng = len(gauges)
    garr = (ctypes.c_void_p * ng)(*[g.h.value for g in gauges])
    sets = (RhsSet * ng)()
    total = 0
    for i in range(ng):
        sets[i].b = bs[i].data_ptr()
        sets[i].x = xs[i].data_ptr()
        sets[i].nrhs = int(bs[i].shape[0])
        total += int(bs[i].shape[0])
    stats = (SolveStat * max(1, total))()
    rc = load_library().dlma_solve(garr, ng, sets, ctypes.byref(opts), stats, _stream())
    _check(rc, allow=(DLMA_ENOTCONV,) if allow_notconv else ())
    st = [dict(outer=s.outer, inner_iters=s.inner_iters, relres=s.relres, converged=bool(s.converged))
          for s in stats[:total]]
    return xs, st


def dlma_lap_eigs(g: Gauge, nev: int, t0: int, nt: int, v0: torch.Tensor, tol: float = 1e-10,
                  max_basis: int = 0, check_every: int = 0, cheb_degree: int = 0, restart_basis: int = 0,
                  restart_keep: int = 0, max_restarts: int = 0, block_size: int = 0, block_iters: int = 0):
    """Lowest nev modes of -lap(t), t = t0..t0+nt-1; v0: [nt][Z][Y][X][3] start vectors.

    Returns (V [nt][nev][Z][Y][X][3] complex128 on the GPU, evals numpy [nt][nev])."""
    import numpy as np
    v0 = _dev(v0)
    T, Z, Y, X = g.dims
    V = torch.empty((nt, nev, Z, Y, X, 3), dtype=torch.complex128, device=v0.device)
    ev = np.zeros((nt, nev), dtype=np.float64)
    o = EigOpts(tol, max_basis, check_every, cheb_degree, restart_basis, restart_keep, max_restarts, block_size,
                block_iters)
    _check(load_library().dlma_lap_eigs(g.h, int(nev), int(t0), int(nt), ctypes.c_void_p(v0.data_ptr()),
                                        ctypes.c_void_p(V.data_ptr()), ev.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(o), _stream()))
    return V, ev


def dlma_project(g: Gauge, t: int, Vt: torch.Tensor, x: torch.Tensor, mode: int, out: torch.Tensor | None = None):
    """mode 0: box(t) x; mode 1: (1 - box(t)) x; zero off timeslice t."""
    Vt = _dev(Vt)
    x = _dev(x)
    out = torch.empty_like(x) if out is None else out
    _check(load_library().dlma_project(g.h, int(t), int(Vt.shape[0]), ctypes.c_void_p(Vt.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                       int(x.shape[0]), int(mode), _stream()))
    return out


def dlma_project_noalloc(g: Gauge, t: int, Vt: torch.Tensor, x: torch.Tensor, mode: int, out: torch.Tensor):
    """dlma_project through the allocation-free entry point: `out` is caller-allocated, the
    library allocates nothing and only enqueues work on the current stream."""
    Vt = _dev(Vt)
    x = _dev(x)
    if out.shape != x.shape or not out.is_contiguous() or out.dtype != x.dtype or not out.is_cuda:
        raise ValueError("out must be a contiguous complex128 GPU tensor shaped like x")
    _check(load_library().dlma_project_noalloc(g.h, int(t), int(Vt.shape[0]), ctypes.c_void_p(Vt.data_ptr()),
                                               ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                               int(x.shape[0]), int(mode), _stream()))
    return out


def _corr_args(Vall, phi_dist, phi, phibar):
    Vall = _dev(Vall)
    phi_dist = _dev(phi_dist) if phi_dist is not None else None
    nd = int(phi_dist.shape[0]) // 4 if phi_dist is not None else 0
    nn = 0
    pp = pb = pd = ctypes.c_void_p(0)
    if phi_dist is not None:
        pd = ctypes.c_void_p(phi_dist.data_ptr())
    if phi is not None:
        phi = _dev(phi)
        phibar = _dev(phibar)
        nn = int(phi.shape[0]) // 4
        pp = ctypes.c_void_p(phi.data_ptr())
        pb = ctypes.c_void_p(phibar.data_ptr())
    return Vall, phi_dist, phi, phibar, nd, nn, pd, pp, pb


def dlma_correlators(g: Gauge, t_src: int, Vall: torch.Tensor, phi_dist: torch.Tensor,
                     phi: torch.Tensor | None = None, phibar: torch.Tensor | None = None, ndil: int = 1):
    """Returns {gamma: {part: complex numpy [T]}} (see dlma.h for the parts).

    phi_dist: solutions for the distillation sources (any number of 4-spin groups);
    phi, phibar: solutions for the sources of noise_sources (ndil = dilution_size of its scheme)."""
    C = dlma_correlators_array(g, t_src, Vall, phi_dist, phi, phibar, ndil)
    Cc = C[..., 0] + 1j * C[..., 1]
    return {GAMMA_NAMES[gi]: {PART_NAMES[p]: Cc[gi, p] for p in range(NPARTS)} for gi in range(2)}


def dlma_correlators_array(g: Gauge, t_src: int, Vall, phi_dist, phi=None, phibar=None, ndil: int = 1):
    """dlma_correlators as the raw host array double[2][NPARTS][T][2] (re, im)."""
    import numpy as np
    Vall, phi_dist, phi, phibar, nd, nn, pd, pp, pb = _corr_args(Vall, phi_dist, phi, phibar)
    C = np.zeros((2, NPARTS, g.dims[0], 2), dtype=np.float64)
    _check(load_library().dlma_correlators(g.h, int(t_src), int(Vall.shape[1]), ctypes.c_void_p(Vall.data_ptr()),
                                           pd, nd, nn, int(ndil), pp, pb, C.ctypes.data_as(ctypes.c_void_p), _stream()))
    return C


def dlma_correlators_grad(g: Gauge, t_src: int, Vall, phi_dist, phi, phibar, G, ndil: int = 1):
    """Gradient fields (grad_dist, grad_phi, grad_phibar) of a real loss whose gradient with
    respect to the correlator pieces is G (host double [2][NPARTS][T][2], dL/dRe C + i dL/dIm C)."""
    import numpy as np
    Vall, phi_dist, phi, phibar, nd, nn, pd, pp, pb = _corr_args(Vall, phi_dist, phi, phibar)
    G = np.ascontiguousarray(G, dtype=np.float64)
    if G.shape != (2, NPARTS, g.dims[0], 2):
        raise ValueError("G must be [2][%d][T][2]" % NPARTS)
    gd = torch.empty_like(phi_dist) if phi_dist is not None else None
    g1 = torch.empty_like(phi) if phi is not None else None
    gq = torch.empty_like(phibar) if phibar is not None else None
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)  # noqa: E731
    _check(load_library().dlma_correlators_grad(g.h, int(t_src), int(Vall.shape[1]), ctypes.c_void_p(Vall.data_ptr()),
                                                pd, nd, nn, int(ndil), pp, pb, G.ctypes.data_as(ctypes.c_void_p),
                                                ptr(gd), ptr(g1), ptr(gq), _stream()))
    return gd, g1, gq


class Correlators(torch.autograd.Function):
    """C = the correlator pieces of dlma_correlators as a complex128 CPU tensor
    [2 (PS, V)][NPARTS][T] (time index Delta), differentiable in the solution fields:
    the backward is dlma_correlators_grad, the hand-written adjoint of the contractions."""

    @staticmethod
    def forward(ctx, phi_dist, phi, phibar, gauge, t_src, Vall, ndil):
        import numpy as np
        det = lambda t: t.detach() if t is not None else None  # noqa: E731
        C = dlma_correlators_array(gauge, t_src, Vall, det(phi_dist), det(phi), det(phibar), ndil)
        ctx.save_for_backward(phi_dist, phi, phibar)
        ctx.gauge, ctx.t_src, ctx.Vall, ctx.ndil = gauge, t_src, Vall, ndil
        return torch.from_numpy(np.ascontiguousarray(C[..., 0] + 1j * C[..., 1]))

    @staticmethod
    def backward(ctx, grad_C):
        import numpy as np
        phi_dist, phi, phibar = ctx.saved_tensors
        Gc = grad_C.detach().cpu().numpy().astype(np.complex128)
        G = np.stack([Gc.real, Gc.imag], axis=-1)
        gd, g1, gq = dlma_correlators_grad(ctx.gauge, ctx.t_src, ctx.Vall, phi_dist, phi, phibar, G, ctx.ndil)
        return gd, g1, gq, None, None, None, None


def correlators(phi_dist, phi, phibar, gauge: Gauge, t_src: int, Vall: torch.Tensor, ndil: int = 1) -> torch.Tensor:
    """Differentiable correlator pieces (see Correlators).  phi_dist, or phi and phibar
    together, may be None: every piece is a sum over source groups, so the solutions can
    be contracted in batches and the results added."""
    return Correlators.apply(phi_dist, phi, phibar, gauge, int(t_src), Vall, int(ndil))


def dlma_profile_enable(on: bool = True):
    _check(load_library().dlma_profile_enable(int(bool(on))))


def dlma_profile_reset():
    _check(load_library().dlma_profile_reset())


def dlma_profile_read(kclass: int):
    n = ctypes.c_longlong()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(load_library().dlma_profile_read(int(kclass), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


def dlma_bench_schur(g: Gauge, prec, nrhs: int, rhs_block: int = 0, napply: int = 20):
    if isinstance(prec, str):
        prec = PREC[prec]
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(load_library().dlma_bench_schur(g.h, int(prec), int(nrhs), int(rhs_block), int(napply),
                                           ctypes.byref(ms), ctypes.byref(by), _stream()))
    return ms.value, by.value


# ---------------------------------------------------------------- source placement (data movement only)

def dist_sources(Vt: torch.Tensor, T: int, t0: int) -> torch.Tensor:
    """Spin-diluted distillation sources v^(k)(t0) x e_s on timeslice t0, index k*4 + s.

    Vt: [nev][Z][Y][X][3] on the GPU.  Returns [4 nev][T][Z][Y][X][4][3]."""
    Vt = _dev(Vt)
    nev = Vt.shape[0]
    out = torch.zeros((nev * 4, T) + tuple(Vt.shape[1:4]) + (4, 3), dtype=torch.complex128, device=Vt.device)
    for s in range(4):
        out[s::4, t0, ..., s, :] = Vt
    return out


DILUTIONS = {"spin": (1, 1), "spin-colour": (3, 1), "spin-eo": (1, 2), "spin-colour-eo": (3, 2)}


def dilution_size(dilution: str) -> int:
    """Dilution components per noise vector besides spin: colours x wall parities."""
    nc, npar = DILUTIONS[dilution]
    return nc * npar


def noise_sources(xi: torch.Tensor, T: int, t0: int, dilution: str = "spin") -> torch.Tensor:
    """Diluted wall noise on timeslice t0: the components P_d xi_r (colour c only and/or
    wall sites of parity p = (t0 + z + y + x) mod 2 only; d = c * npar + p), each
    spin-diluted: P_d xi_r x e_s at index (r * ndil + d) * 4 + s.  xi: [N_r][Z][Y][X][3]."""
    if not xi.is_cuda:
        raise ValueError("tensor must be on the GPU")
    nc, npar = DILUTIONS[dilution]
    ndil = nc * npar
    nn = xi.shape[0]
    Z, Y, X = xi.shape[1:4]
    xi = xi.to(torch.complex128)
    out = torch.zeros((nn * ndil * 4, T, Z, Y, X, 4, 3), dtype=torch.complex128, device=xi.device)
    idx = torch.arange(Z * Y * X, device=xi.device)
    par = ((t0 + idx // (Y * X) + (idx // X) % Y + idx % X) % 2).reshape(Z, Y, X)
    for c in range(nc):
        for p in range(npar):
            comp = torch.zeros_like(xi)
            cols = slice(c, c + 1) if nc == 3 else slice(0, 3)
            comp[..., cols] = xi[..., cols]
            if npar == 2:
                comp[:, par != p] = 0
            d = c * npar + p
            for s in range(4):
                out[(d * 4 + s)::(ndil * 4), t0, ..., s, :] = comp
    return out


def dlma_dot(a: torch.Tensor, b: torch.Tensor) -> complex:
    """<a, b> = sum conj(a) b over all elements (complex128 GPU tensors of equal size)."""
    import numpy as np
    a = _dev(a)
    b = _dev(b)
    if a.numel() != b.numel():
        raise ValueError("size mismatch")
    out = np.zeros(2, dtype=np.float64)
    _check(load_library().dlma_dot(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), int(a.numel()),
                                   out.ctypes.data_as(ctypes.c_void_p), _stream()))
    return complex(out[0], out[1])


# ---------------------------------------------------------------- differentiation

def kappa_of_m0(m0: float) -> float:
    return 1.0 / (2.0 * m0 + 8.0)


class DiracSolve(torch.autograd.Function):
    """x = D(m0)^-1 b with the hand-written adjoint as backward.

    forward:  dlma_solve (the configured precision; FP64 defect correction to tol)
    backward: grad_b  = D^-dag grad_x = g5 D^-1 g5 grad_x  (dlma_solve with dagger = 1)
              grad_m0 = -Re <grad_b, x>                      (dlma_dot), since dD/dm0 = 1
    in PyTorch's convention for complex tensors (the gradient of a real loss L with
    respect to z is dL/dRe z + i dL/dIm z)."""

    @staticmethod
    def forward(ctx, b, m0, gauge, opts):
        kappa = kappa_of_m0(float(m0))
        if gauge.kappa != kappa:
            dlma_set_mass(gauge, kappa)
        (x,), _ = dlma_solve([gauge], [b.detach()], opts=opts)
        ctx.save_for_backward(x)
        ctx.gauge = gauge
        ctx.opts = opts
        ctx.kappa = kappa
        return x

    @staticmethod
    def backward(ctx, grad_x):
        (x,) = ctx.saved_tensors
        g = ctx.gauge
        if g.kappa != ctx.kappa:
            dlma_set_mass(g, ctx.kappa)
        o = SolveOpts()
        ctypes.memmove(ctypes.byref(o), ctypes.byref(ctx.opts), ctypes.sizeof(SolveOpts))
        o.dagger = 1
        o.use_x0 = 0
        (gb,), _ = dlma_solve([g], [grad_x.contiguous()], opts=o)
        gm = -dlma_dot(gb, x).real
        return gb, torch.tensor(gm, dtype=torch.float64, device=x.device), None, None


def dirac_solve(b: torch.Tensor, m0: torch.Tensor, gauge: Gauge, opts: SolveOpts | None = None) -> torch.Tensor:
    """Differentiable solve; m0 is a 0-dim float64 tensor (bare mass, m0 = 1/(2 kappa) - 4)."""
    return DiracSolve.apply(b, m0, gauge, opts or default_opts())


def dlma_bench_copy(nbytes: int = 1 << 31, reps: int = 10) -> float:
    """Measured stream bandwidth in GB/s (read + write) of the library's copy kernel."""
    ms = ctypes.c_double()
    _check(load_library().dlma_bench_copy(int(nbytes), int(reps), ctypes.byref(ms), _stream()))
    return 2.0 * nbytes / (ms.value * 1e-3) / 1e9
