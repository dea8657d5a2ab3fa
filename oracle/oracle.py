"""FP64 CPU oracle for distillation low-mode averaging (arXiv:2201.09729).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline of the benchmark may import this module.  It shares no code with the
GPU library: the Dirac operator, clover term, solver and Laplacian live in
``dirac_oracle.c`` (plain C, loaded with ctypes); the eigensolver, projector,
sources and contractions below are numpy, written from the definitions.

Paper references (sections and equations of the paper):
  * eq. (1): spatial covariant Laplacian lap(t), distillation projector
    box(t) = V(t) V(t)^dag, spin-orthogonal basis of the four-fold degenerate modes;
  * eq. (2): split C = C_rest + 2 C_mixed + C_dist by inserting 1 = (1-box) + box
    at sink and source;
  * eq. (3): one-end stochastic estimators for C_dist, C_rest and C_mixed;
  * eq. (4): the solutions phi = D^-1 eta and phibar = D^-1 (1 - box) eta;
  * Sec. 2: Laplacian eigenmodes per timeslice with no preconditioning,
    O(a)-improved Wilson fermions, periodic boundary conditions, wall sources.

Readings where the paper is silent (the Dirac operator, gamma basis, clover
normalisation, noise distribution, which traces are reported) follow the
conventions stated in ``dirac_oracle.c`` and in the docstrings below.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import scipy.linalg

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i = ctypes.c_int
        dbl = ctypes.c_double
        lib.orc_gamma.argtypes = [P]
        lib.orc_field_strength.argtypes = [P, P, P]
        lib.orc_clover.argtypes = [P, P, dbl, dbl, P]
        lib.orc_dirac.argtypes = [P, P, P, P, P, i]
        lib.orc_dirac_dag.argtypes = [P, P, P, P, P, i]
        lib.orc_cgls.argtypes = [P, P, P, P, P, dbl, i, P, P]
        lib.orc_cgls.restype = i
        lib.orc_cgls_fixed.argtypes = [P, P, P, P, P, i]
        lib.orc_cgls_fixed.restype = dbl
        lib.orc_laplacian.argtypes = [P, P, i, P, P, i]
        lib.orc_num_threads.restype = i
        _lib = lib
    return _lib


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _dims(U):
    d = np.ascontiguousarray(np.array(U.shape[:4], dtype=np.int32))
    return d


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ---------------------------------------------------------------- conventions

def m0_from_kappa(kappa: float) -> float:
    """Bare mass of the Wilson operator: kappa = 1/(2 m0 + 8)."""
    return 1.0 / (2.0 * kappa) - 4.0


def gammas() -> np.ndarray:
    """[5][4][4]: gamma_0..gamma_3 (t, x, y, z) and gamma_5, as used by the C oracle."""
    out = np.zeros((5, 4, 4), dtype=np.complex128)
    _load().orc_gamma(_ptr(out))
    return out


# ---------------------------------------------------------------- Dirac operator

def field_strength(U) -> np.ndarray:
    """Fhat_{mu nu}(x) = (Q - Q^dag)/8 for the planes (01,02,03,12,13,23): [V][6][3][3]."""
    U = _c(U)
    V = int(np.prod(U.shape[:4]))
    F = np.zeros((V, 6, 3, 3), dtype=np.complex128)
    _load().orc_field_strength(_ptr(_dims(U)), _ptr(U), _ptr(F))
    return F


def clover(U, kappa: float, csw: float) -> np.ndarray:
    """A(x) = (4+m0) + csw (i/2) sum_{mu<nu} sigma_{mu nu} x Fhat_{mu nu}: [V][12][12]."""
    U = _c(U)
    V = int(np.prod(U.shape[:4]))
    A = np.zeros((V, 12, 12), dtype=np.complex128)
    _load().orc_clover(_ptr(_dims(U)), _ptr(U), float(kappa), float(csw), _ptr(A))
    return A


def dirac(U, A, psi, dagger: bool = False) -> np.ndarray:
    """D psi (or D^dag psi = g5 D g5 psi) for psi of shape [n][T][Z][Y][X][4][3]."""
    U = _c(U)
    psi = _c(psi)
    out = np.zeros_like(psi)
    n = psi.shape[0]
    f = _load().orc_dirac_dag if dagger else _load().orc_dirac
    f(_ptr(_dims(U)), _ptr(U), _ptr(_c(A)), _ptr(psi), _ptr(out), int(n))
    return out


def even_mask(dims) -> np.ndarray:
    """[T][Z][Y][X]: 1.0 on even sites (t + z + y + x even), 0.0 on odd sites."""
    T, Z, Y, X = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return ((t + z + y + x) % 2 == 0).astype(np.float64)


def schur(U, A, psi, dagger: bool = False) -> np.ndarray:
    """Even-odd reduced operator on the even sites of psi [n][T][Z][Y][X][4][3]:
        Dhat psi_e = D_ee psi_e - D_eo D_oo^-1 D_oe psi_e,
    the Schur complement of D's blocks between even and odd sites.  The hopping term
    of D only links sites of opposite parity, so D_ee = A_ee and D_oo = A_oo.  With
    dagger, the same complement of D^dag (whose odd-odd block is A_oo^dag).
    Odd sites of psi are ignored; odd sites of the result are zero.

    The paper needs only D^-1 (Sec. 2, eq. (4)); this is the definition of the
    reduced system that an even-odd preconditioned solver iterates on (a reading:
    the paper does not fix the solver), written out from the full operator."""
    psi = _c(psi)
    n, T, Z, Y, X = psi.shape[:5]
    ev = even_mask((T, Z, Y, X))[None, :, :, :, :, None, None]
    od = 1.0 - ev
    xe = psi * ev
    dx = dirac(U, A, xe, dagger)              # A_ee x_e on even sites, D_oe x_e on odd sites
    Ainv = np.linalg.inv(_c(A).reshape(T, Z, Y, X, 12, 12))
    if dagger:
        Ainv = np.conj(np.swapaxes(Ainv, -1, -2))   # (A^dag)^-1
    y = (dx * od).reshape(n, T, Z, Y, X, 12)
    z = np.einsum("tzyxab,ntzyxb->ntzyxa", Ainv, y).reshape(psi.shape) * od   # D_oo^-1 D_oe x_e
    return (dx - dirac(U, A, z, dagger)) * ev


def solve(U, A, b, tol: float = 1e-10, maxiter: int = 20000, x0=None):
    """x = D^-1 b per right-hand side by CG on the normal equations (CGLS).

    Returns (x, iterations[n], true relative residual[n], converged[n]).
    """
    U = _c(U)
    A = _c(A)
    b = _c(b)
    x = np.zeros_like(b) if x0 is None else _c(x0).copy()
    n = b.shape[0]
    its = np.zeros(n, dtype=np.int32)
    res = np.zeros(n)
    conv = np.zeros(n, dtype=bool)
    d = _dims(U)
    for r in range(n):
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0)
        xr = np.ascontiguousarray(x[r])
        br = np.ascontiguousarray(b[r])
        st = _load().orc_cgls(_ptr(d), _ptr(U), _ptr(A), _ptr(br), _ptr(xr), float(tol),
                              int(maxiter), ctypes.byref(it), ctypes.byref(rr))
        x[r] = xr
        its[r] = it.value
        res[r] = rr.value
        conv[r] = st == 0
    return x, its, res, conv


def cgls_fixed(U, A, b, niter: int):
    """Run exactly niter CGLS iterations on one right-hand side [T][Z][Y][X][4][3] from x=0.

    Returns (x, recursion relative residual).  Used to time the oracle."""
    U = _c(U)
    b = _c(b)
    x = np.zeros_like(b)
    r = _load().orc_cgls_fixed(_ptr(_dims(U)), _ptr(U), _ptr(_c(A)), _ptr(b), _ptr(x), int(niter))
    return x, float(r)


def true_residual(U, A, x, b) -> np.ndarray:
    """|b - D x| / |b| per right-hand side."""
    r = _c(b) - dirac(U, A, x)
    axes = tuple(range(1, r.ndim))
    return np.sqrt(np.sum(np.abs(r) ** 2, axis=axes) / np.sum(np.abs(b) ** 2, axis=axes))


# ---------------------------------------------------------------- Laplacian (eq. 1)

def laplacian(U, t: int, v) -> np.ndarray:
    """lap(t) v for colour vectors v of shape [n][Z][Y][X][3] on timeslice t."""
    U = _c(U)
    v = _c(v)
    out = np.zeros_like(v)
    _load().orc_laplacian(_ptr(_dims(U)), _ptr(U), int(t), _ptr(v), _ptr(out), int(v.shape[0]))
    return out


def phase_fix(vecs: np.ndarray) -> np.ndarray:
    """Make the component of largest modulus of each vector real and positive.

    Ties (moduli within 1e-10 of the maximum) go to the lowest flat index."""
    out = np.array(vecs, dtype=np.complex128, copy=True)
    flat = out.reshape(out.shape[0], -1)
    for k in range(flat.shape[0]):
        a = np.abs(flat[k])
        i = int(np.nonzero(a >= a.max() - 1e-10)[0][0])
        flat[k] *= np.conj(flat[k, i]) / a[i]
    return out


def lap_eigs(U, t: int, nev: int, v0, tol: float = 1e-10, maxm: int | None = None,
             check_every: int = 5):
    """Lowest nev eigenpairs of -lap(t) by plain Lanczos with full re-orthogonalisation.

    The operator -lap(t) is Hermitian with spectrum in [0, 12]; the low-lying
    modes of the paper (Sec. 2) are those with lap(t) eigenvalue closest to 0.
    Each step: w = -lap q_j; alpha_j = <q_j, w>; w -= alpha_j q_j + beta_{j-1} q_{j-1};
    two passes of classical Gram-Schmidt against all previous q; beta_j = |w|.
    Convergence: |beta_m s_{m,i}| <= tol * 12 for the nev smallest Ritz values
    (s = eigenvectors of the tridiagonal matrix, solved with LAPACK via scipy).

    Returns (evals of lap(t), descending (<= 0), vectors [nev][Z][Y][X][3]) with the
    phase convention of phase_fix.
    """
    U = _c(U)
    shp = tuple(U.shape[1:4]) + (3,)
    n = int(np.prod(shp))
    if maxm is None:
        maxm = n
    maxm = min(maxm, n)
    Q = np.zeros((maxm + 1, n), dtype=np.complex128)
    q = np.asarray(v0, dtype=np.complex128).reshape(n)
    Q[0] = q / np.linalg.norm(q)
    alpha, beta = [], []
    m = 0
    S = theta = None
    for j in range(maxm):
        w = -laplacian(U, t, Q[j].reshape((1,) + shp)).reshape(n)
        a = float(np.vdot(Q[j], w).real)
        w = w - a * Q[j]
        if j > 0:
            w = w - beta[-1] * Q[j - 1]
        for _ in range(2):
            w = w - Q[: j + 1].T @ (np.conj(Q[: j + 1]) @ w)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        m = j + 1
        exhausted = b < 1e-13
        if m >= nev and (m % check_every == 0 or exhausted or m == maxm):
            theta, S = scipy.linalg.eigh_tridiagonal(np.array(alpha), np.array(beta[:-1]))
            res = np.abs(b * S[-1, :nev])
            if exhausted or np.all(res <= tol * 12.0):
                break
        if exhausted:
            break
        Q[j + 1] = w / b
    if S is None or S.shape[0] != m:
        theta, S = scipy.linalg.eigh_tridiagonal(np.array(alpha), np.array(beta[:-1]))
    Y = (Q[:m].T @ S[:, :nev]).T  # [nev][n]
    # re-orthonormalise (Ritz vectors are orthonormal up to rounding)
    qq, rr = np.linalg.qr(Y.T)
    Y = (qq * np.sign(np.diagonal(rr).real)[None, :]).T
    vecs = phase_fix(Y.reshape((nev,) + shp))
    return -theta[:nev], vecs


# ---------------------------------------------------------------- projector and sources

def _tcoef(Vt, psi_t):
    """c[k][s] = <v_k, psi_s> over one timeslice: Vt [nev][Z][Y][X][3], psi_t [Z][Y][X][4][3]."""
    return np.einsum("kzyxc,zyxsc->ks", np.conj(Vt), psi_t)


def project(Vt, psi, t: int, mode: int) -> np.ndarray:
    """On timeslice t: mode 0 -> box(t) psi, mode 1 -> (1 - box(t)) psi; zero elsewhere.

    box(t) = V(t) V(t)^dag acts on colour and space and trivially on spin (eq. 1)."""
    psi = _c(psi)
    out = np.zeros_like(psi)
    for r in range(psi.shape[0]):
        pt = psi[r, t]
        c = _tcoef(Vt, pt)
        proj = np.einsum("kzyxc,ks->zyxsc", Vt, c)
        out[r, t] = proj if mode == 0 else pt - proj
    return out


def dist_sources(Vt, T: int, t0: int) -> np.ndarray:
    """v^(k)(t0) x e_s for k < nev, s < 4, index k*4 + s: [4 nev][T][Z][Y][X][4][3]."""
    nev = Vt.shape[0]
    shp = Vt.shape[1:4]
    out = np.zeros((nev * 4, T) + tuple(shp) + (4, 3), dtype=np.complex128)
    for k in range(nev):
        for s in range(4):
            out[k * 4 + s, t0, ..., s, :] = Vt[k]
    return out


DILUTIONS = {"spin": (1, 1), "spin-colour": (3, 1), "spin-eo": (1, 2), "spin-colour-eo": (3, 2)}


def dilution_size(dilution: str) -> int:
    """Dilution components per noise vector besides spin: colours x parities."""
    nc, npar = DILUTIONS[dilution]
    return nc * npar


def noise_sources(xi, T: int, t0: int, dilution: str = "spin") -> np.ndarray:
    """Diluted wall noise on timeslice t0 (the stochastic wall sources of Sec. 2).

    Each noise vector xi_r is split into the components P_d xi_r, d = c * npar + p:
    colour c only (colour dilution, nc = 3) and wall sites of parity
    p = (t0 + z + y + x) mod 2 only (even-odd dilution, npar = 2); each component
    is then spin-diluted, giving P_d xi_r x e_s with index (r * ndil + d) * 4 + s.
    "spin" alone is nc = npar = 1.  Returns [4 ndil N_r][T][Z][Y][X][4][3]."""
    nc, npar = DILUTIONS[dilution]
    nn = xi.shape[0]
    Z, Y, X = xi.shape[1:4]
    z, y, x = np.indices((Z, Y, X))
    par = (t0 + z + y + x) % 2
    ndil = nc * npar
    out = np.zeros((nn * ndil * 4, T, Z, Y, X, 4, 3), dtype=np.complex128)
    for r in range(nn):
        for c in range(nc):
            for p in range(npar):
                comp = np.array(xi[r], dtype=np.complex128)
                if nc == 3:
                    keep = np.zeros(3, bool)
                    keep[c] = True
                    comp[..., ~keep] = 0
                if npar == 2:
                    comp[par != p] = 0
                d = c * npar + p
                for s in range(4):
                    out[(r * ndil + d) * 4 + s, t0, ..., s, :] = comp
    return out


# ---------------------------------------------------------------- contractions (eq. 2-4)

GAMMA_NAMES = ("PS", "V")


def _gamma_list(name, g):
    if name == "PS":
        return [g[4]]
    if name == "V":
        return [g[1], g[2], g[3]]
    raise ValueError(name)


def _apply_X(X, Vall, psi):
    """X_t psi on every timeslice, X in {'1','P','Q'}; psi [T][Z][Y][X][4][3]."""
    if X == "1":
        return psi
    out = np.empty_like(psi)
    for t in range(psi.shape[0]):
        c = _tcoef(Vall[t], psi[t])
        proj = np.einsum("kzyxc,ks->zyxsc", Vall[t], c)
        out[t] = proj if X == "P" else psi[t] - proj
    return out


def _tdot(a, b):
    """<a, b>_t for all t: a, b [T][Z][Y][X][4][3] -> [T]."""
    return np.einsum("tzyxsc,tzyxsc->t", np.conj(a), b)


def _spin(M, psi):
    return np.einsum("st,...tc->...sc", M, psi)


def estimator(Vall, t0, phi_rows, phiY_rows, X: str, name: str, ndil: int = 1) -> np.ndarray:
    """One-end diluted estimator (eq. 3):

    C_XY(t) = 1/N_r sum_{r,d} sum_{s,s'} (G g5)_{s s'} < phiY_{r,d,s'}, g5 G X_t phi_{r,d,s} >_t

    phi_rows, phiY_rows: [N_r * ndil][4][T][Z][Y][X][4][3], the solutions for the
    components P_d xi_r x e_s (spin index second).  The components d of one noise
    vector are summed, the N_r noise vectors averaged.  For the vector channel the
    three spatial G are averaged.  Output indexed by Delta = (t - t0) mod T."""
    g = gammas()
    g5 = g[4]
    if phi_rows.shape[0] % ndil:
        raise ValueError("source groups must be a multiple of the dilution size")
    Nr = phi_rows.shape[0] // ndil
    Ng = phi_rows.shape[0]
    T = phi_rows.shape[2]
    acc = np.zeros(T, dtype=np.complex128)
    glist = _gamma_list(name, g)
    for G in glist:
        GL = g5 @ G
        GR = G @ g5
        for r in range(Ng):
            for s in range(4):
                xp = _spin(GL, _apply_X(X, Vall, phi_rows[r, s]))
                for sp in range(4):
                    if GR[s, sp] != 0:
                        acc += GR[s, sp] * _tdot(phiY_rows[r, sp], xp)
    acc /= Nr * len(glist)
    return np.roll(acc, -t0)


def perambulator(Vall, phi_dist_rows) -> np.ndarray:
    """tau[t][k, s][l, s'] = < v_k(t) x e_s, phi_{l,s'} >_t; phi_dist_rows [nev][4][T][...]."""
    return np.einsum("tkzyxc,lptzyxsc->tkslp", np.conj(Vall), phi_dist_rows)


def c_dist_exact(Vall, t0, phi_dist_rows, name: str) -> np.ndarray:
    """C_dist(t) = tr[g5 G box(t) S(t,t0) box(t0) G g5 S(t,t0)^dag] from the perambulator:

    sum_{k,l} tr_spin[ g5G tau_{kl} Gg5 tau_{kl}^dag ]  (eq. 3, first line)."""
    g = gammas()
    g5 = g[4]
    tau = perambulator(Vall, phi_dist_rows)  # [T][k][s][l][s']
    glist = _gamma_list(name, g)
    acc = np.zeros(tau.shape[0], dtype=np.complex128)
    for G in glist:
        GL = g5 @ G
        GR = G @ g5
        acc += np.einsum("ab,tkblc,cd,tkald->t", GL, tau, GR, np.conj(tau))
    acc /= len(glist)
    return np.roll(acc, -t0)


def c_qp_exact(Vall, t0, phi_dist_rows, name: str) -> np.ndarray:
    """Mixed term with (1-box) at the sink and box at the source, exact from the
    distillation solutions: sum_l sum_{s,s'} (G g5)_{s s'} < phi_{l,s'}, g5 G Q_t phi_{l,s} >_t."""
    g = gammas()
    g5 = g[4]
    nev = phi_dist_rows.shape[0]
    T = phi_dist_rows.shape[2]
    acc = np.zeros(T, dtype=np.complex128)
    glist = _gamma_list(name, g)
    for G in glist:
        GL = g5 @ G
        GR = G @ g5
        for l in range(nev):
            for s in range(4):
                xp = _spin(GL, _apply_X("Q", Vall, phi_dist_rows[l, s]))
                for sp in range(4):
                    if GR[s, sp] != 0:
                        acc += GR[s, sp] * _tdot(phi_dist_rows[l, sp], xp)
    acc /= len(glist)
    return np.roll(acc, -t0)


PARTS = ("QQ_est", "PQ_est", "QP_est", "PP_est", "11_est", "PP_exact", "QP_exact")


def correlators(Vall, t0: int, phi_dist, phi, phibar, names=GAMMA_NAMES, ndil: int = 1):
    """All correlator pieces for source timeslice t0.

    Vall: [T][nev][Z][Y][X][3] Laplacian eigenvectors of every timeslice.
    phi_dist: [4 nev] solutions for the distillation sources (index k*4+s).
    phi, phibar: [4 ndil N_r] solutions D^-1 eta and D^-1 (1-box(t0)) eta for the
    diluted noise sources of noise_sources (index (r*ndil + d)*4 + s).

    Returns {name: {part: [T] complex}} with parts
      QQ_est = C_rest estimate, PQ_est = C_mixed estimate (box at sink, 1-box at
      source, the paper's C_mixed), QP_est, PP_est, 11_est (full correlator),
      PP_exact = C_dist from the perambulator, QP_exact from the distillation solves.
    Raw traces: no volume factor, no minus sign; V averages the three spatial gammas.
    """
    T = phi.shape[1]
    nev = phi_dist.shape[0] // 4
    Ng = phi.shape[0] // 4
    sh = phi.shape[1:]
    pd = phi_dist.reshape((nev, 4) + sh)
    p1 = phi.reshape((Ng, 4) + sh)
    pq = phibar.reshape((Ng, 4) + sh)
    pp = p1 - pq  # D^-1 box eta
    out = {}
    for name in names:
        res = {
            "QQ_est": estimator(Vall, t0, p1, pq, "Q", name, ndil),
            "PQ_est": estimator(Vall, t0, p1, pq, "P", name, ndil),
            "QP_est": estimator(Vall, t0, p1, pp, "Q", name, ndil),
            "PP_est": estimator(Vall, t0, p1, pp, "P", name, ndil),
            "11_est": estimator(Vall, t0, p1, p1, "1", name, ndil),
            "PP_exact": c_dist_exact(Vall, t0, pd, name),
            "QP_exact": c_qp_exact(Vall, t0, pd, name),
        }
        out[name] = res
    return out


def correlators_vjp(Vall, t0: int, phi_dist, phi, phibar, G, ndil: int = 1):
    """Gradient of a real loss L through `correlators` (the backward of eqs. (3)-(4)'s
    contractions): G[name][part] is dL/dRe C + i dL/dIm C for each piece ([T], indexed by
    Delta = (t - t0) mod T; missing entries count as zero).  Returns (grad_phi_dist,
    grad_phi, grad_phibar), shaped like the inputs, such that to first order
    dL = Re sum_f <grad_f, d f>.

    Every piece has the form  c / |Gamma list| sum_Gamma sum_grp sum_{s,s'} N_{s s'}
    <A_{grp,s'}, M X_t B_{grp,s}>_t  with M = g5 Gamma, N = Gamma g5 (see `estimator`,
    `c_dist_exact`, `c_qp_exact`: for C_dist, A = B = phi_dist and X = box, since
    box(t') S^dag collapses to the distillation solutions).  Differentiating the
    sesquilinear form term by term:
        grad B_{grp,s}  += w(t) conj(N_{s s'}) X_t M^dag A_{grp,s'}
        grad A_{grp,s'} += conj(w(t)) N_{s s'} M X_t B_{grp,s}
    on timeslice t, with w(t) = G(t - t0) c / |Gamma list|."""
    g = gammas()
    g5 = g[4]
    sh = phi_dist.shape[1:]
    nd = phi_dist.shape[0] // 4
    Ng = phi.shape[0] // 4 if phi is not None else 0
    pd = phi_dist.reshape((nd, 4) + sh)
    gd = np.zeros_like(pd)
    if Ng:
        p1 = phi.reshape((Ng, 4) + sh)
        pq = phibar.reshape((Ng, 4) + sh)
        pp = p1 - pq
        g1 = np.zeros_like(p1)
        gq = np.zeros_like(pq)
        Nr = Ng // ndil
    # piece: (A rows, B rows, X, normalisation, how grad A splits into (grad phi, grad phibar, grad dist))
    pieces = {"PP_exact": ("dist", "dist", "P", 1.0), "QP_exact": ("dist", "dist", "Q", 1.0)}
    if Ng:
        pieces.update({"QQ_est": ("bar", "one", "Q", 1.0 / Nr), "PQ_est": ("bar", "one", "P", 1.0 / Nr),
                       "QP_est": ("P", "one", "Q", 1.0 / Nr), "PP_est": ("P", "one", "P", 1.0 / Nr),
                       "11_est": ("one", "one", "1", 1.0 / Nr)})
    rows = {"dist": pd}
    if Ng:
        rows.update({"one": p1, "bar": pq, "P": pp})

    def add_grad(kind, grp, s, v):
        if kind == "dist":
            gd[grp, s] += v
        elif kind == "one":
            g1[grp, s] += v
        elif kind == "bar":
            gq[grp, s] += v
        else:  # phi - phibar
            g1[grp, s] += v
            gq[grp, s] -= v

    for name, parts in G.items():
        glist = _gamma_list(name, g)
        for part, Gt in parts.items():
            if part not in pieces:
                continue
            akind, bkind, X, c = pieces[part]
            w = np.roll(np.asarray(Gt, dtype=np.complex128), t0) * c / len(glist)  # w[t] = G(t - t0) ...
            wt = w[:, None, None, None, None, None]
            A, B = rows[akind], rows[bkind]
            for Gm in glist:
                M = g5 @ Gm
                N = Gm @ g5
                for grp in range(A.shape[0]):
                    for s in range(4):
                        for sp in range(4):
                            if N[s, sp] == 0:
                                continue
                            add_grad(bkind, grp, s, wt * np.conj(N[s, sp]) * _apply_X(X, Vall, _spin(np.conj(M.T), A[grp, sp])))
                            add_grad(akind, grp, sp, np.conj(wt) * N[s, sp] * _spin(M, _apply_X(X, Vall, B[grp, s])))
    out_d = gd.reshape(phi_dist.shape)
    if not Ng:
        return out_d, None, None
    return out_d, g1.reshape(phi.shape), gq.reshape(phibar.shape)
