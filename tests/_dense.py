"""Brute-force helpers for the CPU pins: the conventions written out as dense
matrices, independent of the oracle's contraction code.

Chiral basis (stated convention): g0 = [[0,-1],[-1,0]], gk = [[0,-i sk],[i sk,0]]
in 2x2 spin blocks, g5 = diag(1,1,-1,-1).
"""
import numpy as np

SIG = [np.array([[0, 1], [1, 0]], complex),
       np.array([[0, -1j], [1j, 0]], complex),
       np.array([[1, 0], [0, -1]], complex)]


def gammas_convention():
    g = np.zeros((5, 4, 4), complex)
    g[0, 0:2, 2:4] = -np.eye(2)
    g[0, 2:4, 0:2] = -np.eye(2)
    for k in range(3):
        g[k + 1, 0:2, 2:4] = -1j * SIG[k]
        g[k + 1, 2:4, 0:2] = 1j * SIG[k]
    g[4] = np.diag([1, 1, -1, -1]).astype(complex)
    return g


G = gammas_convention()
G5 = G[4]

# direction mu -> array axis of [T][Z][Y][X]
AXIS = {0: 0, 1: 3, 2: 2, 3: 1}


def extent(dims, mu):
    return dims[AXIS[mu]]


def dense_operator(apply, n, batch=512, dtype=complex):
    """Dense matrix of a linear map given as apply(columns[k][n]) -> [k][n]."""
    M = np.zeros((n, n), dtype=dtype)
    for s in range(0, n, batch):
        e = min(n, s + batch)
        cols = np.zeros((e - s, n), dtype=dtype)
        cols[np.arange(e - s), np.arange(s, e)] = 1.0
        M[:, s:e] = apply(cols).T
    return M


def dense_dirac(orc, U, A):
    dims = U.shape[:4]
    n = int(np.prod(dims)) * 12
    shp = tuple(dims) + (4, 3)

    def ap(cols):
        k = cols.shape[0]
        return orc.dirac(U, A, cols.reshape((k,) + shp)).reshape(k, n)

    return dense_operator(ap, n)


def timeslice_index(dims, t):
    """Flat indices (spinor layout) of timeslice t."""
    T, Z, Y, X = dims
    per = Z * Y * X * 12
    return np.arange(t * per, (t + 1) * per)


def dense_box(Vt):
    """box(t) x 1_spin on one timeslice, in (site, spin, colour) order: [n][n]."""
    nev = Vt.shape[0]
    L3 = int(np.prod(Vt.shape[1:4]))
    Vm = Vt.reshape(nev, L3, 3)
    P = np.zeros((L3, 4, 3, L3, 4, 3), complex)
    pc = np.einsum("kmc,knd->mcnd", Vm, np.conj(Vm))
    for s in range(4):
        P[:, s, :, :, s, :] = pc
    return P.reshape(L3 * 12, L3 * 12)


def spin_op(M, L3):
    """1_site x M x 1_colour on one timeslice."""
    return np.kron(np.kron(np.eye(L3), M), np.eye(3))


def dense_trace(S, dims, Vall, t, t0, Gam, X, Y):
    """tr[g5 G X_t S(t,t0) Y_t0 G g5 S(t,t0)^dag] with X, Y in {'1','P','Q'}."""
    L3 = int(np.prod(dims[1:]))
    it = timeslice_index(dims, t)
    i0 = timeslice_index(dims, t0)
    Stt = S[np.ix_(it, i0)]
    n = L3 * 12
    I = np.eye(n)

    def proj(which, tt):
        if which == "1":
            return I
        P = dense_box(Vall[tt])
        return P if which == "P" else I - P

    L = spin_op(G5 @ Gam, L3)
    R = spin_op(Gam @ G5, L3)
    M = L @ proj(X, t) @ Stt @ proj(Y, t0) @ R @ np.conj(Stt.T)
    return np.trace(M)


def gauge_transform_links(U, g):
    """U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag."""
    Ug = np.empty_like(U)
    for mu in range(4):
        gp = np.roll(g, -1, axis=AXIS[mu])
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.conj(np.swapaxes(gp, -1, -2))
    return Ug


def wall_noise_matrix(xi, dims, t0, ncol, npar):
    """sum_d P_d xi xi^dag P_d on the wall t0 in (site, colour) order, for one noise vector
    xi [Z][Y][X][3] diluted into ncol colour blocks (1 or 3) and npar parity blocks (1 or 2)."""
    Z, Y, X = dims[1:]
    L3 = Z * Y * X
    v = np.asarray(xi, complex).reshape(L3, 3)
    z, y, x = np.indices((Z, Y, X))
    par = ((t0 + z + y + x) % 2).reshape(L3)
    N = np.zeros((L3 * 3, L3 * 3), complex)
    for c in range(ncol):
        for p in range(npar):
            w = v.copy()
            if ncol == 3:
                w[:, [k for k in range(3) if k != c]] = 0
            if npar == 2:
                w[par != p, :] = 0
            f = w.reshape(-1)
            N += np.outer(f, np.conj(f))
    return N


def dense_trace_noise(S, dims, Vall, t, t0, Gam, X, Y, Nwall):
    """tr[g5 G X_t S(t,t0) (N x 1_spin) Y_t0 G g5 S(t,t0)^dag]: what the one-end
    estimator computes for one noise vector whose diluted outer product is N."""
    L3 = int(np.prod(dims[1:]))
    it = timeslice_index(dims, t)
    i0 = timeslice_index(dims, t0)
    Stt = S[np.ix_(it, i0)]
    n = L3 * 12
    I = np.eye(n)
    N4 = Nwall.reshape(L3, 3, L3, 3)
    Nfull = np.einsum("mcnd,st->mscntd", N4, np.eye(4)).reshape(n, n)

    def proj(which, tt):
        if which == "1":
            return I
        P = dense_box(Vall[tt])
        return P if which == "P" else I - P

    L = spin_op(G5 @ Gam, L3)
    R = spin_op(Gam @ G5, L3)
    M = L @ proj(X, t) @ Stt @ Nfull @ proj(Y, t0) @ R @ np.conj(Stt.T)
    return np.trace(M)
