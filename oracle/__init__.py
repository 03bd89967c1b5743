"""Oracle: plain FP64 CPU reference of the tangent-point hot path.

TEST INFRASTRUCTURE ONLY -- imported by the tests, by ``__graft_entry__.smoke()`` and by
the CPU-baseline leg of ``bench.py``; never by the library.  It shares no code with the
HIP path.  The pair sums live in ``tp_oracle.c`` (plain loops, double precision); the
sparse and small dense linear algebra lives here on numpy/scipy.

Every function cites the passage of "Repulsive Surfaces" (Yu et al. 2021) it writes out.
Readings of points the paper leaves open are listed in the docstrings.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.sparse.csgraph import connected_components

from . import build as _build

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        i64, d = ctypes.c_int64, ctypes.c_double
        L.tpo_faces.argtypes = [_dp, _ip, i64, _dp, _dp, _dp]
        L.tpo_energy_faces_rows.argtypes = [_dp, _dp, _dp, i64, d, d, i64, i64, _dp]
        L.tpo_energy_faces.argtypes = [_dp, _dp, _dp, i64, d, d]
        L.tpo_energy_faces.restype = d
        L.tpo_energy.argtypes = [_dp, i64, _ip, i64, d, d]
        L.tpo_energy.restype = d
        L.tpo_gradient_rows.argtypes = [_dp, i64, _ip, i64, d, d, i64, i64, _dp, _dp]
        L.tpo_face_to_vertex.argtypes = [_dp, i64, _ip, i64, _dp, _dp]
        L.tpo_gradient.argtypes = [_dp, i64, _ip, i64, d, d, _dp]
        L.tpo_gradient.restype = d
        L.tpo_fractional_rows.argtypes = [_dp, i64, _ip, i64, d, _dp, ctypes.c_int, i64, i64, _dp]
        L.tpo_fractional_apply.argtypes = [_dp, i64, _ip, i64, d, _dp, ctypes.c_int, _dp]
        L.tpo_fractional_apply.restype = ctypes.c_int
        _lp = ctypes.POINTER(ctypes.c_int64)
        L.tpo_gradient_rowlist.argtypes = [_dp, i64, _ip, i64, d, d, _lp, i64, _dp, _dp]
        L.tpo_fractional_rowlist.argtypes = [_dp, i64, _ip, i64, d, _dp, ctypes.c_int, _lp, i64, _dp]
        L.tpo_fractional_gather.argtypes = [_ip, i64, i64, _dp, ctypes.c_int, _dp]
        L.tpo_face_gradients.argtypes = [_dp, _ip, i64, _dp, ctypes.c_int, _dp]
        L.tpo_sobolev_rowlist.argtypes = [_dp, i64, _ip, i64, d, _dp, ctypes.c_int, _lp, i64, _dp]
        L.tpo_sobolev_gather.argtypes = [_dp, _ip, i64, i64, _dp, ctypes.c_int, _dp]
        L.tpo_sobolev_apply.argtypes = [_dp, i64, _ip, i64, d, _dp, ctypes.c_int, _dp]
        L.tpo_sobolev_apply.restype = ctypes.c_int
        L.tpo_obstacle.argtypes = [_dp, i64, _ip, i64, _dp, _ip, i64, d, _dp]
        L.tpo_obstacle.restype = d
        L.tpo_bh_frozen.argtypes = [_dp, _dp, i64, _ip, i64, d, d, d, ctypes.c_int, _dp, _lp]
        L.tpo_bh_frozen.restype = d
        L.tpo_bh_order.argtypes = [_dp, _ip, i64, ctypes.c_int, _lp]
        L.tpo_bh_fractional.argtypes = [_dp, i64, _ip, i64, d, d, ctypes.c_int, _dp, ctypes.c_int, _dp]
        L.tpo_bh_fractional.restype = ctypes.c_int
        L.tpo_bct_fractional.argtypes = [_dp, i64, _ip, i64, d, d, ctypes.c_int, _dp, ctypes.c_int, _dp, _lp]
        L.tpo_bct_fractional.restype = ctypes.c_int
        L.tpo_obstacle_bh.argtypes = [_dp, i64, _ip, i64, _dp, _ip, i64, d, d, ctypes.c_int, _dp, _lp]
        L.tpo_obstacle_bh.restype = d
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _prep(V, F):
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    assert V.ndim == 2 and V.shape[1] == 3 and F.ndim == 2 and F.shape[1] == 3
    return V, F


# ----------------------------------------------------------------------------------
# Exponents.  The paper fixes alpha = p, beta = 2p with p = 6 (Sec. 2.1) and derives
# s = 2 - n/p for surfaces (n = 2, Sec. 2.3); the preconditioner applies L^sigma with
# sigma = 2 - s (Sec. 5.2).  For independent (alpha, beta) we read s = (beta - 2)/alpha,
# which equals 2 - 2/p when beta = 2 alpha (an extrapolation, flagged in the design notes).
DEFAULT_ALPHA = 6.0
DEFAULT_BETA = 12.0


def sobolev_s(alpha: float = DEFAULT_ALPHA, beta: float = DEFAULT_BETA) -> float:
    return (beta - 2.0) / alpha


def preconditioner_sigma(alpha: float = DEFAULT_ALPHA, beta: float = DEFAULT_BETA) -> float:
    return 2.0 - sobolev_s(alpha, beta)


# ----------------------------------------------------------------------------------
# Pair sums (C).

def faces(V, F):
    """Barycenters X (nF x 3), unit normals N (nF x 3), areas a (nF) (Sec. 3.1)."""
    V, F = _prep(V, F)
    nF = F.shape[0]
    X, N, A = np.empty((nF, 3)), np.empty((nF, 3)), np.empty(nF)
    lib().tpo_faces(_d(V), _i(F), nF, _d(X), _d(N), _d(A))
    return X, N, A


def energy_faces(X, N, A, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA) -> float:
    """E = sum_S sum_{T != S} K(S,T) a_S a_T on given face quantities (eq. DiscreteEnergy)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    N = np.ascontiguousarray(N, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    return float(lib().tpo_energy_faces(_d(X), _d(N), _d(A), A.shape[0], alpha, beta))


def energy(V, F, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA) -> float:
    """Discrete tangent-point energy (eq. DiscreteEnergy with eq. DiscreteTangentPointKernel)."""
    V, F = _prep(V, F)
    return float(lib().tpo_energy(_d(V), V.shape[0], _i(F), F.shape[0], alpha, beta))


def gradient(V, F, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """(E, dE) with dE (nV x 3) the exact differential by the chain rule (Sec. 3.1)."""
    V, F = _prep(V, F)
    dE = np.empty_like(V)
    E = lib().tpo_gradient(_d(V), V.shape[0], _i(F), F.shape[0], alpha, beta, _d(dE))
    return float(E), dE


def gradient_rows(V, F, s0, s1, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """Per-face partial derivatives (dE/dX_S, dE/dN_S, dE/da_S) and energy rows for
    faces S in [s0, s1): the pair loop of ``gradient`` over a band of rows."""
    V, F = _prep(V, F)
    n = s1 - s0
    g = np.empty((n, 7))
    Erow = np.empty(n)
    lib().tpo_gradient_rows(_d(V), V.shape[0], _i(F), F.shape[0], alpha, beta, s0, s1, _d(g), _d(Erow))
    return g, Erow


def _incident_faces(F, verts):
    F = np.asarray(F)
    mask = np.isin(F, np.asarray(verts)).any(axis=1)
    return np.nonzero(mask)[0].astype(np.int64)


def gradient_at_vertices(V, F, verts, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """Exact dE at the listed vertices only: the pair sums are taken for the faces incident
    to them (all T), then chained to vertices; O(|faces| nF) instead of O(nF^2)."""
    V, F = _prep(V, F)
    rows = _incident_faces(F, verts)
    g = np.zeros((F.shape[0], 7))
    gr = np.empty((rows.size, 7))
    lib().tpo_gradient_rowlist(_d(V), V.shape[0], _i(F), F.shape[0], alpha, beta,
                               rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), rows.size,
                               _d(gr), None)
    g[rows] = gr
    dE = np.empty_like(V)
    lib().tpo_face_to_vertex(_d(V), V.shape[0], _i(F), F.shape[0], _d(g), _d(dE))
    return dE[np.asarray(verts)]


def fractional_at_vertices(V, F, u, verts, sigma):
    """Exact (L^sigma u) at the listed vertices only (rows of the incident faces)."""
    V, F = _prep(V, F)
    U = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(V.shape[0], -1))
    k = U.shape[1]
    rows = _incident_faces(F, verts)
    w = np.zeros((F.shape[0], k))
    wr = np.empty((rows.size, k))
    lib().tpo_fractional_rowlist(_d(V), V.shape[0], _i(F), F.shape[0], sigma, _d(U), k,
                                 rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), rows.size, _d(wr))
    w[rows] = wr
    Lu = np.empty((V.shape[0], k))
    lib().tpo_fractional_gather(_i(F), F.shape[0], V.shape[0], _d(w), k, _d(Lu))
    return Lu[np.asarray(verts)]


def fractional_apply(V, F, u, sigma=None, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """L^sigma u for u of shape (nV,) or (nV, k), k <= 64 (eq. DiscreteLaplacianQuartic)."""
    V, F = _prep(V, F)
    if sigma is None:
        sigma = preconditioner_sigma(alpha, beta)
    u = np.asarray(u, dtype=np.float64)
    vec = u.ndim == 1
    U = np.ascontiguousarray(u.reshape(u.shape[0], -1))
    k = U.shape[1]
    Lu = np.empty_like(U)
    rc = lib().tpo_fractional_apply(_d(V), V.shape[0], _i(F), F.shape[0], sigma, _d(U), k, _d(Lu))
    if rc != 0:
        raise ValueError("k must be in [1, 64]")
    return Lu[:, 0] if vec else Lu


def fractional_rows(V, F, u, s0, s1, sigma):
    V, F = _prep(V, F)
    U = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(V.shape[0], -1))
    k = U.shape[1]
    w = np.empty((s1 - s0, k))
    lib().tpo_fractional_rows(_d(V), V.shape[0], _i(F), F.shape[0], sigma, _d(U), k, s0, s1, _d(w))
    return w


# ----------------------------------------------------------------------------------
# Dense fractional operator by Algorithm 1 (tiny meshes only).

def dense_fractional_matrix(V, F, sigma):
    """|V| x |V| matrix L^sigma assembled pair by pair as in Algorithm 1 (Sec. 2.4).

    'All distinct pairs of faces' is read as all ordered pairs S != T, which is the sum
    of eq. DiscreteLaplacianQuartic; phi_i(S) = 1/3 for the corners of S, 0 otherwise."""
    V, F = _prep(V, F)
    X, _, A = faces(V, F)
    nV, nF = V.shape[0], F.shape[0]
    L = np.zeros((nV, nV))
    for S in range(nF):
        for T in range(nF):
            if S == T:
                continue
            verts = sorted(set(F[S].tolist()) | set(F[T].tolist()))
            phiS = {v: (1.0 / 3.0 if v in F[S] else 0.0) for v in verts}
            phiT = {v: (1.0 / 3.0 if v in F[T] else 0.0) for v in verts}
            h = np.linalg.norm(X[S] - X[T]) ** (-(2.0 * sigma + 2.0)) * A[S] * A[T]
            for i in verts:
                for j in verts:
                    L[i, j] += (phiS[i] - phiT[i]) * (phiS[j] - phiT[j]) * h
    return L


# ----------------------------------------------------------------------------------
# The inner-product operator A = B + B0 (Sec. 2.4; discrete terms in Sec. 3.2.1; applied in
# the factored form of Sec. 5.1.2 and 5.1.3).  Its kernel exponent is 2s (sigma = s - 1).

def face_gradients(V, F, u):
    """D u(S): gradient of the piecewise linear u on every face (nF x k x 3)."""
    V, F = _prep(V, F)
    U = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(V.shape[0], -1))
    k = U.shape[1]
    Du = np.empty((F.shape[0], k, 3))
    lib().tpo_face_gradients(_d(V), _i(F), F.shape[0], _d(U), k, _d(Du))
    return Du


def sobolev_apply(V, F, u, s=None, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """A u = (B + B0) u for u of shape (nV,) or (nV, k), k <= 64."""
    V, F = _prep(V, F)
    if s is None:
        s = sobolev_s(alpha, beta)
    u = np.asarray(u, dtype=np.float64)
    vec = u.ndim == 1
    U = np.ascontiguousarray(u.reshape(u.shape[0], -1))
    k = U.shape[1]
    Au = np.empty_like(U)
    rc = lib().tpo_sobolev_apply(_d(V), V.shape[0], _i(F), F.shape[0], s, _d(U), k, _d(Au))
    if rc != 0:
        raise ValueError("k must be in [1, 64]")
    return Au[:, 0] if vec else Au


def sobolev_at_vertices(V, F, u, verts, s):
    """Exact (A u) at the listed vertices only (rows of the incident faces)."""
    V, F = _prep(V, F)
    U = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(V.shape[0], -1))
    k = U.shape[1]
    rows = _incident_faces(F, verts)
    z = np.zeros((F.shape[0], 4 * k))
    zr = np.empty((rows.size, 4 * k))
    lib().tpo_sobolev_rowlist(_d(V), V.shape[0], _i(F), F.shape[0], s, _d(U), k,
                              rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), rows.size, _d(zr))
    z[rows] = zr
    Au = np.empty((V.shape[0], k))
    lib().tpo_sobolev_gather(_d(V), _i(F), F.shape[0], V.shape[0], _d(z), k, _d(Au))
    return Au[np.asarray(verts)]


def dense_sobolev_inverse(V, F, s=None, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """R -> A^+ P R with A = B + B0 assembled densely from sobolev_apply on the unit vectors
    (small meshes only), P the global mean removal and the result of global mean zero: A's
    null space is the global constants (the low-order term couples connected components)."""
    V, F = _prep(V, F)
    if s is None:
        s = sobolev_s(alpha, beta)
    n = V.shape[0]
    A = np.empty((n, n))
    for c0 in range(0, n, 64):
        c1 = min(n, c0 + 64)
        E = np.zeros((n, c1 - c0))
        E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
        A[:, c0:c1] = sobolev_apply(V, F, E, s)
    A = 0.5 * (A + A.T) + np.ones((n, n))     # the constants' part of A^+ P R is removed below

    def inverse(R):
        R = np.asarray(R, dtype=np.float64)
        Y = np.linalg.solve(A, R - R.mean(0))
        return Y - Y.mean(0)
    return inverse


def dense_sobolev_matrices(V, F, s):
    """|V| x |V| matrices B and B0 assembled pair by pair from eqs. DiscreteHighOrderTerm and
    DiscreteLowOrderTerm (tiny meshes only), over all ordered pairs S != T.

    D phi_i(S) is taken from its definition d phi_i (df)^+ (Sec. 2.4): df is the 3 x 2
    Jacobian of the affine map from the unit triangle onto S, and ^+ its Moore-Penrose
    pseudoinverse (numpy.linalg.pinv).  K2(S,T) = |N_S . (X_S - X_T)|^2 / |X_S - X_T|^4 is
    used as written, not symmetrized."""
    V, F = _prep(V, F)
    X, N, A = faces(V, F)
    nV, nF = V.shape[0], F.shape[0]
    # barycentric coordinates on the unit triangle: phi_0 = 1 - x - y, phi_1 = x, phi_2 = y
    dphi_ref = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    Dphi = []
    for S in range(nF):
        fi, fj, fk = V[F[S]]
        df = np.stack([fj - fi, fk - fi], axis=1)      # 3 x 2
        pinv = np.linalg.pinv(df)                       # 2 x 3
        Dphi.append({int(F[S][c]): dphi_ref[c] @ pinv for c in range(3)})
    B = np.zeros((nV, nV))
    B0 = np.zeros((nV, nV))
    zero = np.zeros(3)
    for S in range(nF):
        for T in range(nF):
            if S == T:
                continue
            verts = sorted(set(F[S].tolist()) | set(F[T].tolist()))
            d = X[S] - X[T]
            r2 = float(d @ d)
            h = r2 ** (-s) * A[S] * A[T]
            K2 = float(N[S] @ d) ** 2 / r2 ** 2
            for i in verts:
                gi = Dphi[S].get(i, zero) - Dphi[T].get(i, zero)
                pi = (1.0 / 3.0 if i in F[S] else 0.0) - (1.0 / 3.0 if i in F[T] else 0.0)
                for j in verts:
                    gj = Dphi[S].get(j, zero) - Dphi[T].get(j, zero)
                    pj = (1.0 / 3.0 if j in F[S] else 0.0) - (1.0 / 3.0 if j in F[T] else 0.0)
                    B[i, j] += float(gi @ gj) * h
                    B0[i, j] += pi * pj * h * K2
    return B, B0


# ----------------------------------------------------------------------------------
# Cotan Laplacian, components and Poisson solves (Sec. 5.2).

def cotan_laplacian(V, F):
    """Weak (stiffness) cotan Laplacian C with C_ij = -1/2 (cot alpha_ij + cot beta_ij) for
    each edge ij and C_ii = -sum_j C_ij.  The paper names only 'the sparse cotan-weighted
    Laplace-Beltrami operator' (Sec. 5.2); this is the textbook form."""
    V, F = _prep(V, F)
    nV = V.shape[0]
    rows, cols, vals = [], [], []
    for c in range(3):
        i, j, k = F[:, c], F[:, (c + 1) % 3], F[:, (c + 2) % 3]
        u = V[j] - V[i]
        w = V[k] - V[i]
        cot = np.einsum("ij,ij->i", u, w) / np.linalg.norm(np.cross(u, w), axis=1)
        h = 0.5 * cot  # weight of the edge (j,k) opposite corner i
        rows += [j, k, j, k]
        cols += [k, j, j, k]
        vals += [-h, -h, h, h]
    C = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nV, nV)).tocsr()
    C.sum_duplicates()
    return C


def components(F, nV):
    """Connected-component label of every vertex (Sec. 7.1 treats each component apart)."""
    F = np.asarray(F)
    r = np.concatenate([F[:, 0], F[:, 1], F[:, 2]])
    c = np.concatenate([F[:, 1], F[:, 2], F[:, 0]])
    G = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(nV, nV))
    n, labels = connected_components(G, directed=False)
    return n, labels


def project_mean_zero(x, labels, ncomp=None):
    """Subtract the unweighted per-component mean of every column (reading of the fixed
    barycenter constraint, Sec. 7.1.1, folded into the Laplacians as in Sec. 7.2)."""
    x = np.array(x, dtype=np.float64, copy=True)
    X2 = x.reshape(x.shape[0], -1)
    if ncomp is None:
        ncomp = int(labels.max()) + 1
    for c in range(ncomp):
        m = labels == c
        X2[m] -= X2[m].mean(axis=0)
    return x


def poisson_solve(C, b, labels, pins=None):
    """Exact solution x of C x = P b with P x = x (per-component mean zero), by a sparse
    direct solve of C bordered with one indicator row per component.

    With pins (vertex indices, Sec. 7.1.2), their rows are appended to the Laplacian as in
    Sec. 7.2: the bordered system [[C, E^T], [E, 0]] with one unit row e_i per pinned vertex
    gives x_i = 0 there and C x = b on the other rows; a component holding a pin has no
    nullspace left, so only the components without pins keep the mean-zero rows."""
    b = np.asarray(b, dtype=np.float64)
    B2 = b.reshape(b.shape[0], -1)
    nV = C.shape[0]
    ncomp = int(labels.max()) + 1
    pins = np.unique(np.asarray([] if pins is None else pins, dtype=np.int64))
    pinned_comp = np.zeros(ncomp, dtype=bool)
    pinned_comp[labels[pins]] = True
    free = np.nonzero(~pinned_comp)[0]
    Bm = sp.coo_matrix((np.ones(nV), (labels, np.arange(nV))), shape=(ncomp, nV)).tocsr()[free]
    Pm = sp.coo_matrix((np.ones(pins.size), (np.arange(pins.size), pins)), shape=(pins.size, nV)).tocsr()
    E = sp.vstack([Bm, Pm]).tocsr()
    M = sp.bmat([[C, E.T], [E, None]], format="csc")
    Pb = B2.copy()
    for c in free:
        msk = labels == c
        Pb[msk] -= Pb[msk].mean(axis=0)
    rhs = np.vstack([Pb, np.zeros((E.shape[0], B2.shape[1]))])
    sol = spla.splu(M).solve(rhs)
    return sol[:nV].reshape(b.shape)


# ----------------------------------------------------------------------------------
# Constraints (Sec. 7.1.3, 7.1.4).

def total_area(V, F) -> float:
    _, _, A = faces(V, F)
    return float(A.sum())


def total_volume(V, F) -> float:
    """Signed volume (1/6) sum_{(ijk)} f_i . (f_j x f_k)."""
    V, F = _prep(V, F)
    return float(np.einsum("ij,ij->i", V[F[:, 0]], np.cross(V[F[:, 1]], V[F[:, 2]])).sum() / 6.0)


def area_gradient(V, F):
    """d(sum_S a_S)/df: for face (i,j,k), d a_S / d f_i = (1/2) N_S x (f_k - f_j), and
    cyclically for j and k."""
    V, F = _prep(V, F)
    _, N, _ = faces(V, F)
    g = np.zeros_like(V)
    for c in range(3):
        i, j, k = F[:, c], F[:, (c + 1) % 3], F[:, (c + 2) % 3]
        np.add.at(g, i, 0.5 * np.cross(N, V[k] - V[j]))
    return g


def volume_gradient(V, F):
    """d Vol/df: for face (i,j,k), d/d f_i [f_i . (f_j x f_k)]/6 = (f_j x f_k)/6, cyclically."""
    V, F = _prep(V, F)
    g = np.zeros_like(V)
    for c in range(3):
        i, j, k = F[:, c], F[:, (c + 1) % 3], F[:, (c + 2) % 3]
        np.add.at(g, i, np.cross(V[j], V[k]) / 6.0)
    return g


# ----------------------------------------------------------------------------------
# Preconditioner (Sec. 5.2) and one projected descent step (Sec. 3, 5.3, 5.4).

def precond_apply(V, F, b, sigma=None, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA, C=None, labels=None, pins=None):
    """A~^{-1} b = C^+ P L^sigma C^+ P b, columnwise (Sec. 5.2).

    Readings: both Laplace-Beltrami factors are the weak cotan matrix C with no mass
    matrix; C^+ P b is the per-component mean-zero solution of C x = P b.  With pins, both
    factors are the Laplacian with the pin rows appended (poisson_solve, Sec. 7.2)."""
    V, F = _prep(V, F)
    if sigma is None:
        sigma = preconditioner_sigma(alpha, beta)
    if C is None:
        C = cotan_laplacian(V, F)
    if labels is None:
        _, labels = components(F, V.shape[0])
    y = poisson_solve(C, b, labels, pins)
    z = fractional_apply(V, F, y, sigma)
    return poisson_solve(C, z, labels, pins)


@dataclass
class StepResult:
    V: np.ndarray          # new vertex positions
    E: float               # energy at the start of the step
    grad_norm: float
    tau: float
    backtracks: int
    direction: np.ndarray  # projected descent direction x (nV x 3)
    phi_before: np.ndarray  # Phi(f)
    phi_after: np.ndarray   # Phi after the corrective step
    phi_trial: np.ndarray = field(default_factory=lambda: np.zeros(0))  # Phi(f + tau x)
    schur: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))


ARMIJO_C = 1e-4
ARMIJO_SHRINK = 0.5
ARMIJO_MAX_BACKTRACKS = 30


def precond_step(V, F, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA, sigma=None, tau=None,
                 line_search=True, constrain_area=True, constrain_volume=True,
                 area_target=None, volume_target=None, inverse=None, area_penalty=0.0,
                 volume_penalty=0.0, obstacle_mesh=None, obstacle_p=6.0, obstacle_weight=0.0,
                 barycenter_motion=False, implicit=None, pins=None):
    """One constrained descent step with A~^{-1} in place of A_3^{-1}, or with the map R -> Y
    given as `inverse` (for instance A_3^{-1} from dense_sobolev_inverse; Sec. 5.4).

    1. g = dE (Sec. 3.1).  2. J = rows of the active constraints: total area (Sec. 7.1.3)
    and total volume (Sec. 7.1.4).  3. Y = A~^{-1} J^T, y_g = A~^{-1} g; Schur matrix
    S = J Y (the paper's -(M/A), eq. SchurComplementMA); direction
    x = -(y_g - Y S^{-1} J y_g), which solves eq. SaddleProblem with A_3^{-1} -> A~^{-1}
    (eq. SchurProjectedExpression, with the sign of the descent direction).
    4. Armijo backtracking from tau0 (constants c = 1e-4, shrink 1/2, at most 30 halvings;
    the paper names the rule but not the constants).  tau0 defaults to the step whose
    largest vertex move is half the mean edge length.  With line_search=False, tau = tau0.
    5. Corrective step h = -Y S^{-1} Phi(f + tau x) (Sec. 5.3.1), added to f + tau x.
    With area_penalty / volume_penalty > 0 the objective is E plus the potentials of Sec. 7.3.1
    (penalty_terms): their gradients join g and the line search, and E of the result is the
    total.  obstacle_mesh = (Vo, Fo) with obstacle_weight > 0 adds weight x the obstacle
    potential (obstacle) to the objective in the same way.  barycenter_motion adds to x, per
    connected component, minus the vertex-area-weighted mean of g (Sec. 7.1.1; vertex area
    = a third of the areas of the faces around the vertex).  pins (vertex indices) adds the
    vertex pin constraints of Sec. 7.1.2 the way Sec. 7.2 prescribes for linear positional
    rows: inside the operator rather than in the Schur complement, i.e. appended to both
    Laplacians of the preconditioner (precond_apply), so every column of Y, and with it the
    direction and the corrective step, vanishes at the pinned vertices."""
    V, F = _prep(V, F)
    if pins is not None and len(pins) and (barycenter_motion or inverse is not None):
        raise ValueError("pins combine with neither barycenter motions nor a given inverse")
    nV = V.shape[0]
    if sigma is None:
        sigma = preconditioner_sigma(alpha, beta)
    C = cotan_laplacian(V, F)
    _, labels = components(F, nV)
    E0, g = gradient(V, F, alpha, beta)
    A0 = total_area(V, F) if area_target is None else area_target
    V0 = total_volume(V, F) if volume_target is None else volume_target
    if area_penalty > 0.0 or volume_penalty > 0.0:
        p0, gp = penalty_terms(V, F, A0, V0, area_penalty, volume_penalty)
        E0, g = E0 + p0, g + gp
    use_obs = obstacle_mesh is not None and obstacle_weight > 0.0
    if use_obs:
        eo, go = obstacle(V, F, obstacle_mesh[0], obstacle_mesh[1], obstacle_p)
        E0, g = E0 + obstacle_weight * eo, g + obstacle_weight * go
    if implicit:
        ei, gi = implicit_potential(V, F, implicit)
        E0, g = E0 + ei, g + gi

    def objective(Vx):
        e = energy(Vx, F, alpha, beta)
        if area_penalty > 0.0 or volume_penalty > 0.0:
            e += penalty_terms(Vx, F, A0, V0, area_penalty, volume_penalty)[0]
        if use_obs:
            e += obstacle_weight * obstacle(Vx, F, obstacle_mesh[0], obstacle_mesh[1], obstacle_p, False)[0]
        if implicit:
            e += implicit_potential(Vx, F, implicit, False)[0]
        return e
    rows, targets, fns = [], [], []
    if constrain_area:
        rows.append(area_gradient(V, F)); targets.append(A0); fns.append(total_area)
    if constrain_volume:
        rows.append(volume_gradient(V, F)); targets.append(V0); fns.append(total_volume)
    R = np.concatenate([g] + rows, axis=1)           # nV x 3(1 + k)
    Y = precond_apply(V, F, R, sigma, C=C, labels=labels, pins=pins) if inverse is None else inverse(R)
    yg = Y[:, 0:3]
    k = len(rows)
    YJ = [Y[:, 3 + 3 * m: 6 + 3 * m] for m in range(k)]
    S = np.array([[np.vdot(rows[a], YJ[b]) for b in range(k)] for a in range(k)]).reshape(k, k)
    if k:
        rhs = np.array([np.vdot(rows[a], yg) for a in range(k)])
        mu = np.linalg.solve(S, rhs)
        x = -(yg - sum(mu[m] * YJ[m] for m in range(k)))
    else:
        x = -yg
    if barycenter_motion:
        Af = faces(V, F)[2]
        av = np.zeros(nV)
        for c in range(3):
            np.add.at(av, F[:, c], Af / 3.0)
        for lab in np.unique(labels):
            idx = labels == lab
            x[idx] -= (av[idx, None] * g[idx]).sum(0) / av[idx].sum()
    phi_before = np.array([fns[m](V, F) - targets[m] for m in range(k)])
    slope = float(np.vdot(g, x))
    if tau is None:
        from_edges = 0.5 * _mean_edge_length(V, F)
        tau0 = from_edges / np.abs(np.linalg.norm(x, axis=1)).max()
    else:
        tau0 = float(tau)
    t = tau0
    bt = 0
    if line_search:
        # a non-finite objective fails the test (written so that NaN is not accepted)
        while not (objective(V + t * x) <= E0 + ARMIJO_C * t * slope) and bt < ARMIJO_MAX_BACKTRACKS:
            t *= ARMIJO_SHRINK
            bt += 1
    Vt = V + t * x
    if line_search and not np.isfinite(objective(Vt)):
        raise FloatingPointError("line search found no step with a finite objective")
    if k:
        phi = np.array([fns[m](Vt, F) - targets[m] for m in range(k)])
        lam = np.linalg.solve(S, phi)
        h = -sum(lam[m] * YJ[m] for m in range(k))
        Vn = Vt + h
        phi_after = np.array([fns[m](Vn, F) - targets[m] for m in range(k)])
    else:
        Vn = Vt
        phi = phi_after = phi_before
    return StepResult(V=Vn, E=E0, grad_norm=float(np.linalg.norm(g)), tau=t, backtracks=bt,
                      direction=x, phi_before=phi_before, phi_after=phi_after, phi_trial=phi, schur=S)


def obstacle(V, F, Vo, Fo, p=6.0, with_grad=True):
    """Static obstacle potential of Sec. 7.3.2 at the surface's face barycenters, integrated over
    the faces, and its differential with respect to the surface vertices (tpo_obstacle)."""
    V, F = _prep(V, F)
    Vo, Fo = _prep(Vo, Fo)
    dE = np.empty_like(V) if with_grad else None
    E = lib().tpo_obstacle(_d(V), V.shape[0], _i(F), F.shape[0], _d(Vo), _i(Fo), Fo.shape[0], p,
                           _d(dE) if with_grad else None)
    return float(E), dE


def obstacle_bh(V, F, Vo, Fo, theta, p=6.0, leaf=8, with_grad=True):
    """The static obstacle potential with Barnes-Hut over the obstacle's faces (tpo_obstacle_bh):
    the tree of bh_gradient built on the obstacle, admissibility for the barycenter of each
    surface face as a point.  Returns (E, dE or None, (far terms, near terms)); theta = 0 is
    obstacle()."""
    V, F = _prep(V, F)
    Vo, Fo = _prep(Vo, Fo)
    dE = np.empty_like(V) if with_grad else None
    cnt = np.zeros(2, dtype=np.int64)
    E = lib().tpo_obstacle_bh(_d(V), V.shape[0], _i(F), F.shape[0], _d(Vo), _i(Fo), Fo.shape[0], float(p),
                              float(theta), int(leaf), _d(dE) if with_grad else None,
                              cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return float(E), dE, (int(cnt[0]), int(cnt[1]))


def implicit_potential(V, F, prims, with_grad=True):
    """Implicit obstacles and attractors of Sec. 7.3.3, evaluated at the face barycenters and
    integrated with the face areas: sum_k w_k sum_T a_T phi_k(X_T), phi = d^-p (obstacle) or
    |d|^p (attractor); d the signed distance to a plane {x : q.x = c} (kind 0, q normalised
    with c) or a sphere of center q and radius c (kind 1).  prims: list of dicts with keys
    kind, q, c, p, w, attract.  Returns (E, dE) with dE by the chain rule through X_T (1/3
    per corner) and a_T (N_T x (f_k - f_j) / 2 per corner i, cyclic)."""
    V, F = _prep(V, F)
    X, N, a = faces(V, F)
    phi = np.zeros(len(a))
    dphi = np.zeros_like(X)
    for pr in prims:
        q = np.asarray(pr["q"], dtype=np.float64)
        if pr["kind"] == 0:
            nq = np.linalg.norm(q)
            n = np.broadcast_to(q / nq, X.shape)
            d = X @ (q / nq) - pr["c"] / nq
        else:
            r = X - q
            rn = np.linalg.norm(r, axis=1)
            n = r / rn[:, None]
            d = rn - pr["c"]
        p, w = pr["p"], pr["w"]
        if pr.get("attract", False):
            f = np.abs(d) ** p
            df = p * np.abs(d) ** (p - 1.0) * np.sign(d)
        else:
            # on or inside the obstacle the potential is +infinity for every p (d^-p alone
            # would be finite for an even p and negative for an odd one when d < 0)
            inside = d <= 0.0
            ds = np.where(inside, 1.0, d)
            f = np.where(inside, np.inf, ds ** (-p))
            df = np.where(inside, -np.inf, -p * ds ** (-p - 1.0))
        phi += w * f
        dphi += (w * df)[:, None] * n
    E = float(np.sum(a * phi))
    if not with_grad:
        return E, None
    dE = np.zeros_like(V)
    for corner in range(3):
        i, j, k = F[:, corner], F[:, (corner + 1) % 3], F[:, (corner + 2) % 3]
        da = 0.5 * np.cross(N, V[k] - V[j])
        np.add.at(dE, i, a[:, None] * dphi / 3.0 + phi[:, None] * da)
    return E, dE


def penalty_terms(V, F, A0, V0, area_weight, volume_weight):
    """Total area and volume potentials of Sec. 7.3.1, w_A (A/A0 - 1)^2 + w_V (V/V0 - 1)^2, and
    their gradient with respect to the vertex positions (nV x 3)."""
    A, Vol = total_area(V, F), total_volume(V, F)
    e = area_weight * (A / A0 - 1.0) ** 2 + volume_weight * (Vol / V0 - 1.0) ** 2
    g = (2.0 * area_weight * (A / A0 - 1.0) / A0) * area_gradient(V, F) + \
        (2.0 * volume_weight * (Vol / V0 - 1.0) / V0) * volume_gradient(V, F)
    return e, g


def _mean_edge_length(V, F) -> float:
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(V[e[:, 0]] - V[e[:, 1]], axis=1).mean())


# ----------------------------------------------------------------------------------
# Barnes-Hut approximation (Sec. 4): tree, admissibility and traversal as written in the
# C oracle; the differential is exact for E_BH with the interaction lists held fixed.

def bh_gradient(V, F, theta, leaf=8, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA, with_grad=True):
    """(E_BH, dE_BH or None, (far terms, near terms))."""
    V, F = _prep(V, F)
    dE = np.empty_like(V) if with_grad else None
    cnt = np.zeros(2, dtype=np.int64)
    E = lib().tpo_bh_frozen(_d(V), _d(V), V.shape[0], _i(F), F.shape[0], alpha, beta, float(theta),
                            int(leaf), _d(dE) if with_grad else None,
                            cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return float(E), dE, (int(cnt[0]), int(cnt[1]))


def bh_energy_frozen(V0, V, F, theta, leaf=8, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """E_BH at vertices V with the tree membership and interaction lists of V0."""
    V0, F = _prep(V0, F)
    V = np.ascontiguousarray(V, dtype=np.float64)
    return float(lib().tpo_bh_frozen(_d(V0), _d(V), V.shape[0], _i(F), F.shape[0], alpha, beta,
                                     float(theta), int(leaf), None, None))


def bh_order(V, F, leaf=8):
    """Sorted face order of the tree (Morton code of the barycenter, ties by index)."""
    V, F = _prep(V, F)
    out = np.empty(F.shape[0], dtype=np.int64)
    lib().tpo_bh_order(_d(V), _i(F), F.shape[0], int(leaf), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def bh_fractional_apply(V, F, u, theta, sigma=None, leaf=8, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """L^sigma u with the Barnes-Hut approximation of the fractional kernel matrix on the
    tree of bh_gradient (tpo_bh_fractional); theta = 0 is fractional_apply."""
    V, F = _prep(V, F)
    if sigma is None:
        sigma = preconditioner_sigma(alpha, beta)
    u = np.asarray(u, dtype=np.float64)
    vec = u.ndim == 1
    U = np.ascontiguousarray(u.reshape(u.shape[0], -1))
    Lu = np.empty_like(U)
    if lib().tpo_bh_fractional(_d(V), V.shape[0], _i(F), F.shape[0], sigma, float(theta), int(leaf), _d(U),
                               U.shape[1], _d(Lu)) != 0:
        raise ValueError("k must be in [1, 64]")
    return Lu[:, 0] if vec else Lu


def bct_fractional_apply(V, F, u, chi, sigma=None, leaf=8, alpha=DEFAULT_ALPHA, beta=DEFAULT_BETA):
    """L^sigma u by the block cluster tree and hierarchical multiplication of Sec. 5.1.4 and
    5.1.5 (tpo_bct_fractional); chi = 0 is fractional_apply.  Returns (Lu, (admissible
    blocks, inadmissible blocks))."""
    V, F = _prep(V, F)
    if sigma is None:
        sigma = preconditioner_sigma(alpha, beta)
    u = np.asarray(u, dtype=np.float64)
    vec = u.ndim == 1
    U = np.ascontiguousarray(u.reshape(u.shape[0], -1))
    Lu = np.empty_like(U)
    cnt = np.zeros(2, dtype=np.int64)
    if lib().tpo_bct_fractional(_d(V), V.shape[0], _i(F), F.shape[0], sigma, float(chi), int(leaf), _d(U),
                                U.shape[1], _d(Lu), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))) != 0:
        raise ValueError("k must be in [1, 63]")
    return (Lu[:, 0] if vec else Lu), (int(cnt[0]), int(cnt[1]))
