"""Oracle of the dynamic remeshing of Sec. 6 (plain Python, test infrastructure only).

The paper's procedure, with L0 the target edge length:
  1. split every edge longer than 3 L0 / 2 and collapse every edge shorter than L0 / 2,
     unless the operation would fold a triangle over;
  2. N times: flip every edge that violates the Delaunay condition until none is left,
     then move every vertex by rho times the area-weighted mean of (circumcenter - vertex)
     over its faces, projected onto the vertex's tangent plane.
Readings (the paper gives the rules, not an order): edges are visited in the order of
their sorted vertex pairs (a < b) as they stand at the start of each pass, an edge is
tested with its current length when it is reached, and edges created during a pass wait
for the next pass; a split puts the new vertex at the midpoint and numbers it next; a
collapse keeps the smaller vertex index at the edge's midpoint and is refused when it would
flip the normal of a remaining face around either end or when the two ends share a
neighbour other than the two opposite vertices (the link condition that keeps the surface
a manifold); the Delaunay condition of an interior edge is that its two opposite angles sum
to at most pi, and a flip is refused when the new edge already exists; flipping sweeps
repeat until a sweep flips nothing (at most `max_sweeps`); the vertex normal of the
projection is the area-weighted mean of the face normals; vertices of boundary edges do
not move.  Faces keep their orientation throughout.  The output is compacted: surviving
vertices and faces in their order.
"""
from __future__ import annotations

import math

import numpy as np


def _edges(F):
    out = set()
    for f in F:
        if f is None:
            continue
        for c in range(3):
            a, b = f[c], f[(c + 1) % 3]
            out.add((min(a, b), max(a, b)))
    return sorted(out)


def _edge_faces(F):
    m = {}
    for q, f in enumerate(F):
        if f is None:
            continue
        for c in range(3):
            a, b = f[c], f[(c + 1) % 3]
            m.setdefault((min(a, b), max(a, b)), []).append(q)
    return m


def _normal(V, f):
    a, b, c = (np.asarray(V[i]) for i in f)
    return np.cross(b - a, c - a)


def _split_pass(V, F, L0):
    for (a, b) in _edges(F):
        ef = _edge_faces(F)
        if (a, b) not in ef:
            continue
        if np.linalg.norm(np.asarray(V[a]) - np.asarray(V[b])) <= 1.5 * L0:
            continue
        m = len(V)
        V.append(list(0.5 * (np.asarray(V[a]) + np.asarray(V[b]))))
        for q in ef[(a, b)]:
            f = F[q]
            c0 = [k for k in range(3) if f[k] not in (a, b)][0]
            x, y, z = f[c0], f[(c0 + 1) % 3], f[(c0 + 2) % 3]   # (z, x, y) cyclic: edge y -> z
            F[q] = [x, y, m]
            F.append([x, m, z])


def _collapse_ok(V, F, ef, a, b):
    na = {v for f in F if f is not None and a in f for v in f} - {a}
    nb = {v for f in F if f is not None and b in f for v in f} - {b}
    opp = {v for q in ef[(a, b)] for v in F[q]} - {a, b}
    if (na & nb) != opp:
        return False
    mid = 0.5 * (np.asarray(V[a]) + np.asarray(V[b]))
    for q, f in enumerate(F):
        if f is None or (a not in f and b not in f) or q in ef[(a, b)]:
            continue
        before = _normal(V, f)
        g = [a if v == b else v for v in f]
        W = {v: (mid if v == a else np.asarray(V[v])) for v in g}
        after = np.cross(W[g[1]] - W[g[0]], W[g[2]] - W[g[0]])
        if float(before @ after) <= 0.0:
            return False
    return True


def _collapse_pass(V, F, L0, alive):
    for (a, b) in _edges(F):
        ef = _edge_faces(F)
        if (a, b) not in ef or not alive[a] or not alive[b]:
            continue
        if np.linalg.norm(np.asarray(V[a]) - np.asarray(V[b])) >= 0.5 * L0:
            continue
        if not _collapse_ok(V, F, ef, a, b):
            continue
        V[a] = list(0.5 * (np.asarray(V[a]) + np.asarray(V[b])))
        for q in ef[(a, b)]:
            F[q] = None
        for q, f in enumerate(F):
            if f is not None and b in f:
                F[q] = [a if v == b else v for v in f]
        alive[b] = False


def _angle(p, q, r):
    """Angle at p of the triangle (p, q, r)."""
    u, w = np.asarray(q) - np.asarray(p), np.asarray(r) - np.asarray(p)
    return math.atan2(np.linalg.norm(np.cross(u, w)), float(u @ w))


def _flip_pass(V, F, max_sweeps):
    flips = 0
    for _ in range(max_sweeps):
        changed = 0
        for (a, b) in _edges(F):
            ef = _edge_faces(F)
            fs = ef.get((a, b), [])
            if len(fs) != 2:
                continue
            f1, f2 = F[fs[0]], F[fs[1]]
            c = [v for v in f1 if v not in (a, b)][0]
            d = [v for v in f2 if v not in (a, b)][0]
            if (min(c, d), max(c, d)) in ef or c == d:
                continue
            if _angle(V[c], V[a], V[b]) + _angle(V[d], V[a], V[b]) <= math.pi:
                continue
            # face fs[0] holds the edge as p -> q (then c); replace the pair by (c, d) faces
            k = f1.index(c)
            p, q = f1[(k + 1) % 3], f1[(k + 2) % 3]
            F[fs[0]] = [c, p, d]
            F[fs[1]] = [d, q, c]
            changed += 1
        flips += changed
        if changed == 0:
            break
    return flips


def _circumcenter(a, b, c):
    a, b, c = (np.asarray(x, dtype=float) for x in (a, b, c))
    u, w = b - a, c - a
    n = np.cross(u, w)
    return a + (np.cross(n, u) * (w @ w) + np.cross(w, n) * (u @ u)) / (2.0 * (n @ n))


def _smooth(V, F, rho, alive):
    nV = len(V)
    num = [np.zeros(3) for _ in range(nV)]
    den = [0.0] * nV
    nrm = [np.zeros(3) for _ in range(nV)]
    ef = _edge_faces(F)
    fixed = set()
    for (a, b), fs in ef.items():
        if len(fs) != 2:
            fixed.update((a, b))
    for f in F:
        if f is None:
            continue
        n = _normal(V, f)
        area = 0.5 * np.linalg.norm(n)
        cc = _circumcenter(V[f[0]], V[f[1]], V[f[2]])
        for v in f:
            num[v] = num[v] + area * (cc - np.asarray(V[v]))
            den[v] += area
            nrm[v] = nrm[v] + 0.5 * n            # area-weighted: |n| / 2 times the unit normal
    out = [list(x) for x in V]
    for v in range(nV):
        if not alive[v] or den[v] == 0.0 or v in fixed:
            continue
        u = rho * num[v] / den[v]
        N = nrm[v] / np.linalg.norm(nrm[v])
        u = u - (u @ N) * N
        out[v] = list(np.asarray(V[v]) + u)
    V[:] = out


def remesh(V, F, L0, iterations=5, rho=0.5, max_sweeps=64):
    """Returns (V, F) after one application of the procedure (numpy arrays, compacted)."""
    V = [list(map(float, x)) for x in np.asarray(V)]
    F = [list(map(int, f)) for f in np.asarray(F)]
    _split_pass(V, F, L0)
    alive = [True] * len(V)
    _collapse_pass(V, F, L0, alive)
    for _ in range(iterations):
        _flip_pass(V, F, max_sweeps)
        _smooth(V, F, rho, alive)
    keep = [v for v in range(len(V)) if alive[v]]
    new = {v: i for i, v in enumerate(keep)}
    Vo = np.array([V[v] for v in keep], dtype=np.float64)
    Fo = np.array([[new[v] for v in f] for f in F if f is not None], dtype=np.int32)
    return Vo, Fo
