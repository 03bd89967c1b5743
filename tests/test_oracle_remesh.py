"""Dynamic remeshing (Sec. 6): the oracle pinned to hand-derived results of single
operations (a split, a flip, a collapse, a refused collapse), to symmetry (smoothing does
not move the vertices of regular meshes) and to invariants of the whole procedure
(Euler characteristic, a consistently oriented manifold, the Delaunay condition after the
flips, tangential motion); then the library's host remesher (tp_remesh, through the C-ABI)
against the oracle: identical faces, positions to rounding.  Runs without a GPU."""
import math
import os

import numpy as np
import pytest

from oracle.remesh import remesh
from paper_2107_01664_amd import meshgen as mg

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2107_01664_amd",
                   "libtpsurf.so")


def edge_faces(F):
    m = {}
    for q, f in enumerate(F):
        for c in range(3):
            a, b = int(f[c]), int(f[(c + 1) % 3])
            m.setdefault((min(a, b), max(a, b)), []).append(q)
    return m


def check_manifold(F, closed=True):
    """Every edge borders two faces (one or two if open), every directed edge appears once
    (consistent orientation), no face repeats a vertex."""
    directed = set()
    for f in F:
        assert len(set(map(int, f))) == 3
        for c in range(3):
            e = (int(f[c]), int(f[(c + 1) % 3]))
            assert e not in directed
            directed.add(e)
    counts = [len(v) for v in edge_faces(F).values()]
    assert all(c == 2 for c in counts) if closed else all(c in (1, 2) for c in counts)
    return len(edge_faces(F))


def euler(V, F):
    return len(V) - len(edge_faces(F)) + len(F)


def angle(p, q, r):
    u, w = q - p, r - p
    return math.atan2(np.linalg.norm(np.cross(u, w)), u @ w)


def max_opposite_angle_sum(V, F):
    worst = 0.0
    for (a, b), fs in edge_faces(F).items():
        if len(fs) != 2:
            continue
        c = [v for v in F[fs[0]] if v not in (a, b)][0]
        d = [v for v in F[fs[1]] if v not in (a, b)][0]
        worst = max(worst, angle(V[c], V[a], V[b]) + angle(V[d], V[a], V[b]))
    return worst


def signed_volume(V, F):
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def test_single_split():
    """Two triangles on a long shared edge (length 3, the others 1.80; L0 = 1.5): only the
    shared edge exceeds 1.5 L0; it is split at its midpoint, each face into two, and the new
    edges (1 and 1.5) are inside [L0/2, 3L0/2], so nothing else changes."""
    V = np.array([[0, 0, 0], [3, 0, 0], [1.5, 1, 0], [1.5, -1, 0]], float)
    F = np.array([[0, 1, 2], [1, 0, 3]], np.int32)
    V1, F1 = remesh(V, F, 1.5, iterations=0)
    assert np.array_equal(V1, np.vstack([V, [[1.5, 0, 0]]]))
    assert F1.tolist() == [[2, 0, 4], [3, 1, 4], [2, 4, 1], [3, 4, 0]]


def test_single_flip():
    """A thin kite: the diagonal (0, 1) has opposite angles of 157.4 degrees each (sum above
    pi), so it is replaced by the diagonal (2, 3) with the orientation kept; the vertices
    all lie on boundary edges and stay."""
    V = np.array([[0, 0, 0], [2, 0, 0], [1, 0.2, 0], [1, -0.2, 0]], float)
    F = np.array([[0, 1, 2], [1, 0, 3]], np.int32)
    V1, F1 = remesh(V, F, 1.4, iterations=1)
    assert np.array_equal(V1, V)
    assert F1.tolist() == [[2, 0, 3], [3, 1, 2]]
    n = np.cross(V[F1[:, 1]] - V[F1[:, 0]], V[F1[:, 2]] - V[F1[:, 0]])
    assert (n[:, 2] > 0).all()


def test_single_collapse_icosahedron():
    """Icosahedron (edge 1.05) with vertex b moved 60% of the way to its neighbour a: edge
    (a, b) has length 0.4 L0 and all others stay within [L0/2, 3L0/2] (second neighbours
    of b at 1.32 L0 at most), so exactly that edge collapses, to its midpoint at vertex a:
    11 vertices, 18 faces, still a closed oriented sphere."""
    m = mg.icosahedron()
    V = m.V.copy()
    L0 = float(np.linalg.norm(V[m.F[0, 0]] - V[m.F[0, 1]]))
    a, b = sorted(map(int, m.F[0, :2]))
    V[b] = V[b] + 0.6 * (V[a] - V[b])
    mid = 0.5 * (V[a] + V[b])
    V1, F1 = remesh(V, m.F, L0, iterations=0)
    assert len(V1) == 11 and len(F1) == 18
    assert np.array_equal(V1[a], mid)
    assert np.array_equal(np.delete(V1, a, axis=0), np.delete(np.delete(V, b, axis=0), a, axis=0))
    check_manifold(F1)
    assert euler(V1, F1) == 2 and signed_volume(V1, F1) > 0


def test_link_condition_refuses_every_collapse():
    """The seven-vertex torus (triangles {i, i+1, i+3} and {i, i+2, i+3} mod 7) joins every
    pair of vertices by an edge, so the ends of any edge share five neighbours but only two
    opposite vertices: every collapse would leave a non-manifold surface and is refused,
    even with every edge far below L0/2."""
    F = np.array([[i, (i + 1) % 7, (i + 3) % 7] for i in range(7)] +
                 [[i, (i + 2) % 7, (i + 3) % 7] for i in range(7)], np.int32)
    assert len(edge_faces(F)) == 21 and all(len(v) == 2 for v in edge_faces(F).values())
    V = np.random.default_rng(3).standard_normal((7, 3))
    V1, F1 = remesh(V, F, 1e3, iterations=0)
    assert np.array_equal(V1, V) and np.array_equal(F1, F)


@pytest.mark.parametrize("kind", ["icosahedron", "flat_grid"])
def test_smoothing_fixes_regular_meshes(kind):
    """On the icosahedron every vertex is equivalent, so the weighted circumcenter mean lies
    on the normal line and its tangential part vanishes; on a regular flat triangle grid the
    six circumcenters around an interior vertex are symmetric about it, and the boundary
    stays.  No edge is split, collapsed or flipped (the meshes are Delaunay, with opposite
    angles summing to 2 pi / 3)."""
    if kind == "icosahedron":
        m = mg.icosahedron()
        V, F = m.V, m.F
    else:
        n = 5
        V = np.array([[i + 0.5 * j, j * math.sqrt(3) / 2, 0.0] for j in range(n) for i in range(n)])
        F = []
        for j in range(n - 1):
            for i in range(n - 1):
                v = j * n + i
                F += [[v, v + 1, v + n], [v + 1, v + n + 1, v + n]]
        F = np.array(F, np.int32)
    L0 = float(np.linalg.norm(V[F[0, 0]] - V[F[0, 1]]))
    V1, F1 = remesh(V, F, L0, iterations=2, rho=0.5)
    assert np.array_equal(F1, F)
    assert np.abs(V1 - V).max() <= 1e-14


def test_smoothing_is_tangential_and_restoring():
    """A flat regular fan with its centre moved within the plane: the centre moves back
    toward the centroid of the ring, stays in the plane (the projection removes the normal
    part) and the ring (boundary) stays."""
    ring = np.array([[math.cos(k * math.pi / 3), math.sin(k * math.pi / 3), 0.0] for k in range(6)])
    V = np.vstack([[[0.12, -0.07, 0.0]], ring])
    F = np.array([[0, 1 + k, 1 + (k + 1) % 6] for k in range(6)], np.int32)
    V1, F1 = remesh(V, F, 1.0, iterations=1, rho=0.5)
    assert np.array_equal(F1, F) and np.array_equal(V1[1:], ring)
    assert V1[0, 2] == 0.0 and np.linalg.norm(V1[0]) < np.linalg.norm(V[0])


def stretched_sphere(level, seed):
    """A noisy icosphere stretched to an ellipsoid 1 x 1 x 2.5: edges from about 0.47 to
    1.9 times the mean, so that one application both splits (about 40 edges at level 2)
    and collapses (10 to 20)."""
    m = mg.add_noise(mg.icosphere(level), 0.02, seed)
    V = m.V * np.array([1.0, 1.0, 2.5])
    return V, m.F


def test_invariants_of_the_procedure():
    """Splits and collapses keep a closed oriented manifold of genus 0; after the final
    flips (rho = 0, so the smoothing moves nothing) every interior edge satisfies the
    Delaunay condition; the long edges are fewer; the enclosed volume changes little."""
    V, F = stretched_sphere(2, 5)
    L0 = float(np.mean([np.linalg.norm(V[a] - V[b]) for a, b in edge_faces(F)]))
    long0 = sum(np.linalg.norm(V[a] - V[b]) > 1.5 * L0 for a, b in edge_faces(F))
    V1, F1 = remesh(V, F, L0, iterations=1, rho=0.0)
    check_manifold(F1)
    assert euler(V1, F1) == 2
    assert len(V1) != len(V)
    assert max_opposite_angle_sum(V1, F1) <= math.pi + 1e-12
    long1 = sum(np.linalg.norm(V1[a] - V1[b]) > 1.5 * L0 for a, b in edge_faces(F1))
    assert long1 < long0
    vol0, vol1 = signed_volume(V, F), signed_volume(V1, F1)
    assert vol1 > 0 and abs(vol1 - vol0) <= 0.03 * vol0


def test_tangential_smoothing_on_a_curved_surface():
    """One smoothing step on a noisy sphere moves each vertex orthogonally to its
    area-weighted normal (computed here independently from the input mesh)."""
    m = mg.add_noise(mg.icosphere(2), 0.02, 11)
    L0 = mg.mean_edge_length(m)
    V1, F1 = remesh(m.V, m.F, L0, iterations=1, rho=0.5)
    # edges from 0.73 to 1.32 L0: no split or collapse; the normals are those of the mesh
    # the smoothing saw (after the flips, which move no vertex)
    assert len(V1) == len(m.V) and len(F1) == len(m.F)
    n = np.zeros_like(m.V)
    fn = np.cross(m.V[F1[:, 1]] - m.V[F1[:, 0]], m.V[F1[:, 2]] - m.V[F1[:, 0]])
    for c in range(3):
        np.add.at(n, F1[:, c], fn)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    d = V1 - m.V
    assert np.abs(np.einsum("ij,ij->i", d, n)).max() <= 1e-12 * max(1.0, np.abs(d).max())
    assert np.abs(d).max() > 1e-4


# ----------------------------------------------------------------- library vs oracle

@pytest.fixture(scope="module")
def tp():
    if not os.path.exists(LIB):
        pytest.skip("libtpsurf.so not built")
    from paper_2107_01664_amd import tpsurf
    tpsurf.lib()
    return tpsurf


def open_sheet(n, seed):
    """A noisy, non-uniform open grid (boundary edges, unequal edge lengths)."""
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.uniform(0.3, 1.7, n))
    y = np.cumsum(rng.uniform(0.3, 1.7, n))
    V = np.array([[x[i], y[j], 0.2 * rng.standard_normal()] for j in range(n) for i in range(n)])
    F = []
    for j in range(n - 1):
        for i in range(n - 1):
            v = j * n + i
            F += [[v, v + 1, v + n + 1], [v, v + n + 1, v + n]]
    return V, np.array(F, np.int32)


@pytest.mark.parametrize("case", ["ellipsoid", "torus", "sheet"])
def test_library_matches_oracle(tp, case):
    if case == "ellipsoid":
        V, F = stretched_sphere(2, 7)
    elif case == "torus":
        m = mg.add_noise(mg.torus(16, 8, 1.0, 0.35), 0.03, 4)
        V, F = m.V, m.F
    else:
        V, F = open_sheet(9, 2)
    L0 = float(np.mean([np.linalg.norm(V[a] - V[b]) for a, b in edge_faces(F)]))
    V0, F0 = remesh(V, F, L0, iterations=3, rho=0.5)
    V1, F1 = tp.tp_remesh(V, F, L0, iterations=3, rho=0.5)
    assert (len(V0), len(F0)) != (len(V), len(F)) or not np.array_equal(F0, F)
    assert np.array_equal(F1, F0)
    assert np.abs(V1 - V0).max() <= 1e-12 * np.abs(V0).max()


def test_library_errors_and_capacity(tp):
    V, F = stretched_sphere(1, 1)
    L0 = 0.5 * float(np.mean([np.linalg.norm(V[a] - V[b]) for a, b in edge_faces(F)]))
    with pytest.raises(tp.TpError, match="INVALID_ARGUMENT"):
        tp.tp_remesh(V, F, 0.0)
    with pytest.raises(tp.TpError, match="INVALID_ARGUMENT"):
        tp.tp_remesh(V, F, L0, rho=1.0)
    Fb = F.copy()
    Fb[3, 1] = len(V)
    with pytest.raises(tp.TpError, match="BAD_INDEX"):
        tp.tp_remesh(V, Fb, L0)
    Vn = V.copy()
    Vn[2, 0] = np.nan
    with pytest.raises(tp.TpError, match="NONFINITE"):
        tp.tp_remesh(Vn, F, L0)
    # too-small outputs report the sizes the result needs
    import ctypes
    nv, nf = ctypes.c_int64(), ctypes.c_int64()
    Vo, Fo = np.empty((4, 3)), np.empty((4, 3), np.int32)
    st = tp.lib().tp_remesh(V.ctypes.data, len(V), np.ascontiguousarray(F, np.int32).ctypes.data, len(F), L0, 1,
                            0.5, Vo.ctypes.data, 4, Fo.ctypes.data, 4, ctypes.byref(nv), ctypes.byref(nf))
    assert st != 0
    V1, F1 = tp.tp_remesh(V, F, L0, iterations=1)
    assert (nv.value, nf.value) == (len(V1), len(F1)) and len(F1) > len(F)
