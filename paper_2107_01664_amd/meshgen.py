"""Seeded synthetic triangle meshes.

This module only builds inputs: vertex positions (float64, nV x 3, row-major) and
faces (int32, nF x 3, 0-based, consistently oriented with outward normals).  It
holds none of the tangent-point method's arithmetic, so both the HIP path and the
CPU oracle can be fed from it.

Shapes follow the workloads of the paper: closed genus-0 and genus-1 surfaces of
10^3 - 10^5 triangles, several components, and smooth bumpy shapes.  The paper's
own meshes are not available; these stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Mesh", "icosahedron", "icosphere", "geodesic_sphere", "torus", "add_noise",
    "linked_tori", "bumpy_sphere", "mean_edge_length", "serving_requests",
    "workload", "random_columns", "build_request_mesh",
]


@dataclass
class Mesh:
    V: np.ndarray  # (nV, 3) float64
    F: np.ndarray  # (nF, 3) int32

    @property
    def nV(self) -> int:
        return int(self.V.shape[0])

    @property
    def nF(self) -> int:
        return int(self.F.shape[0])

    def copy(self) -> "Mesh":
        return Mesh(self.V.copy(), self.F.copy())


def _mesh(V, F) -> Mesh:
    return Mesh(np.ascontiguousarray(V, dtype=np.float64),
                np.ascontiguousarray(F, dtype=np.int32))


def icosahedron() -> Mesh:
    """Regular icosahedron inscribed in the unit sphere (12 vertices, 20 faces)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int32)
    return _mesh(V, F)


def icosphere(level: int, radius: float = 1.0) -> Mesh:
    """Icosphere by midpoint subdivision: every level splits each face 1->4 at edge
    midpoints and projects the new vertices onto the sphere.  F = 20*4^L, V = 10*4^L+2."""
    m = icosahedron()
    V = [tuple(v) for v in m.V]
    F = m.F.tolist()
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = (np.asarray(V[a]) + np.asarray(V[b])) * 0.5
                p = p / np.linalg.norm(p)
                idx = len(V)
                V.append(tuple(p))
                cache[key] = idx
            return idx

        newF = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            newF += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        F = newF
    return _mesh(np.asarray(V) * radius, np.asarray(F))


def geodesic_sphere(freq: int, radius: float = 1.0) -> Mesh:
    """Frequency-n geodesic sphere: a barycentric grid on every icosahedron face,
    welded along edges and projected to the sphere.  F = 20 n^2, V = 10 n^2 + 2."""
    n = int(freq)
    if n < 1:
        raise ValueError("freq must be >= 1")
    ico = icosahedron()
    keys: dict[tuple, int] = {}
    V: list[np.ndarray] = []

    def vid(corners, w) -> int:
        key = tuple(sorted((int(c), int(x)) for c, x in zip(corners, w) if x != 0))
        idx = keys.get(key)
        if idx is None:
            p = sum(ico.V[c] * (x / n) for c, x in zip(corners, w))
            p = p / np.linalg.norm(p)
            idx = len(V)
            V.append(p)
            keys[key] = idx
        return idx

    F = []
    for A, B, C in ico.F:
        corners = (A, B, C)
        grid = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                k = n - i - j
                grid[(i, j)] = vid(corners, (k, i, j))  # weight k on A, i on B, j on C
        for i in range(n):
            for j in range(n - i):
                a, b, c = grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]
                F.append([a, b, c])
                if i + j < n - 1:
                    F.append([b, grid[(i + 1, j + 1)], c])
    return _mesh(np.asarray(V) * radius, np.asarray(F))


def torus(nu: int, nv: int, R: float = 1.0, r: float = 0.3) -> Mesh:
    """Torus of revolution sampled on an nu x nv grid, u = 2 pi i/nu around the core
    circle, v = 2 pi j/nv around the tube.  Quad (i,j),(i+1,j),(i+1,j+1),(i,j+1) is cut
    along its (i,j)-(i+1,j+1) diagonal; faces are oriented outward.  F = 2 nu nv."""
    i = np.arange(nu)[:, None]
    j = np.arange(nv)[None, :]
    u = 2.0 * np.pi * i / nu
    v = 2.0 * np.pi * j / nv
    x = (R + r * np.cos(v)) * np.cos(u)
    y = (R + r * np.cos(v)) * np.sin(u)
    z = r * np.sin(v) * np.ones_like(u)
    V = np.stack([x, y, z], axis=-1).reshape(-1, 3)
    ii, jj = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = ii * nv + jj
    b = ((ii + 1) % nu) * nv + jj
    c = ((ii + 1) % nu) * nv + (jj + 1) % nv
    d = ii * nv + (jj + 1) % nv
    # interleave the two triangles of each quad so neighbouring faces stay close in memory
    F = np.stack([np.stack([a, b, c], -1).reshape(-1, 3),
                  np.stack([a, c, d], -1).reshape(-1, 3)], axis=1).reshape(-1, 3)
    return _mesh(V, F)


def add_noise(mesh: Mesh, sigma: float, seed: int) -> Mesh:
    """x_v += sigma * xi_v with xi_v ~ N(0, I_3) i.i.d. per vertex (numpy default_rng(seed))."""
    rng = np.random.default_rng(seed)
    return _mesh(mesh.V + sigma * rng.standard_normal(mesh.V.shape), mesh.F)


def mean_edge_length(mesh: Mesh) -> float:
    V, F = mesh.V, mesh.F
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(V[e[:, 0]] - V[e[:, 1]], axis=1).mean())


def linked_tori(nu: int = 160, nv: int = 80, R: float = 1.0, r: float = 0.25,
                offset: float = 1.0) -> Mesh:
    """Two interlinked tori.  Torus B is torus A rotated +90 degrees about x,
    (x,y,z) -> (x,-z,y), then shifted by `offset` along x.  With R = offset = 1 the two
    core circles stay exactly 1 apart, so the tubes are 1 - 2r apart everywhere."""
    A = torus(nu, nv, R, r)
    VB = np.stack([A.V[:, 0] + offset, -A.V[:, 2], A.V[:, 1]], axis=1)
    V = np.concatenate([A.V, VB])
    F = np.concatenate([A.F, A.F + A.nV])
    return _mesh(V, F)


def _real_sph_harm(l: int, m: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    Y = sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2.0) * (np.real(Y) if m > 0 else np.imag(Y))


def bumpy_sphere(level: int = 7, lmax: int = 8, amplitude: float = 0.05, seed: int = 0) -> Mesh:
    """Icosphere of the given level with radial low-frequency bumps:
    r(v) = 1 + amplitude * b(v)/max|b|, b = sum_{l<=lmax} sum_m c_lm Y_lm(v) with real
    spherical harmonics and c_lm ~ N(0,1) drawn in (l, m) order from default_rng(seed)."""
    m = icosphere(level)
    rng = np.random.default_rng(seed)
    x, y, z = m.V.T
    theta = np.arccos(np.clip(z, -1.0, 1.0))  # polar
    phi = np.arctan2(y, x)                    # azimuth
    b = np.zeros(m.nV)
    for l in range(lmax + 1):
        for mm in range(-l, l + 1):
            b += rng.standard_normal() * _real_sph_harm(l, mm, theta, phi)
    rad = 1.0 + amplitude * b / np.abs(b).max()
    return _mesh(m.V * rad[:, None], m.F)


def serving_requests(n: int = 512, seed: int = 0, fmin: float = 2000.0,
                     fmax: float = 200000.0, steps: int = 10):
    """Request mix for the serving workload: each request is a noisy icosphere or torus
    (probability 1/2 each) whose triangle count F* is log-uniform in [fmin, fmax].
    Icosphere: geodesic frequency round(sqrt(F*/20)) clipped to [10, 100].  Torus:
    nv = round(sqrt(F*/4)), nu = 2 nv, R = 1, r = 0.3.  Noise sigma = 0.01 x mean edge
    length, seeded per request.  Returns a list of dicts (the meshes are built lazily)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        kind = "sphere" if rng.random() < 0.5 else "torus"
        fstar = math.exp(rng.uniform(math.log(fmin), math.log(fmax)))
        if kind == "sphere":
            freq = int(min(100, max(10, round(math.sqrt(fstar / 20.0)))))
            spec = {"kind": kind, "freq": freq, "nF": 20 * freq * freq}
        else:
            nv = max(3, int(round(math.sqrt(fstar / 4.0))))
            spec = {"kind": kind, "nu": 2 * nv, "nv": nv, "nF": 4 * nv * nv}
        spec.update({"id": q, "seed": seed * 100003 + q, "steps": steps})
        out.append(spec)
    return out


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate (requests/s):
    cumulative sums of exponential gaps, default_rng(seed); rate = inf gives all zeros."""
    if not math.isfinite(rate):
        return np.zeros(n)
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def build_request_mesh(spec: dict) -> Mesh:
    if spec["kind"] == "sphere":
        m = geodesic_sphere(spec["freq"])
    else:
        m = torus(spec["nu"], spec["nv"], 1.0, 0.3)
    return add_noise(m, 0.01 * mean_edge_length(m), spec["seed"])


def workload(name: str) -> Mesh:
    """The named synthetic workloads.

    small_sphere : icosphere level 3 (642 vertices, 1,280 faces), noise 0.01, seed 0
    torus40k     : torus R=1, r=0.3 on a 200 x 100 grid (40,000 faces), noise 0.002 r, seed 0
    linked_tori  : two linked tori R=1, r=0.25, 160 x 80 each (51,200 faces), no noise
    bumpy327k    : icosphere level 7 (327,680 faces) with l<=8 harmonic bumps of amplitude 0.05
    """
    if name == "small_sphere":
        return add_noise(icosphere(3), 0.01, 0)
    if name == "torus40k":
        return add_noise(torus(200, 100, 1.0, 0.3), 0.002 * 0.3, 0)
    if name == "linked_tori":
        return linked_tori(160, 80, 1.0, 0.25, 1.0)
    if name == "bumpy327k":
        return bumpy_sphere(7, 8, 0.05, 0)
    raise KeyError(name)


def random_columns(nV: int, k: int, seed: int) -> np.ndarray:
    """u ~ N(0,1) per vertex and column, row-major (nV, k), default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((nV, k)))
