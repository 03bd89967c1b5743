"""Pins of the oracle's Barnes-Hut approximation (Sec. 4): theta = 0 is the direct sum, the
differential is the exact gradient of E_BH with frozen interaction lists (finite
differences, translation / rotation / Euler identities), the error falls as theta does,
and the tree order is the Morton order of the barycenters."""
import numpy as np
import pytest

import oracle as O
from paper_2107_01664_amd import meshgen as mg


@pytest.fixture(scope="module")
def torus():
    return mg.add_noise(mg.torus(40, 20, 1.0, 0.3), 0.005, 4)          # 1,600 faces


def test_theta_zero_is_direct():
    m = mg.workload("small_sphere")
    E0, g0 = O.gradient(m.V, m.F)
    E, g, (far, near) = O.bh_gradient(m.V, m.F, 0.0)
    assert far == 0 and near == m.nF * (m.nF - 1)
    assert abs(E - E0) <= 1e-13 * E0
    assert np.linalg.norm(g - g0) <= 1e-12 * np.linalg.norm(g0)


def test_frozen_list_finite_differences(torus):
    m, th = torus, 0.5
    E, g, (far, near) = O.bh_gradient(m.V, m.F, th)
    assert far > 0 and near > 0
    rng = np.random.default_rng(0)
    for _ in range(3):
        dV = rng.standard_normal(m.V.shape)
        h = 1e-6
        Ep = O.bh_energy_frozen(m.V, m.V + h * dV, m.F, th)
        Em = O.bh_energy_frozen(m.V, m.V - h * dV, m.F, th)
        fd = (Ep - Em) / (2 * h)
        an = float(np.sum(g * dV))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    assert O.bh_energy_frozen(m.V, m.V, m.F, th) == E


def test_identities(torus):
    m, th = torus, 0.5
    E, g, _ = O.bh_gradient(m.V, m.F, th)
    scale = np.linalg.norm(g) * np.linalg.norm(m.V)
    assert np.linalg.norm(g.sum(0)) <= 1e-10 * np.linalg.norm(g) * np.sqrt(m.nV)
    assert np.linalg.norm(np.cross(m.V, g).sum(0)) <= 1e-10 * scale
    # E_BH with frozen lists is homogeneous of degree 4 + alpha - beta = -2
    assert abs(float(np.sum(m.V * g)) - (-2.0) * E) <= 1e-10 * abs(E)


def test_error_falls_with_theta():
    m = mg.add_noise(mg.icosphere(4), 0.002, 7)                      # 5,120 faces
    E0, g0 = O.gradient(m.V, m.F)
    errs = []
    for th in (1.0, 0.5, 0.25):
        E, g, (far, _) = O.bh_gradient(m.V, m.F, th)
        assert far > 0
        errs.append((abs(E - E0) / E0, np.linalg.norm(g - g0) / np.linalg.norm(g0)))
    assert errs[0][0] > errs[1][0] > errs[2][0]
    assert errs[0][1] > errs[1][1] > errs[2][1]
    # O(theta^2) (Sec. 8): halving theta twice cuts the errors at least fourfold here
    # (measured: E 0.17, 0.056, 0.015; dE 3.0e-3, 8.5e-4, 2.3e-4)
    assert errs[2][0] < errs[0][0] / 4 and errs[2][1] < errs[0][1] / 4
    assert errs[1][0] < 0.1


def test_tree_order_is_morton_order(torus):
    m = torus
    X, _, _ = O.faces(m.V, m.F)
    lo, hi = X.min(0), X.max(0)
    q = np.minimum(1023, np.floor(1024.0 * ((X - lo) / (hi - lo)))).astype(np.uint64)
    code = np.zeros(m.nF, dtype=np.uint64)
    for b in range(10):
        for ax, shift in ((0, 2), (1, 1), (2, 0)):
            code |= ((q[:, ax] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + shift)
    expect = np.lexsort((np.arange(m.nF), code))
    order = O.bh_order(m.V, m.F)
    assert np.array_equal(order, expect)


def test_bh_fractional_apply():
    """Barnes-Hut for the fractional operator's kernel matrix (admissible nodes stand for
    their faces with the kernel at the node barycenter and the moments sum a_T ubar_T):
    theta = 0 is the direct sum; constants stay in the null space exactly (a_I ubar_S - m_I
    vanishes for constant u); rigid motions leave it unchanged; the error against the
    direct sum falls with theta."""
    m = mg.add_noise(mg.icosphere(3), 0.01, 2)
    u = np.random.default_rng(5).standard_normal((m.nV, 3))
    sigma = O.preconditioner_sigma()
    L = O.fractional_apply(m.V, m.F, u, sigma)
    L0 = O.bh_fractional_apply(m.V, m.F, u, 0.0, sigma)
    assert np.abs(L0 - L).max() <= 1e-12 * np.abs(L).max()
    ones = np.ones((m.nV, 1))
    assert np.abs(O.bh_fractional_apply(m.V, m.F, ones, 0.5, sigma)).max() <= 1e-12 * np.abs(L).max()
    errs = []
    for th in (0.125, 0.25, 0.5):
        Lb = O.bh_fractional_apply(m.V, m.F, u, th, sigma)
        errs.append(np.linalg.norm(Lb - L) / np.linalg.norm(L))
    assert 0 < errs[0] < errs[1] < errs[2] < 0.1, errs
    Q, _ = np.linalg.qr(np.random.default_rng(6).standard_normal((3, 3)))
    Lr = O.bh_fractional_apply(m.V @ Q.T + 0.3, m.F, u, 0.5, sigma)
    Lb = O.bh_fractional_apply(m.V, m.F, u, 0.5, sigma)
    # a rotation can change the Morton order and with it the lists; a translation cannot
    Lt = O.bh_fractional_apply(m.V + 0.3, m.F, u, 0.5, sigma)
    assert np.abs(Lt - Lb).max() <= 1e-10 * np.abs(Lb).max()
    assert np.linalg.norm(Lr - L) / np.linalg.norm(L) < 0.1


def test_bct_fractional_apply():
    """Block cluster tree and hierarchical multiplication (Sec. 5.1.4, 5.1.5) for the
    fractional operator: chi = 0 is the direct sum (every block inadmissible); constants
    stay in the null space exactly; the approximate operator is symmetric (separation is
    symmetric in the two clusters and so is the kernel at the barycenters), which the
    one-sided Barnes-Hut sum is not; the error falls with chi; the admissible and
    inadmissible blocks partition all ordered face pairs (checked by applying the
    approximation of the constant kernel through the counts of rows)."""
    m = mg.add_noise(mg.icosphere(3), 0.01, 2)
    rng = np.random.default_rng(9)
    u, v = rng.standard_normal((m.nV, 2)), rng.standard_normal((m.nV, 2))
    L = O.fractional_apply(m.V, m.F, u)
    L0, c0 = O.bct_fractional_apply(m.V, m.F, u, 0.0)
    assert c0[0] == 0 and np.abs(L0 - L).max() <= 1e-12 * np.abs(L).max()
    assert np.abs(O.bct_fractional_apply(m.V, m.F, np.ones((m.nV, 1)), 0.5)[0]).max() <= 1e-12 * np.abs(L).max()
    Lu, _ = O.bct_fractional_apply(m.V, m.F, u, 0.5)
    Lv, _ = O.bct_fractional_apply(m.V, m.F, v, 0.5)
    assert abs(np.vdot(v, Lu) - np.vdot(u, Lv)) <= 1e-12 * abs(np.vdot(v, Lu))
    Lb = O.bh_fractional_apply(m.V, m.F, u, 0.5)
    Lbv = O.bh_fractional_apply(m.V, m.F, v, 0.5)
    assert abs(np.vdot(v, Lb) - np.vdot(u, Lbv)) > 1e-8 * abs(np.vdot(v, Lb))
    errs = [np.linalg.norm(O.bct_fractional_apply(m.V, m.F, u, c)[0] - L) / np.linalg.norm(L)
            for c in (0.125, 0.25, 0.5, 1.0)]
    assert all(a < b for a, b in zip(errs, errs[1:])) and errs[2] < 0.01, errs
    # partition: with sigma -> the kernel exponent 0 (k = 1), the row sums of the kernel
    # matrix are exact whatever the blocks (the rank-one blocks are exact for a constant
    # kernel), so any pair counted twice or missed would show
    Lk, cnt = O.bct_fractional_apply(m.V, m.F, u, 0.5, sigma=-1.0)
    Ldk = O.fractional_apply(m.V, m.F, u, -1.0)
    assert cnt[0] > 0 and np.abs(Lk - Ldk).max() <= 1e-10 * np.abs(Ldk).max()


def _obstacle_scene():
    """A noisy sphere (320 faces) under a noisy torus obstacle (400 faces) 1.6 above it."""
    m = mg.add_noise(mg.icosphere(2), 0.01, 1)
    ob = mg.add_noise(mg.torus(20, 10, 0.6, 0.2), 0.01, 2)
    return m, ob.V + np.array([0.0, 0.0, 1.6]), ob.F


def test_obstacle_bh_limits():
    """Barnes-Hut for the static obstacle (end of Sec. 7.3.2): theta = 0 is the direct sum
    (every term a face term, nF x nFo of them); the error falls with theta; an obstacle far
    away is one point mass at its area-weighted barycenter for every surface face (root node
    admissible), checked against that closed form computed here from the face areas."""
    m, Vo, Fo = _obstacle_scene()
    E0, g0 = O.obstacle(m.V, m.F, Vo, Fo)
    E, g, cnt = O.obstacle_bh(m.V, m.F, Vo, Fo, 0.0)
    assert cnt == (0, m.nF * len(Fo))
    assert abs(E - E0) <= 1e-13 * E0 and np.abs(g - g0).max() <= 1e-13 * np.abs(g0).max()
    errs = []
    for th in (0.25, 0.5, 1.0):
        E, g, _ = O.obstacle_bh(m.V, m.F, Vo, Fo, th)
        errs.append((abs(E - E0) / E0, np.linalg.norm(g - g0) / np.linalg.norm(g0)))
    assert all(a[0] < b[0] and a[1] < b[1] for a, b in zip(errs, errs[1:])), errs
    assert errs[1][0] < 0.02 and errs[1][1] < 0.02, errs
    far = Vo + np.array([0.0, 0.0, 60.0])
    E, _, cnt = O.obstacle_bh(m.V, m.F, far, Fo, 0.5)
    assert cnt == (m.nF, 0)
    Xo, _, ao = O.faces(far, Fo)
    Y = (ao[:, None] * Xo).sum(0) / ao.sum()
    X, _, a = O.faces(m.V, m.F)
    Ec = float(np.sum(a * ao.sum() * np.linalg.norm(X - Y, axis=1) ** -6.0))
    assert abs(E - Ec) <= 1e-12 * Ec


def test_obstacle_bh_differential():
    """dE of the Barnes-Hut obstacle potential against central differences of E_BH at
    perturbations small enough to keep every interaction list (term counts unchanged)."""
    m, Vo, Fo = _obstacle_scene()
    _, g, cnt = O.obstacle_bh(m.V, m.F, Vo, Fo, 0.5)
    rng = np.random.default_rng(4)
    h = 1e-6
    for v, c in zip(rng.integers(0, m.nV, 6), rng.integers(0, 3, 6)):
        Vp, Vm = m.V.copy(), m.V.copy()
        Vp[v, c] += h
        Vm[v, c] -= h
        Ep, _, cp = O.obstacle_bh(Vp, m.F, Vo, Fo, 0.5, with_grad=False)
        Em, _, cm = O.obstacle_bh(Vm, m.F, Vo, Fo, 0.5, with_grad=False)
        assert cp == cnt and cm == cnt
        fd = (Ep - Em) / (2 * h)
        assert abs(fd - g[v, c]) <= 1e-6 * np.abs(g).max(), (v, c, fd, g[v, c])
