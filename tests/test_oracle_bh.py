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
