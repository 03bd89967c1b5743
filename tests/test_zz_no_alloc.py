"""The entry point that allocates nothing (tp_energy_faces_noalloc), through the C-ABI,
against the allocating tp_energy_faces on the same face quantities, and both against the
FP64 oracle: two calls in a row, the second on a smaller input, for each precision."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_2107_01664_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_01664_amd import tpsurf
    tpsurf.lib()
    return tpsurf


def _faces(m):
    X, N, a = O.faces(m.V, m.F)
    return [torch.from_numpy(np.ascontiguousarray(q)).to("cuda") for q in (X, N, a)], (X, N, a)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_noalloc_energy_matches_allocating_entry_point(tp, prec):
    big = mg.add_noise(mg.torus(37, 23, 1.0, 0.3), 0.004, 2)        # 1,702 faces, ragged tiles
    small = mg.add_noise(mg.icosphere(2), 0.02, 3)                    # 320 faces, < one i-tile
    params = tp.default_params(precision=prec)
    tol_oracle = 1e-11 if prec == 2 else (1e-4 if prec == 1 else 1e-5)
    for m in (big, small, big):
        print(f"[no-alloc] prec={prec} nF={m.nF}", flush=True)
        (X, N, a), (Xh, Nh, ah) = _faces(m)
        E_ref = tp.tp_energy_faces(X, N, a, params)
        E_na = tp.tp_energy_faces_noalloc(X, N, a, params)
        torch.cuda.synchronize()
        assert abs(E_na - E_ref) <= 1e-12 * abs(E_ref), (E_na, E_ref)
        E0 = O.energy_faces(Xh, Nh, ah)
        assert abs(E_na - E0) <= tol_oracle * E0, (E_na, E0)


def test_noalloc_rejects_too_many_faces(tp):
    """nF beyond the scratch limit is an argument error raised before any device work."""
    m = mg.add_noise(mg.icosphere(2), 0.02, 3)
    (X, N, a), _ = _faces(m)
    E = ctypes.c_double()
    st = tp.lib().tp_energy_faces_noalloc(X.data_ptr(), N.data_ptr(), a.data_ptr(), 65537,
                                          ctypes.byref(tp.default_params(precision=0)), ctypes.byref(E), None)
    assert st == tp.TP_E_INVALID_ARGUMENT
    st = tp.lib().tp_energy_faces_noalloc(X.data_ptr(), N.data_ptr(), a.data_ptr(), m.nF,
                                          ctypes.byref(tp.default_params(precision=3)), ctypes.byref(E), None)
    assert st == tp.TP_E_INVALID_ARGUMENT
