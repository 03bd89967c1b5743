"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on the same seeded
inputs.  Tolerances (relative, normwise): energy and differential 1e-5 for FP32 pair terms
with FP64 accumulation, 1e-11 for FP64 pair terms."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2107_01664_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-11
# FP32 pair terms from FP32-rounded barycenters (no hi/lo split): reported, not held to
# 1e-5 -- q = N.d cancels for near pairs on smooth surfaces, which is what hi/lo fixes.
TOL32_NAIVE = 1e-4


@pytest.fixture(scope="module")
def tp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_01664_amd import tpsurf
    tpsurf.lib()
    return tpsurf


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def tol_for(prec):
    # 4, 5: the naive FP32 pair terms of 1 with FP32 (plain or compensated) per-face sums
    return {0: TOL32, 1: TOL32_NAIVE, 2: TOL64, 3: TOL32, 4: TOL32_NAIVE, 5: TOL32_NAIVE}[prec]


MESHES = {
    "small_sphere": lambda: mg.workload("small_sphere"),                     # 1280 faces
    "geodesic9": lambda: mg.add_noise(mg.geodesic_sphere(9), 0.01, 1),       # 1620 faces, ragged
    "torus37x23": lambda: mg.add_noise(mg.torus(37, 23, 1.0, 0.3), 0.004, 2),  # 1702 faces
    "icosahedron": lambda: mg.add_noise(mg.icosahedron(), 0.02, 3),          # 20 faces, < 1 tile
    "linked_small": lambda: mg.linked_tori(24, 12, 1.0, 0.25, 1.0),           # 1152 faces, 2 parts
}


@pytest.fixture(scope="module")
def meshes():
    return {k: f() for k, f in MESHES.items()}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("prec", [0, 1, 2, 3, 4, 5])
def test_energy_gradient_parity(tp, meshes, name, prec):
    m = meshes[name]
    print(f"[parity] energy/gradient {name} nF={m.nF} precision={prec}", flush=True)
    E0, g0 = O.gradient(m.V, m.F)
    p = tp.default_params(precision=prec)
    V, F = dev(m.V), dev(m.F, torch.int32)
    E = tp.tp_energy(V, F, p)
    E1, g1 = tp.tp_gradient(V, F, p)
    g1 = g1.cpu().numpy()
    t = tol_for(prec)
    assert abs(E - E0) <= t * E0, (E, E0)
    assert abs(E1 - E0) <= t * E0, (E1, E0)
    assert rel(g1, g0) <= t, rel(g1, g0)


@pytest.mark.parametrize("alpha,beta", [(4.0, 9.0), (3.5, 8.0), (8.0, 16.0)])
@pytest.mark.parametrize("prec", [0, 2])
def test_general_exponents(tp, meshes, alpha, beta, prec):
    m = meshes["geodesic9"]
    print(f"[parity] exponents alpha={alpha} beta={beta} precision={prec}", flush=True)
    E0, g0 = O.gradient(m.V, m.F, alpha, beta)
    p = tp.default_params(alpha=alpha, beta=beta, precision=prec)
    E1, g1 = tp.tp_gradient(dev(m.V), dev(m.F, torch.int32), p)
    t = tol_for(prec)
    print(f"  E rel {abs(E1 - E0) / E0:.2e}, dE rel {rel(g1.cpu().numpy(), g0):.2e}", flush=True)
    assert abs(E1 - E0) <= t * E0
    assert rel(g1.cpu().numpy(), g0) <= t
    if prec == 0:                      # the energy kernel of the line search, same policy
        E2 = tp.tp_energy(dev(m.V), dev(m.F, torch.int32), p)
        assert abs(E2 - E0) <= t * E0


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("prec", [0, 1, 3])
def test_gradient_symmetric(tp, meshes, name, prec):
    """The symmetric E + dE kernel (each unordered pair once, for both rows) forced at small
    sizes: E and dE against the oracle and against the row-by-row kernel, on meshes of one
    block, of ragged last blocks and of two components, with and without the FP64 near
    field."""
    m = meshes[name]
    print(f"[parity] symmetric gradient {name} precision={prec}", flush=True)
    E0, g0 = O.gradient(m.V, m.F)
    V, F = dev(m.V), dev(m.F, torch.int32)
    Es, gs = tp.tp_gradient(V, F, tp.default_params(precision=prec, sym_pairs=1))
    Er, gr = tp.tp_gradient(V, F, tp.default_params(precision=prec, sym_pairs=0))
    gs, gr = gs.cpu().numpy(), gr.cpu().numpy()
    t = tol_for(prec)
    assert abs(Es - E0) <= t * E0, (Es, E0)
    assert rel(gs, g0) <= t, rel(gs, g0)
    assert abs(Es - Er) <= t * E0, (Es, Er)
    assert rel(gs, gr) <= t, rel(gs, gr)


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("prec", [0, 1, 3])
def test_energy_symmetric(tp, meshes, name, prec):
    """The symmetric energy kernel (each unordered pair once, one FP64 partial per pair of
    blocks) forced at small sizes: against the oracle and the row-by-row kernel, on meshes of
    one block (20 faces), of ragged last blocks and of two components, with and without the
    FP64 near field."""
    m = meshes[name]
    print(f"[parity] symmetric energy {name} precision={prec}", flush=True)
    E0 = O.energy(m.V, m.F)
    V, F = dev(m.V), dev(m.F, torch.int32)
    Es = tp.tp_energy(V, F, tp.default_params(precision=prec, sym_pairs=1))
    Er = tp.tp_energy(V, F, tp.default_params(precision=prec, sym_pairs=0))
    t = tol_for(prec)
    assert abs(Es - E0) <= t * E0, (Es, E0)
    assert abs(Es - Er) <= t * E0, (Es, Er)


@pytest.mark.parametrize("alpha,beta", [(4.0, 9.0), (8.0, 16.0)])
def test_energy_symmetric_general_exponents(tp, meshes, alpha, beta):
    m = meshes["geodesic9"]
    print(f"[parity] symmetric energy alpha={alpha} beta={beta}", flush=True)
    E0 = O.energy(m.V, m.F, alpha, beta)
    E1 = tp.tp_energy(dev(m.V), dev(m.F, torch.int32), tp.default_params(alpha=alpha, beta=beta, precision=0,
                                                                            sym_pairs=1))
    assert abs(E1 - E0) <= tol_for(0) * E0


@pytest.mark.parametrize("alpha,beta", [(4.0, 9.0), (8.0, 16.0)])
def test_gradient_symmetric_general_exponents(tp, meshes, alpha, beta):
    m = meshes["geodesic9"]
    print(f"[parity] symmetric gradient alpha={alpha} beta={beta}", flush=True)
    E0, g0 = O.gradient(m.V, m.F, alpha, beta)
    p = tp.default_params(alpha=alpha, beta=beta, precision=0, sym_pairs=1)
    E1, g1 = tp.tp_gradient(dev(m.V), dev(m.F, torch.int32), p)
    t = tol_for(0)
    assert abs(E1 - E0) <= t * E0
    assert rel(g1.cpu().numpy(), g0) <= t


@pytest.mark.parametrize("k", [1, 3, 9, 11])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_fractional_parity(tp, meshes, k, prec):
    m = meshes["torus37x23"]
    print(f"[parity] fractional k={k} precision={prec}", flush=True)
    u = mg.random_columns(m.nV, k, 1)
    L0 = O.fractional_apply(m.V, m.F, u, 1.0 / 3.0)
    L1 = tp.tp_fractional_apply(dev(m.V), dev(m.F, torch.int32), dev(u), tp.default_params(precision=prec))
    L1 = L1.cpu().numpy()
    for c in range(k):
        assert rel(L1[:, c], L0[:, c]) <= tol_for(prec), (c, rel(L1[:, c], L0[:, c]))


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("k", [1, 3, 4, 7, 9])
@pytest.mark.parametrize("prec", [0, 1, 3])
def test_fractional_symmetric(tp, meshes, name, k, prec):
    """The symmetric fractional apply (each unordered pair once, for both rows) forced at
    small sizes: against the oracle, and against the row-by-row kernel, on meshes of one
    block (20 faces), of ragged last blocks and of two components."""
    m = meshes[name]
    print(f"[parity] symmetric fractional {name} k={k} precision={prec}", flush=True)
    u = mg.random_columns(m.nV, k, 1)
    L0 = O.fractional_apply(m.V, m.F, u, 1.0 / 3.0)
    V, F, du = dev(m.V), dev(m.F, torch.int32), dev(u)
    Ls = tp.tp_fractional_apply(V, F, du, tp.default_params(precision=prec, sym_pairs=1)).cpu().numpy()
    Lr = tp.tp_fractional_apply(V, F, du, tp.default_params(precision=prec, sym_pairs=0)).cpu().numpy()
    for c in range(k):
        assert rel(Ls[:, c], L0[:, c]) <= tol_for(prec), (c, rel(Ls[:, c], L0[:, c]))
        assert rel(Ls[:, c], Lr[:, c]) <= tol_for(prec), (c, rel(Ls[:, c], Lr[:, c]))


@pytest.mark.parametrize("name", ["small_sphere", "geodesic9", "torus37x23", "linked_small"])
@pytest.mark.parametrize("band", [1, 2, 3])
def test_symmetric_bands_equal_one_launch(tp, meshes, name, band):
    """The symmetric kernels run in bands of rows of blocks (one launch and one reduction per
    band): every band height gives bit for bit the result of a single band, since each face's
    slices are added in the same order; meshes of 5 to 7 blocks, ragged last blocks, two
    components, with the FP64 near field."""
    m = meshes[name]
    print(f"[parity] symmetric bands {name} band={band}", flush=True)
    V, F = dev(m.V), dev(m.F, torch.int32)
    one = tp.default_params(sym_pairs=1)
    banded = tp.default_params(sym_pairs=1, sym_band=band)
    E1, g1 = tp.tp_gradient(V, F, one)
    Eb, gb = tp.tp_gradient(V, F, banded)
    assert Eb == E1
    assert torch.equal(gb, g1)
    for k in (3, 9):
        du = dev(mg.random_columns(m.nV, k, 4))
        L1 = tp.tp_fractional_apply(V, F, du, one)
        Lb = tp.tp_fractional_apply(V, F, du, banded)
        assert torch.equal(Lb, L1), k


def test_symmetric_band_rejects_negative(tp, meshes):
    m = meshes["small_sphere"]
    with pytest.raises(tp.TpError):
        tp.tp_gradient(dev(m.V), dev(m.F, torch.int32), tp.default_params(sym_band=-1))


def test_fractional_symmetric_errors(tp, meshes):
    m = meshes["small_sphere"]
    u = dev(mg.random_columns(m.nV, 1, 1))
    with pytest.raises(tp.TpError):
        tp.tp_fractional_apply(dev(m.V), dev(m.F, torch.int32), u, tp.default_params(sym_pairs=2))


def test_fractional_sigma_override(tp, meshes):
    m = meshes["small_sphere"]
    u = mg.random_columns(m.nV, 2, 5)
    L0 = O.fractional_apply(m.V, m.F, u, 0.6)
    L1 = tp.tp_fractional_apply(dev(m.V), dev(m.F, torch.int32), dev(u), tp.default_params(sigma=0.6))
    assert rel(L1.cpu().numpy(), L0) <= TOL32


def test_energy_faces_sphere_closed_form(tp):
    """Face data on a sphere with radial normals: K = (2R)^-6 for every pair, at 327,680
    faces (the size of the bumpy-sphere workload)."""
    rng = np.random.default_rng(7)
    n = 327680
    P = rng.standard_normal((n, 3))
    N = P / np.linalg.norm(P, axis=1, keepdims=True)
    R = 0.8
    A = rng.uniform(0.5, 1.5, n) * 4 * math.pi * R * R / n
    expect = (2 * R) ** -6 * (A.sum() ** 2 - (A ** 2).sum())
    for prec in (0, 2):
        E = tp.tp_energy_faces(dev(R * N), dev(N), dev(A), tp.default_params(precision=prec))
        assert abs(E - expect) <= tol_for(prec) * expect, (prec, E, expect)


def test_deterministic(tp, meshes):
    m = meshes["torus37x23"]
    V, F = dev(m.V), dev(m.F, torch.int32)
    E1, g1 = tp.tp_gradient(V, F)
    E2, g2 = tp.tp_gradient(V, F)
    assert E1 == E2 and torch.equal(g1, g2)
    u = dev(mg.random_columns(m.nV, 3, 3))
    assert torch.equal(tp.tp_fractional_apply(V, F, u), tp.tp_fractional_apply(V, F, u))


# ----------------------------------------------------------------- preconditioner, step

def test_precond_apply(tp, meshes):
    m = meshes["small_sphere"]
    b = mg.random_columns(m.nV, 3, 4)
    x0 = O.precond_apply(m.V, m.F, b, 1.0 / 3.0)
    x1, rep = tp.tp_precond_apply(dev(m.V), dev(m.F, torch.int32), dev(b))
    x1 = x1.cpu().numpy()
    assert rep.cg_relres[0] <= 1e-10 and rep.cg_relres[1] <= 1e-10
    assert rel(x1, x0) <= 1e-5, rel(x1, x0)


def test_poisson_residual_two_components(tp, meshes):
    """Per-component mean-zero solutions on two linked tori; CG residual recomputed by the
    oracle's cotan matrix."""
    m = meshes["linked_small"]
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        b = mg.random_columns(m.nV, 2, 8)
        x, rep = P.precond_apply(dev(b))
        x0 = O.precond_apply(m.V, m.F, b, 1.0 / 3.0)
        assert rel(x.cpu().numpy(), x0) <= 1e-5


@pytest.mark.parametrize("name", ["small_sphere", "linked_small"])
def test_step_fixed_tau(tp, meshes, name):
    m = meshes[name]
    tau = 2e-3
    ref = O.precond_step(m.V, m.F, tau=tau, line_search=False)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        rep = P.step(tp.step_opts(tau0=tau, line_search=0), direction=d)
        Vn = P.vertices().cpu().numpy()
    x = d.cpu().numpy()
    assert rel(x, ref.direction) <= 1e-4, rel(x, ref.direction)
    assert rel(Vn - m.V, ref.V - m.V) <= 1e-4
    assert abs(rep.E - ref.E) <= TOL32 * ref.E
    assert rep.slope < 0
    assert np.abs(np.asarray(rep.phi_after)).max() <= 10 * np.abs(ref.phi_after).max() + 1e-12


def test_step_armijo_decreases(tp, meshes):
    m = meshes["small_sphere"]
    ref = O.precond_step(m.V, m.F)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        rep = P.step()
    assert rep.E_new < rep.E
    assert rep.backtracks == ref.backtracks
    assert abs(rep.tau - ref.tau) <= 1e-6 * ref.tau


# ------------------------------------------------------------------- failure handling

def test_errors(tp, meshes):
    m = meshes["icosahedron"]
    V, F = dev(m.V), dev(m.F, torch.int32)
    bad = m.F.copy()
    bad[3, 1] = m.nV + 5
    with pytest.raises(tp.TpError) as e:
        tp.tp_energy(V, dev(bad, torch.int32))
    assert e.value.status == 3
    deg = m.V.copy()
    deg[m.F[0, 1]] = deg[m.F[0, 0]]
    with pytest.raises(tp.TpError) as e:
        tp.tp_energy(dev(deg), F)
    assert e.value.status == 2
    nan = m.V.copy()
    nan[4, 2] = np.nan
    with pytest.raises(tp.TpError) as e:
        tp.tp_gradient(dev(nan), F)
    assert e.value.status == 4
    with pytest.raises(tp.TpError) as e:
        tp.tp_energy(V, F, tp.default_params(alpha=0.5))
    assert e.value.status == 1
    # iteration cap: plain CG on the icosahedron, preconditioned CG on a larger torus (on
    # the icosahedron the two-level preconditioner is the exact inverse: one iteration)
    for pc, mesh in ((0, m), (1, meshes["torus37x23"])):
        Vm, Fm = dev(mesh.V), dev(mesh.F, torch.int32)
        with tp.Problem(Vm, Fm, tp.default_params(cg_maxiter=1, cg_precond=pc)) as P:
            with pytest.raises(tp.TpError) as e:
                P.precond_apply(dev(mg.random_columns(mesh.nV, 1, 0)))
            assert e.value.status == 5
            x, rep = P.precond_apply(dev(mg.random_columns(mesh.nV, 1, 0)), allow_not_converged=True)
            assert rep.cg_iters[0] == 1


# -------------------------------------------------------------- full-size workloads

@pytest.fixture(scope="module")
def torus40k():
    return mg.workload("torus40k")


def test_torus40k_full_size(tp, torus40k):
    """40,000-face torus in the launch configuration the benchmark times: energy against
    the full oracle sum, dE and L^sigma u at sampled vertices against the oracle."""
    m = torus40k
    print("[parity] torus40k full size", flush=True)
    V, F = dev(m.V), dev(m.F, torch.int32)
    u = mg.random_columns(m.nV, 3, 1)
    with tp.Problem(V, F) as P:
        E, g = P.gradient()
        Lu = P.fractional_apply(dev(u))
    g = g.cpu().numpy()
    Lu = Lu.cpu().numpy()
    E0 = O.energy(m.V, m.F)
    assert abs(E - E0) <= TOL32 * E0, (E, E0)
    verts = np.random.default_rng(0).choice(m.nV, 32, replace=False)
    g0 = O.gradient_at_vertices(m.V, m.F, verts)
    # normwise over the sample, relative to the sample's norm
    assert rel(g[verts], g0) <= TOL32, rel(g[verts], g0)
    L0 = O.fractional_at_vertices(m.V, m.F, u, verts, 1.0 / 3.0)
    assert rel(Lu[verts], L0) <= TOL32, rel(Lu[verts], L0)
    # properties that hold at any size
    scale = np.abs(g).sum()
    assert np.abs(g.sum(0)).max() <= 1e-6 * scale
    # Euler: sum f.dE = (4 + 6 - 12) E; an error dE' with |dE'| <= 1e-5 |dE| moves the sum
    # by at most |f| |dE'| (Cauchy-Schwarz)
    assert abs((m.V * g).sum() + 2.0 * E) <= TOL32 * np.linalg.norm(m.V) * np.linalg.norm(g)


def test_bumpy327k_fp64_sampled(tp):
    """327,680-face bumpy sphere (the precision-sweep mesh): the FP64 direct sums, which
    the sweep uses as its reference, against the oracle at sampled vertices; translation
    and Euler identities over the whole mesh."""
    m = mg.workload("bumpy327k")
    print("[parity] bumpy327k FP64 at sampled vertices", flush=True)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32), tp.default_params(precision=2)) as P:
        E, g = P.gradient()
    g = g.cpu().numpy()
    verts = np.random.default_rng(0).choice(m.nV, 12, replace=False)
    g0 = O.gradient_at_vertices(m.V, m.F, verts)
    assert rel(g[verts], g0) <= 1e-10, rel(g[verts], g0)
    # FP32 pair terms with the FP64 near field meet 1e-5 at full size (over the whole mesh,
    # against the FP64 sums just pinned)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32), tp.default_params(precision=3)) as P:
        E3, g3 = P.gradient()
    g3 = g3.cpu().numpy()
    print(f"[parity] bumpy327k near64: E {abs(E3 - E) / E:.2e} dE {rel(g3, g):.2e}", flush=True)
    assert abs(E3 - E) <= TOL32 * E and rel(g3, g) <= TOL32
    scale = np.abs(g).sum()
    assert np.abs(g.sum(0)).max() <= 1e-9 * scale
    assert abs((m.V * g).sum() + 2.0 * E) <= 1e-9 * np.linalg.norm(m.V) * np.linalg.norm(g)


def test_bumpy327k_bands_bit_identical(tp):
    """At full size the symmetric kernels run in bands of rows (45 for E + dE within the
    512 MB partial buffer): a band height of 13 blocks instead of the default gives bit for
    bit the same E, dE, E alone and L^sigma u (k = 3), since each face's slices are added
    in the same order."""
    m = mg.workload("bumpy327k")
    print("[parity] bumpy327k symmetric kernels, two band heights", flush=True)
    V, F = dev(m.V), dev(m.F, torch.int32)
    u = dev(mg.random_columns(m.nV, 3, 5))
    out = []
    for band in (0, 13):
        with tp.Problem(V, F, tp.default_params(sym_band=band)) as P:
            E, g = P.gradient()
            Ee = P.energy()
            L = P.fractional_apply(u)
            out.append((E, g.clone(), Ee, L.clone()))
    (E0, g0, Ee0, L0), (E1, g1, Ee1, L1) = out
    assert E1 == E0 and Ee1 == Ee0
    assert torch.equal(g1, g0) and torch.equal(L1, L0)
    assert abs(Ee0 - E0) <= TOL32 * E0   # the energy kernel against the E of E + dE


def test_torus40k_poisson(tp, torus40k):
    m = torus40k
    b = mg.random_columns(m.nV, 3, 2)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        x, rep = P.precond_apply(dev(b))
    x = x.cpu().numpy()
    assert rep.cg_relres[0] <= 1e-10 and rep.cg_relres[1] <= 1e-10
    # second solve's residual against the oracle's matrix: C x = P (L y)
    C = O.cotan_laplacian(m.V, m.F)
    _, labels = O.components(m.F, m.nV)
    y = O.poisson_solve(C, b, labels)
    z = O.project_mean_zero(O.fractional_apply(m.V, m.F, y, 1.0 / 3.0), labels)
    # the second solve's right-hand side is the GPU's FP32-pair fractional apply, so the
    # residual against the oracle's right-hand side is bounded by that apply's tolerance
    r = np.linalg.norm(z - C @ x) / np.linalg.norm(z)
    assert r <= TOL32, r
    assert rel(x, O.poisson_solve(C, z, labels)) <= 1e-4


def test_linked_tori_full_step(tp):
    """Full step on the 51,200-face linked tori: tangent to the constraints, a descent
    direction, energy decreases, constraints restored to second order."""
    m = mg.workload("linked_tori")
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        rep = P.step(direction=d)
    x = d.cpu().numpy()
    JA, JV = O.area_gradient(m.V, m.F), O.volume_gradient(m.V, m.F)
    assert abs(np.vdot(JA, x)) <= 1e-6 * np.linalg.norm(JA) * np.linalg.norm(x)
    assert abs(np.vdot(JV, x)) <= 1e-6 * np.linalg.norm(JV) * np.linalg.norm(x)
    assert rep.slope < 0 and rep.E_new < rep.E
    assert abs(rep.phi_after[0]) <= abs(rep.phi_trial[0]) + 1e-9


def test_linked_tori_step_vs_oracle(tp):
    """The full-size C3 step (51,200 faces, two components, area and volume constraints) at
    a fixed tau against the oracle's step (Sec. 5.3 with the preconditioner of Sec. 5.2):
    the projected direction and the corrected vertices within 1e-4 (FP32 pair terms move
    the right-hand sides by ~1e-6 and the Poisson solves stop at 1e-10)."""
    m = mg.workload("linked_tori")
    tau = 1e-3
    print("[parity] linked tori step vs oracle: oracle step (about 20 s of CPU)", flush=True)
    ref = O.precond_step(m.V, m.F, tau=tau, line_search=False)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        rep = P.step(tp.step_opts(tau0=tau, line_search=0), direction=d)
        Vn = P.vertices().cpu().numpy()
    x = d.cpu().numpy()
    print("  direction error", rel(x, ref.direction), "vertex error", rel(Vn - m.V, ref.V - m.V), flush=True)
    assert rel(x, ref.direction) <= 1e-4
    assert rel(Vn - m.V, ref.V - m.V) <= 1e-4
    assert abs(rep.E - ref.E) <= TOL32 * ref.E
    assert np.allclose(rep.phi_after, ref.phi_after, rtol=1e-3, atol=1e-12 * O.total_area(m.V, m.F))


# ------------------------------------------------- preconditioned vs plain Poisson solves

# serving-mix meshes with one row whose entries reach five aggregates (more than the solver
# keeps in registers)
REQUEST_MESHES = {
    "request_sphere": {"kind": "sphere", "freq": 11, "nF": 2420, "id": 29, "seed": 29, "steps": 4},
    "request_torus": {"kind": "torus", "nu": 68, "nv": 34, "nF": 4624, "id": 19, "seed": 19, "steps": 4},
}


@pytest.mark.parametrize("name", ["small_sphere", "linked_small", "tiny_tori", "request_sphere",
                                  "request_torus"])
def test_pcg_matches_plain_cg(tp, meshes, name):
    """Two-level Schwarz preconditioned CG and plain CG reach the same per-component
    mean-zero solution; the preconditioned one in fewer iterations.  'tiny_tori' has
    components smaller than one block (whole-component blocks); the request meshes have a
    row touching five aggregates, which must not send the solve to plain CG."""
    if name == "tiny_tori":
        m = mg.linked_tori(8, 6, 1.0, 0.25, 1.0)
    elif name in REQUEST_MESHES:
        m = mg.build_request_mesh(REQUEST_MESHES[name])
    else:
        m = meshes[name]
    b = mg.random_columns(m.nV, 3, 9)
    V, F = dev(m.V), dev(m.F, torch.int32)
    out = {}
    for pc in (0, 1):
        with tp.Problem(V, F, tp.default_params(cg_precond=pc)) as P:
            x, rep = P.precond_apply(dev(b))
            out[pc] = (x.cpu().numpy(), list(rep.cg_iters), list(rep.cg_relres))
    x0 = O.precond_apply(m.V, m.F, b, 1.0 / 3.0)
    for pc in (0, 1):
        assert max(out[pc][2]) <= 1e-10
        assert rel(out[pc][0], x0) <= 1e-5, (pc, rel(out[pc][0], x0))
    print(f"[pcg] {name}: iterations plain {out[0][1]} preconditioned {out[1][1]}", flush=True)
    assert out[1][1][0] <= out[0][1][0]
    if name in REQUEST_MESHES:
        assert out[1][1][0] <= 0.7 * out[0][1][0]


@pytest.mark.parametrize("pc", [0, 1])
def test_poisson_true_residual_torus40k(tp, torus40k, pc):
    """CG reports the true relative residual; recomputed here with the oracle's cotan
    matrix it must meet 1e-10 (up to the rounding of the recomputation)."""
    m = torus40k
    b = mg.random_columns(m.nV, 9, 3)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32), tp.default_params(cg_precond=pc)) as P:
        x, rep = P.poisson_solve(dev(b))
    print(f"[pcg] torus40k k=9 precond={pc} iterations {rep.cg_iters[0]} relres {rep.cg_relres[0]:.2e} "
          f"ms {rep.t_ms[0]:.2f}", flush=True)
    assert rep.cg_relres[0] <= 1e-10
    C = O.cotan_laplacian(m.V, m.F)
    _, labels = O.components(m.F, m.nV)
    Pb = O.project_mean_zero(b, labels)
    x = x.cpu().numpy()
    r = np.linalg.norm(Pb - C @ x, axis=0) / np.linalg.norm(Pb, axis=0)
    assert r.max() <= 2e-10, r
    assert np.abs(O.project_mean_zero(x, labels) - x).max() <= 1e-12 * np.abs(x).max()


@pytest.fixture(scope="module")
def sphere41k():
    return mg.add_noise(mg.icosphere(6), 0.001, 1)


@pytest.mark.parametrize("k", [1, 3, 9])
def test_pcg_multi_launch_sphere41k(tp, sphere41k, k):
    """More blocks (321) than workgroups resident at once: the preconditioned solve runs as
    one launch per phase.  Its solution meets 1e-10 in the true residual recomputed with the
    oracle's cotan matrix, is per-component mean-zero, and takes far fewer iterations than
    plain CG."""
    m = sphere41k
    b = mg.random_columns(m.nV, k, 5)
    its = {}
    for pc in (1, 0):
        with tp.Problem(dev(m.V), dev(m.F, torch.int32), tp.default_params(cg_precond=pc)) as P:
            x, rep = P.poisson_solve(dev(b))
        print(f"[pcg] sphere41k k={k} precond={pc} iterations {rep.cg_iters[0]} relres {rep.cg_relres[0]:.2e} "
              f"ms {rep.t_ms[0]:.2f}", flush=True)
        assert rep.cg_relres[0] <= 1e-10
        its[pc] = rep.cg_iters[0]
        if pc == 1:
            C = O.cotan_laplacian(m.V, m.F)
            _, labels = O.components(m.F, m.nV)
            Pb = O.project_mean_zero(b, labels)
            xs = x.cpu().numpy()
            r = np.linalg.norm(Pb - C @ xs, axis=0) / np.linalg.norm(Pb, axis=0)
            assert r.max() <= 2e-10, r
            assert np.abs(O.project_mean_zero(xs, labels) - xs).max() <= 1e-12 * np.abs(xs).max()
    assert its[1] <= 0.4 * its[0], its


def test_pcg_multi_launch_iteration_cap(tp, sphere41k):
    """The multi-launch solve stops at the iteration budget (also across its batches of
    iterations and its restarts): the status is 'not converged' and the report counts the
    budget, for a budget inside the first batch and one across several."""
    m = sphere41k
    b = dev(mg.random_columns(m.nV, 2, 0))
    for cap in (5, 37):
        with tp.Problem(dev(m.V), dev(m.F, torch.int32), tp.default_params(cg_maxiter=cap)) as P:
            with pytest.raises(tp.TpError) as e:
                P.poisson_solve(b)
            assert e.value.status == 5
            x, rep = P.poisson_solve(b, allow_not_converged=True)
        assert rep.cg_iters[0] == cap
        assert 1e-10 < rep.cg_relres[0] < 1.0
        assert torch.isfinite(x).all()


def test_pcg_multi_launch_two_components(tp):
    """Two linked tori on 320 x 160 grids (102,400 vertices, 800 blocks, two components):
    the multi-launch solve keeps each component's solution mean-zero, meets 1e-10 in the
    true residual of the oracle's cotan matrix, and needs well under the ~1,300 iterations
    of plain CG at this size."""
    m = mg.linked_tori(320, 160, 1.0, 0.25, 1.0)
    b = mg.random_columns(m.nV, 3, 7)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        x, rep = P.poisson_solve(dev(b))
    print(f"[pcg] linked tori {m.nV} vertices: iterations {rep.cg_iters[0]} relres {rep.cg_relres[0]:.2e} "
          f"ms {rep.t_ms[0]:.2f}", flush=True)
    assert rep.cg_relres[0] <= 1e-10
    C = O.cotan_laplacian(m.V, m.F)
    _, labels = O.components(m.F, m.nV)
    assert labels.max() == 1
    Pb = O.project_mean_zero(b, labels)
    xs = x.cpu().numpy()
    r = np.linalg.norm(Pb - C @ xs, axis=0) / np.linalg.norm(Pb, axis=0)
    assert r.max() <= 2e-10, r
    assert np.abs(O.project_mean_zero(xs, labels) - xs).max() <= 1e-12 * np.abs(xs).max()
    assert rep.cg_iters[0] <= 600


def test_pcg_columns_together_like_alone(tp, torus40k):
    """The columns of one solve are independent systems: solved together (k = 9) they take
    about as many iterations as the slowest one solved alone.  The right-hand sides are
    those of the preconditioner's second solve (L^sigma of a first solution), on which an
    iteration that amplifies rounding (the pipelined form) needed ten times more."""
    m = torus40k
    b = mg.random_columns(m.nV, 9, 2)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        x1, _ = P.poisson_solve(dev(b))
        Lx = P.fractional_apply(x1)
        alone = [P.poisson_solve(Lx[:, c:c + 1].contiguous())[1].cg_iters[0] for c in range(9)]
        x9, rep = P.poisson_solve(Lx.contiguous())
        for c in range(9):
            xc, _ = P.poisson_solve(Lx[:, c:c + 1].contiguous())
            assert rel(x9[:, c].cpu().numpy(), xc[:, 0].cpu().numpy()) <= 1e-8
    print(f"[pcg] torus40k second-solve right-hand sides: alone {alone}, together {rep.cg_iters[0]}", flush=True)
    assert rep.cg_relres[0] <= 1e-10
    assert rep.cg_iters[0] <= max(alone) + 5


# ---------------------------------------------------- inner-product operator A = B + B0

S_SOB = 5.0 / 3.0   # s = (beta - 2) / alpha for alpha = 6, beta = 12


@pytest.mark.parametrize("k", [1, 3, 4, 7])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_sobolev_parity(tp, meshes, k, prec):
    """A u on a 1702-face torus (ragged last tile) against the oracle, column by column;
    k = 4 and 7 take more than one group of three columns."""
    m = meshes["torus37x23"]
    print(f"[parity] sobolev k={k} precision={prec}", flush=True)
    u = mg.random_columns(m.nV, k, 7)
    A0 = O.sobolev_apply(m.V, m.F, u, S_SOB)
    A1 = tp.tp_sobolev_apply(dev(m.V), dev(m.F, torch.int32), dev(u), tp.default_params(precision=prec))
    A1 = A1.cpu().numpy()
    errs = [rel(A1[:, c], A0[:, c]) for c in range(k)]
    print("  errors", ["%.2e" % e for e in errs], flush=True)
    assert max(errs) <= tol_for(prec), errs


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", [0, 1, 3])
def test_sobolev_symmetric(tp, meshes, name, k, prec):
    """The symmetric pair kernel of A u (each unordered pair once, for both rows) forced at
    small sizes: against the oracle column by column and against the row-by-row kernel, on
    meshes of one block, of ragged last blocks and of two components."""
    m = meshes[name]
    print(f"[parity] symmetric sobolev {name} k={k} precision={prec}", flush=True)
    u = mg.random_columns(m.nV, k, 7)
    A0 = O.sobolev_apply(m.V, m.F, u, S_SOB)
    V, F, du = dev(m.V), dev(m.F, torch.int32), dev(u)
    As = tp.tp_sobolev_apply(V, F, du, tp.default_params(precision=prec, sym_pairs=1)).cpu().numpy()
    Ar = tp.tp_sobolev_apply(V, F, du, tp.default_params(precision=prec, sym_pairs=0)).cpu().numpy()
    for c in range(k):
        assert rel(As[:, c], A0[:, c]) <= tol_for(prec), (c, rel(As[:, c], A0[:, c]))
        assert rel(As[:, c], Ar[:, c]) <= tol_for(prec), (c, rel(As[:, c], Ar[:, c]))


@pytest.mark.parametrize("alpha,beta", [(4.0, 9.0), (6.0, 10.0)])
def test_sobolev_symmetric_general_exponents(tp, meshes, alpha, beta):
    """The symmetric kernel of A u at other exponents: the operator's order 2s follows
    s = (beta - 2) / alpha (7/4 and 4/3 here), against the oracle with that s."""
    m = meshes["geodesic9"]
    s_op = (beta - 2.0) / alpha
    print(f"[parity] symmetric sobolev alpha={alpha} beta={beta} s={s_op}", flush=True)
    u = mg.random_columns(m.nV, 3, 9)
    A0 = O.sobolev_apply(m.V, m.F, u, s_op)
    A1 = tp.tp_sobolev_apply(dev(m.V), dev(m.F, torch.int32), dev(u),
                             tp.default_params(alpha=alpha, beta=beta, precision=0, sym_pairs=1)).cpu().numpy()
    for c in range(3):
        assert rel(A1[:, c], A0[:, c]) <= tol_for(0), (c, rel(A1[:, c], A0[:, c]))


def test_fractional_symmetric_sigma_override(tp, meshes):
    """The symmetric fractional apply with sigma = 0.6 (kernel |d|^-3.2) against the oracle."""
    m = meshes["torus37x23"]
    u = mg.random_columns(m.nV, 3, 6)
    L0 = O.fractional_apply(m.V, m.F, u, 0.6)
    L1 = tp.tp_fractional_apply(dev(m.V), dev(m.F, torch.int32), dev(u),
                                tp.default_params(sigma=0.6, sym_pairs=1)).cpu().numpy()
    for c in range(3):
        assert rel(L1[:, c], L0[:, c]) <= tol_for(3), (c, rel(L1[:, c], L0[:, c]))


@pytest.mark.parametrize("band", [1, 2])
def test_sobolev_symmetric_bands(tp, meshes, band):
    """Bands of rows give bit for bit the result of one band (7 blocks, ragged last block)."""
    m = meshes["torus37x23"]
    u = dev(mg.random_columns(m.nV, 3, 8))
    V, F = dev(m.V), dev(m.F, torch.int32)
    A1 = tp.tp_sobolev_apply(V, F, u, tp.default_params(sym_pairs=1))
    Ab = tp.tp_sobolev_apply(V, F, u, tp.default_params(sym_pairs=1, sym_band=band))
    assert torch.equal(Ab, A1)


@pytest.mark.parametrize("name", ["small_sphere", "linked_small", "icosahedron", "geodesic9"])
def test_sobolev_coordinates(tp, meshes, name):
    """A applied to the coordinate functions (the operator A_3 of the descent direction acts
    on them) and to constants (annihilated)."""
    m = meshes[name]
    print(f"[parity] sobolev coordinates {name}", flush=True)
    u = np.ascontiguousarray(m.V)
    A0 = O.sobolev_apply(m.V, m.F, u, S_SOB)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        A1 = P.sobolev_apply(dev(u)).cpu().numpy()
        c1 = P.sobolev_apply(torch.ones((m.nV, 2), dtype=torch.float64, device="cuda")).cpu().numpy()
    for c in range(3):
        assert rel(A1[:, c], A0[:, c]) <= TOL32, (c, rel(A1[:, c], A0[:, c]))
    assert np.abs(c1).max() <= 1e-6 * np.abs(A0).max()


def test_sobolev_torus40k_sampled(tp, torus40k):
    """The 40,000-face torus with three columns (one launch of the pair kernel, the
    configuration the benchmark times): sampled vertices against the oracle; symmetry
    u^T A v = v^T A u and A 1 = 0 at full size."""
    m = torus40k
    print("[parity] sobolev torus40k", flush=True)
    u = mg.random_columns(m.nV, 3, 3)
    v = mg.random_columns(m.nV, 3, 4)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        Au = P.sobolev_apply(dev(u)).cpu().numpy()
        Av = P.sobolev_apply(dev(v)).cpu().numpy()
        A1 = P.sobolev_apply(torch.ones((m.nV, 1), dtype=torch.float64, device="cuda")).cpu().numpy()
    verts = np.random.default_rng(1).choice(m.nV, 24, replace=False)
    A0 = O.sobolev_at_vertices(m.V, m.F, u, verts, S_SOB)
    assert rel(Au[verts], A0) <= TOL32, rel(Au[verts], A0)
    for c in range(3):
        a, b = float(v[:, c] @ Au[:, c]), float(u[:, c] @ Av[:, c])
        scale = np.linalg.norm(v[:, c]) * np.linalg.norm(Au[:, c])
        assert abs(a - b) <= TOL32 * scale, (c, a, b, scale)
    assert np.abs(A1).max() <= 1e-6 * np.abs(Au).max()


def test_sobolev_errors(tp, meshes):
    m = meshes["small_sphere"]
    V, F = dev(m.V), dev(m.F, torch.int32)
    with tp.Problem(V, F) as P:
        for k in (0, 65):
            st = tp.lib().tp_problem_sobolev_apply(P._h, V.data_ptr(), k, V.data_ptr())
            assert st == 1, st
        assert tp.lib().tp_problem_sobolev_apply(P._h, None, 3, V.data_ptr()) == 1


# ------------------------------------------------------------- GMRES on A = B + B0

def _dense_sobolev(m):
    """Dense A from the oracle's products with the unit vectors (small meshes only)."""
    n = m.nV
    A = np.empty((n, n))
    for c0 in range(0, n, 64):
        c1 = min(n, c0 + 64)
        E = np.zeros((n, c1 - c0))
        E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
        A[:, c0:c1] = O.sobolev_apply(m.V, m.F, E, S_SOB)
    return 0.5 * (A + A.T)


def _mean_zero(x):
    return x - x.mean(0)


def _solve_mesh(meshes, name):
    # two linked tori on 25 x 11 grids: a regular grid whose sizes are both multiples of 3
    # has vertex 3-colourings whose face averages vanish, which L^sigma (and so the
    # preconditioner) annihilates; these sizes avoid them
    if name == "linked_25x11":
        return mg.linked_tori(25, 11, 1.0, 0.25, 1.0)
    return meshes[name]


@pytest.mark.parametrize("name,precond", [("small_sphere", 0), ("small_sphere", 1), ("linked_25x11", 1)])
def test_sobolev_solve_fp64(tp, meshes, name, precond):
    """GMRES with FP64 pair terms to 1e-10: the residual measured with the oracle's operator,
    global mean zero, and the dense solution within cond(A) x tolerance.  On the two linked
    tori A's null space is the global constants only (the low-order term couples the two
    components), so the relative translation of the tori is part of the solution."""
    m = _solve_mesh(meshes, name)
    print(f"[parity] sobolev solve fp64 {name} precond={precond}", flush=True)
    b = mg.random_columns(m.nV, 3, 11)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32), tp.default_params(precision=2)) as P:
        x, rep = P.sobolev_solve(dev(b), rtol=1e-10, restart=40, maxiter=800, precond=precond)
    x = x.cpu().numpy()
    print("  report", rep, flush=True)
    Pb = _mean_zero(b)
    r = Pb - O.sobolev_apply(m.V, m.F, x, S_SOB)
    for c in range(3):
        assert np.linalg.norm(r[:, c]) <= 1e-9 * np.linalg.norm(Pb[:, c]), c
    assert np.abs(x.mean(0)).max() <= 1e-12 * np.abs(x).max()
    A = _dense_sobolev(m)
    ev = np.linalg.eigvalsh(A)
    assert ev[1] > 1e-8 * ev[-1]     # the null space is the global constants alone
    one = np.ones((m.nV, 1))
    xs = np.linalg.solve(A + one @ one.T, Pb)
    cond = ev[-1] / ev[1]
    assert rel(x, xs) <= 10.0 * cond * 1e-10, (rel(x, xs), cond)


def test_sobolev_solve_fp32(tp, meshes):
    """Default precision (FP32 pair terms) to 1e-6 on a two-component mesh: the reported
    true residual meets the tolerance, and the residual with the oracle's operator is within
    the FP32 operator's own error (about 3e-7 of |A x|, measured above) of it."""
    m = _solve_mesh(meshes, "linked_25x11")
    print("[parity] sobolev solve fp32", flush=True)
    b = mg.random_columns(m.nV, 3, 12)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        x, rep = P.sobolev_solve(dev(b), rtol=1e-6, restart=30, maxiter=300)
    x = x.cpu().numpy()
    print("  report", rep, flush=True)
    assert rep["relres"] <= 1e-6
    Pb = _mean_zero(b)
    r = Pb - O.sobolev_apply(m.V, m.F, x, S_SOB)
    for c in range(3):
        assert np.linalg.norm(r[:, c]) <= 3e-6 * np.linalg.norm(Pb[:, c]), c


def test_sobolev_solve_sphere20k(tp):
    """A 20,480-face noisy icosphere (irregular vertex degrees), three columns (the descent
    direction's right-hand side dE) to 1e-5 with FP32 pair terms: the reported residual
    meets it; A x against the oracle at sampled vertices equals P b there up to the
    tolerance and the operator's FP32 error."""
    m = mg.add_noise(mg.icosphere(5), 0.003, 21)
    print("[parity] sobolev solve sphere20k", flush=True)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        _, dE = P.gradient()
        x, rep = P.sobolev_solve(dE, rtol=1e-5, restart=50, maxiter=500)
        b = dE.cpu().numpy()
    x = x.cpu().numpy()
    print("  report", rep, flush=True)
    assert rep["relres"] <= 1e-5
    # with the diagonal term the spread of the preconditioned spectrum stays small: the
    # paper's preconditioner alone does not reach 1e-3 here within 200 iterations
    assert rep["iters"] <= 40, rep
    Pb = b - b.mean(0)
    verts = np.random.default_rng(2).choice(m.nV, 16, replace=False)
    Ax = O.sobolev_at_vertices(m.V, m.F, x, verts, S_SOB)
    # sampled rows: the residual there is bounded by the whole residual
    assert np.linalg.norm(Ax - Pb[verts]) <= 2e-5 * np.linalg.norm(Pb), np.linalg.norm(Ax - Pb[verts])


def test_sobolev_solve_cap_and_errors(tp, meshes):
    m = meshes["small_sphere"]
    b = dev(mg.random_columns(m.nV, 2, 13))
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        x, rep = P.sobolev_solve(b, rtol=1e-14, restart=5, maxiter=3, check=False)
        assert rep["status"] == 5 and rep["iters"] == 3, rep          # TP_E_NOT_CONVERGED
        assert np.isfinite(x.cpu().numpy()).all()
        L = tp.lib()
        r = tp.GmresReport()
        import ctypes
        for args in [(0.0, 10, 10), (1e-6, 0, 10), (1e-6, 10, 0), (1e-6, 101, 10)]:
            st = L.tp_problem_sobolev_solve(P._h, b.data_ptr(), 2, args[0], args[1], args[2], 1, x.data_ptr(),
                                            ctypes.byref(r))
            assert st == 1, (args, st)
        st = L.tp_problem_sobolev_solve(P._h, b.data_ptr(), 2, 1e-6, 10, 10, 2, x.data_ptr(), ctypes.byref(r))
        assert st == 1, st


@pytest.mark.parametrize("prec,rtol,tol", [(2, 1e-10, 1e-6), (0, 1e-5, 1e-3), (0, 1e-4, 1e-2)])
def test_step_true_operator(tp, meshes, prec, rtol, tol):
    """A descent step whose direction uses A_3^{-1} by GMRES (solver = 1) against the
    oracle's step with the dense A^+ (fixed tau): direction, new vertices, constraints."""
    m = meshes["small_sphere"]
    print(f"[parity] step with GMRES on A, precision={prec}", flush=True)
    tau = 2e-3
    ref = O.precond_step(m.V, m.F, tau=tau, line_search=False, inverse=O.dense_sobolev_inverse(m.V, m.F, S_SOB))
    with tp.Problem(dev(m.V), dev(m.F, torch.int32), tp.default_params(precision=prec)) as P:
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        rep = P.step(tp.step_opts(tau0=tau, line_search=0, solver=1, solver_rtol=rtol, solver_maxiter=400),
                     direction=d)
        Vn = P.vertices().cpu().numpy()
    x = d.cpu().numpy()
    print("  gmres iters", rep.cg_iters[0], "relres", rep.cg_relres[0], "precond cg", rep.cg_iters[1],
          "direction error", rel(x, ref.direction), flush=True)
    assert rel(x, ref.direction) <= tol, rel(x, ref.direction)
    assert rel(Vn - m.V, ref.V - m.V) <= tol
    assert rep.slope < 0
    assert np.abs(np.asarray(rep.phi_after)).max() <= 10 * np.abs(ref.phi_after).max() + 1e-12


def test_sobolev_solve_many_components(tp):
    """17 separate noisy icosahedra (more components than the coarse solve takes): the solve
    is the Galerkin one on the functions of mean zero per component, P A x = P b with P the
    per-component mean removal; checked against the dense oracle solution of that system."""
    base = mg.add_noise(mg.icosahedron(), 0.05, 5)
    nc = 17
    offs = [np.array([3.0 * (q % 5), 3.0 * (q // 5), 0.4 * q]) for q in range(nc)]
    V = np.concatenate([base.V + o for o in offs])
    F = np.concatenate([base.F + q * base.nV for q in range(nc)]).astype(np.int32)
    n = V.shape[0]
    print("[parity] sobolev solve with 17 components", flush=True)
    b = mg.random_columns(n, 2, 17)
    with tp.Problem(dev(V), dev(F, torch.int32), tp.default_params(precision=2)) as P:
        x, rep = P.sobolev_solve(dev(b), rtol=1e-10, restart=40, maxiter=400)
    x = x.cpu().numpy()
    print("  report", rep, flush=True)
    _, labels = O.components(F, n)
    Q = np.stack([(labels == l).astype(float) for l in range(nc)], 1)
    Pc = np.eye(n) - Q @ np.diag(1.0 / Q.sum(0)) @ Q.T
    A = _dense_sobolev(mg.Mesh(V, F))
    xs = np.linalg.solve(Pc @ A @ Pc + Q @ Q.T, Pc @ b)
    assert np.abs(Q.T @ x).max() <= 1e-10 * np.abs(x).max()
    assert rel(x, xs) <= 1e-7, rel(x, xs)


def test_sobolev_solve_multi_launch_preconditioner(tp, sphere41k):
    """41K-vertex sphere: the preconditioner's Poisson solves take the multi-launch form
    (more blocks than one cooperative launch holds); GMRES to 1e-4 on dE, A x against the
    oracle at sampled vertices."""
    m = sphere41k
    print("[parity] sobolev solve sphere41k", flush=True)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        _, dE = P.gradient()
        x, rep = P.sobolev_solve(dE, rtol=1e-4, restart=50, maxiter=200)
        b = dE.cpu().numpy()
    x = x.cpu().numpy()
    print("  report", rep, flush=True)
    assert rep["relres"] <= 1e-4 and rep["iters"] <= 40, rep
    Pb = b - b.mean(0)
    verts = np.random.default_rng(3).choice(m.nV, 8, replace=False)
    Ax = O.sobolev_at_vertices(m.V, m.F, x, verts, S_SOB)
    assert np.linalg.norm(Ax - Pb[verts]) <= 2e-4 * np.linalg.norm(Pb), np.linalg.norm(Ax - Pb[verts])


def test_step_penalties(tp, meshes):
    """Area and volume potentials in place of the hard constraints (targets 10 % off the
    current values, so the potentials' gradients matter): the step at fixed tau against the
    oracle's, and the reported total objective."""
    m = meshes["small_sphere"]
    print("[parity] step with area and volume potentials", flush=True)
    A0, V0 = 0.9 * O.total_area(m.V, m.F), 1.1 * O.total_volume(m.V, m.F)
    tau = 2e-3
    ref = O.precond_step(m.V, m.F, tau=tau, line_search=False, constrain_area=False, constrain_volume=False,
                         area_target=A0, volume_target=V0, area_penalty=5.0, volume_penalty=5.0)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        rep = P.step(tp.step_opts(tau0=tau, line_search=0, constrain_area=0, constrain_volume=0, area_target=A0,
                                  volume_target=V0, area_penalty=5.0, volume_penalty=5.0), direction=d)
        Vn = P.vertices().cpu().numpy()
    x = d.cpu().numpy()
    print("  direction error", rel(x, ref.direction), "E", rep.E, ref.E, flush=True)
    assert rel(x, ref.direction) <= 1e-4, rel(x, ref.direction)
    assert rel(Vn - m.V, ref.V - m.V) <= 1e-4
    assert abs(rep.E - ref.E) <= TOL32 * ref.E
    E_new = O.energy(Vn, m.F) + O.penalty_terms(Vn, m.F, A0, V0, 5.0, 5.0)[0]
    assert abs(rep.E_new - E_new) <= TOL32 * E_new
    assert rep.slope < 0
    # a zero target (the potential divides by it) is an argument error before any work
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        for kw in (dict(volume_target=0.0, volume_penalty=1.0), dict(area_target=0.0, area_penalty=1.0)):
            with pytest.raises(tp.TpError) as ei:
                P.step(tp.step_opts(constrain_area=0, constrain_volume=0, **kw))
            assert ei.value.status == 1, ei.value
        assert np.array_equal(P.vertices().cpu().numpy(), m.V)


def _obstacle_mesh():
    ob = mg.add_noise(mg.icosphere(2), 0.02, 9)   # 320 faces (a ragged last LDS tile)
    return 0.4 * ob.V + np.array([1.6, 0.3, -0.1]), ob.F


@pytest.mark.parametrize("p", [6.0, 4.5])
def test_obstacle_energy(tp, meshes, p):
    """Obstacle potential and its differential (FP64 pair terms) against the oracle."""
    m = meshes["small_sphere"]
    Vo, Fo = _obstacle_mesh()
    print(f"[parity] obstacle potential p={p}", flush=True)
    E0, g0 = O.obstacle(m.V, m.F, Vo, Fo, p)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        P.set_obstacle(dev(Vo), dev(Fo, torch.int32), p=p, weight=1.0)
        E1, g1 = P.obstacle_energy()
    assert abs(E1 - E0) <= 1e-12 * E0, (E1, E0)
    assert rel(g1.cpu().numpy(), g0) <= 1e-11


def test_step_obstacle(tp, meshes):
    """A step with the obstacle potential (weight 0.05) and both hard constraints, fixed tau,
    against the oracle's step; the total objective in the report."""
    m = meshes["small_sphere"]
    Vo, Fo = _obstacle_mesh()
    print("[parity] step with an obstacle", flush=True)
    tau, w = 2e-3, 0.05
    ref = O.precond_step(m.V, m.F, tau=tau, line_search=False, obstacle_mesh=(Vo, Fo), obstacle_weight=w)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        P.set_obstacle(dev(Vo), dev(Fo, torch.int32), p=6.0, weight=w)
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        rep = P.step(tp.step_opts(tau0=tau, line_search=0), direction=d)
        Vn = P.vertices().cpu().numpy()
        with pytest.raises(tp.TpError):
            P.set_obstacle(dev(Vo), dev(Fo, torch.int32), p=-1.0, weight=1.0)
    x = d.cpu().numpy()
    print("  direction error", rel(x, ref.direction), flush=True)
    assert rel(x, ref.direction) <= 1e-4, rel(x, ref.direction)
    assert rel(Vn - m.V, ref.V - m.V) <= 1e-4
    assert abs(rep.E - ref.E) <= TOL32 * ref.E
    E_new = O.energy(Vn, m.F) + w * O.obstacle(Vn, m.F, Vo, Fo, 6.0, False)[0]
    assert abs(rep.E_new - E_new) <= TOL32 * E_new


def test_step_barycenter_motion(tp, meshes):
    """Barycenter motions on two linked tori (per-component translations added back), fixed
    tau, against the oracle's step."""
    m = meshes["linked_small"]
    print("[parity] step with barycenter motions", flush=True)
    tau = 2e-3
    ref = O.precond_step(m.V, m.F, tau=tau, line_search=False, barycenter_motion=True)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        rep = P.step(tp.step_opts(tau0=tau, line_search=0, barycenter_motion=1), direction=d)
        Vn = P.vertices().cpu().numpy()
    x = d.cpu().numpy()
    print("  direction error", rel(x, ref.direction), flush=True)
    assert rel(x, ref.direction) <= 1e-4, rel(x, ref.direction)
    assert rel(Vn - m.V, ref.V - m.V) <= 1e-4
    assert abs(rep.slope - float(np.vdot(O.gradient(m.V, m.F)[1], ref.direction))) <= 1e-4 * abs(rep.slope)


IMPLICIT = [dict(kind=0, q=[0.0, 0.2, 1.0], c=-2.0, p=6.0, w=0.5, attract=False),
            dict(kind=1, q=[0.1, -0.2, 0.3], c=3.0, p=2.0, w=0.3, attract=True)]


def _add_implicit(P, prims):
    for pr in prims:
        P.add_implicit(pr["kind"], pr["q"], pr["c"], p=pr["p"], weight=pr["w"], attract=pr["attract"])


def test_implicit_energy(tp, meshes):
    """Implicit plane obstacle and sphere attractor against the oracle (FP64)."""
    m = meshes["small_sphere"]
    print("[parity] implicit potentials", flush=True)
    E0, g0 = O.implicit_potential(m.V, m.F, IMPLICIT)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        _add_implicit(P, IMPLICIT)
        E1, g1 = P.implicit_energy()
        with pytest.raises(tp.TpError):
            P.add_implicit(1, [0, 0, 0], -1.0)     # radius must be positive
    assert abs(E1 - E0) <= 1e-12 * abs(E0), (E1, E0)
    assert rel(g1.cpu().numpy(), g0) <= 1e-11


def test_step_implicit(tp, meshes):
    """A step with the implicit potentials and both hard constraints, fixed tau, against the
    oracle's step."""
    m = meshes["small_sphere"]
    print("[parity] step with implicit potentials", flush=True)
    tau = 2e-3
    ref = O.precond_step(m.V, m.F, tau=tau, line_search=False, implicit=IMPLICIT)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        _add_implicit(P, IMPLICIT)
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        rep = P.step(tp.step_opts(tau0=tau, line_search=0), direction=d)
        Vn = P.vertices().cpu().numpy()
    x = d.cpu().numpy()
    print("  direction error", rel(x, ref.direction), flush=True)
    assert rel(x, ref.direction) <= 1e-4, rel(x, ref.direction)
    assert rel(Vn - m.V, ref.V - m.V) <= 1e-4
    assert abs(rep.E - ref.E) <= TOL32 * ref.E
    E_new = O.energy(Vn, m.F) + O.implicit_potential(Vn, m.F, IMPLICIT, False)[0]
    assert abs(rep.E_new - E_new) <= TOL32 * E_new


@pytest.mark.parametrize("p", [6.0, 3.0])
def test_step_implicit_barrier(tp, meshes, p):
    """A plane just below the mesh that the first Armijo trial would cross (Sec. 7.3.3): the
    barrier is +infinity there for even and odd p, so the GPU line search halves the step
    like the oracle's and every barycenter of the result stays above the plane."""
    m = meshes["small_sphere"]
    print(f"[parity] implicit barrier p={p}", flush=True)
    zmin = O.faces(m.V, m.F)[0][:, 2].min()
    plane = [dict(kind=0, q=[0.0, 0.0, 1.0], c=zmin - 0.02, p=p, w=1e-14, attract=False)]
    ref = O.precond_step(m.V, m.F, constrain_area=False, constrain_volume=False, implicit=plane)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        _add_implicit(P, plane)
        rep = P.step(tp.step_opts(constrain_area=0, constrain_volume=0))
        Vn = P.vertices().cpu().numpy()
    assert rep.backtracks == ref.backtracks and abs(rep.tau - ref.tau) <= 1e-6 * ref.tau
    assert O.faces(Vn, m.F)[0][:, 2].min() > zmin - 0.02
    assert math.isfinite(rep.E_new)
    assert rel(Vn - m.V, ref.V - m.V) <= 1e-4


def test_step_warm_start(tp, meshes):
    """Warm-started Poisson solves (the previous step's solutions as initial guesses): the
    first step starts from zero; later steps start warm, need fewer iterations than cold
    solves of the same systems, and give the same steps to the solver tolerance."""
    m = meshes["torus37x23"]
    print("[parity] warm-started steps", flush=True)
    out = {}
    for warm in (0, 1):
        with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
            reps = [P.step(tp.step_opts(warm_start=warm)) for _ in range(3)]
            out[warm] = (P.vertices().cpu().numpy(), reps)
    (Vc, cold), (Vw, warm) = out[0], out[1]
    assert [r.warm_started for r in cold] == [0, 0, 0]
    assert [r.warm_started for r in warm] == [0, 1, 1]
    assert list(warm[0].cg_iters) == list(cold[0].cg_iters)
    for s in (1, 2):
        print(f"  step {s}: iterations cold {list(cold[s].cg_iters)} warm {list(warm[s].cg_iters)}", flush=True)
        assert sum(warm[s].cg_iters) < sum(cold[s].cg_iters)
        # tau0 follows the direction's largest vertex move, equal to the solver tolerance
        assert abs(warm[s].tau - cold[s].tau) <= 1e-6 * cold[s].tau and warm[s].backtracks == cold[s].backtracks
        assert max(warm[s].cg_relres) <= 1e-10
    assert rel(Vw - m.V, Vc - m.V) <= 1e-7


@pytest.mark.parametrize("name", ["torus37x23", "linked_small"])
def test_setup_beside_pair_work(tp, meshes, name):
    """After a solve, new vertex positions start the cotan values and the preconditioner's
    set-up on a second stream, beside the energy, differential and fractional launches that
    follow.  Everything computed then equals bit for bit what a problem of the same face
    order computes with the set-up done in line: after one change of positions, after two
    changes in a row (the second waits for the first's set-up before it overwrites the
    positions), and with pins set while a set-up runs."""
    m = meshes[name]
    print(f"[parity] set-up beside the pair work {name}", flush=True)
    rng = np.random.default_rng(11)
    V1 = m.V + 2e-3 * rng.standard_normal(m.V.shape)
    V2 = m.V + 4e-3 * rng.standard_normal(m.V.shape)
    F = dev(m.F, torch.int32)
    b = dev(mg.random_columns(m.nV, 3, 4))
    u = dev(mg.random_columns(m.nV, 3, 5))
    _, labels = O.components(m.F, m.nV)
    pins = [int(np.nonzero(labels == 0)[0][7])]

    def run(P):
        E, g = P.gradient()
        Lu = P.fractional_apply(u)
        x, rep = P.precond_apply(b)
        return E, g.cpu().numpy(), Lu.cpu().numpy(), x.cpu().numpy(), list(rep.cg_iters)

    def in_line(V, with_pins=False):
        # face order and block partition from m.V, as for the problem below; the first new
        # positions start a set-up that the second call waits for and discards, so the
        # set-up for V runs in line, on the problem's stream
        with tp.Problem(dev(m.V), F) as Q:
            Q.precond_apply(b)
            Q.set_vertices(dev(V))
            Q.set_vertices(dev(V))
            if with_pins:
                Q.set_pins(pins)
            return run(Q)

    def same(got, ref):
        assert got[0] == ref[0]
        for a, r in zip(got[1:4], ref[1:4]):
            assert np.array_equal(a, r)
        assert got[4] == ref[4]

    ref1, ref2, ref1p = in_line(V1), in_line(V2), in_line(V1, True)
    with tp.Problem(dev(m.V), F) as P:
        P.precond_apply(b)
        P.set_vertices(dev(V1))          # starts the set-up beside the pair work
        same(run(P), ref1)
        P.set_vertices(dev(V2))
        P.set_vertices(dev(V1))          # waits for the set-up of V2 first
        same(run(P), ref1)
        P.set_vertices(dev(V2))
        same(run(P), ref2)
        P.set_vertices(dev(V1))
        P.set_pins(pins)                 # waits, then the pinned matrix is set up in line
        same(run(P), ref1p)


@pytest.mark.parametrize("name", ["small_sphere", "linked_small"])
def test_step_vertex_pins(tp, meshes, name):
    """Vertex pins (Sec. 7.1.2) as rows of the preconditioner's Laplacians (Sec. 7.2): the
    pinned Poisson solve and the step at fixed tau against the oracle's, the pinned vertices
    exactly in place after two steps; pins combine with neither barycenter motions nor
    solver 1."""
    m = meshes[name]
    _, labels = O.components(m.F, m.nV)
    pins = [3, 40] if name == "small_sphere" else [int(np.nonzero(labels == 0)[0][5])]
    print(f"[parity] vertex pins {name} {pins}", flush=True)
    b = mg.random_columns(m.nV, 3, 4)
    C = O.cotan_laplacian(m.V, m.F)
    x0 = O.poisson_solve(C, b, labels, pins)
    tau = 2e-3
    ref = O.precond_step(m.V, m.F, tau=tau, line_search=False, pins=pins)
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        P.set_pins(pins)
        x, _ = P.poisson_solve(dev(b))
        d = torch.empty((m.nV, 3), dtype=torch.float64, device="cuda")
        P.step(tp.step_opts(tau0=tau, line_search=0), direction=d)
        V1 = P.vertices().cpu().numpy()
        P.step()
        V2 = P.vertices().cpu().numpy()
        with pytest.raises(tp.TpError):
            P.step(tp.step_opts(barycenter_motion=1))
    x = x.cpu().numpy()
    assert rel(x, x0) <= 1e-6 and np.abs(x[pins]).max() == 0.0
    dd = d.cpu().numpy()
    print("  direction error", rel(dd, ref.direction), flush=True)
    assert rel(dd, ref.direction) <= 1e-4
    assert np.abs(dd[pins]).max() == 0.0
    assert rel(V1 - m.V, ref.V - m.V) <= 1e-4
    assert np.array_equal(V1[pins], m.V[pins]) and np.array_equal(V2[pins], m.V[pins])


def test_remesh_then_step(tp):
    """Remeshing between steps (Sec. 6): a stretched noisy sphere is remeshed on the host
    (tp_remesh) and a new problem created from the result; its step decreases the energy
    and keeps the area and volume constraints, like a problem of the original mesh."""
    m = mg.add_noise(mg.icosphere(3), 0.02, 5)
    V = m.V * np.array([1.0, 1.0, 2.5])
    L0 = float(np.mean(np.linalg.norm(V[m.F[:, 0]] - V[m.F[:, 1]], axis=1)))
    Vr, Fr = tp.tp_remesh(V, m.F, L0, iterations=3, rho=0.5)
    print(f"[parity] remesh then step: {m.nF} -> {len(Fr)} faces", flush=True)
    assert len(Fr) != m.nF
    with tp.Problem(dev(Vr), dev(Fr, torch.int32)) as P:
        reps = [P.step() for _ in range(2)]
    for r in reps:
        assert r.E_new < r.E
        for q in range(2):
            assert abs(r.phi_after[q]) <= max(1e-9, abs(r.phi_trial[q]))


def test_profile_counts_every_kind(tp, meshes):
    """The launch timing of the four all-pairs kinds: each profiled call adds one launch,
    its ordered pairs and a positive device time; nothing is counted while disabled, and
    reset clears the figures."""
    m = meshes["torus37x23"]
    print("[parity] profile counts", flush=True)
    nF = m.nF
    u = dev(mg.random_columns(m.nV, 3, 1))
    with tp.Problem(dev(m.V), dev(m.F, torch.int32)) as P:
        def calls():
            P.energy()
            P.gradient()
            P.fractional_apply(u)
            P.sobolev_apply(u)
        calls()
        torch.cuda.synchronize()
        tp.profile_reset()
        tp.profile_enable(True)
        calls()
        calls()
        tp.profile_enable(False)
        calls()
        for kind in (tp.KIND_ENERGY, tp.KIND_GRAD, tp.KIND_FRAC, tp.KIND_SOBOLEV):
            st = tp.profile_get(kind)
            assert st["launches"] == 2, (kind, st)
            assert st["pairs_total"] == 2.0 * nF * (nF - 1), (kind, st)
            assert st["ms_total"] > 0.0, (kind, st)
            cols = 3.0 if kind in (tp.KIND_FRAC, tp.KIND_SOBOLEV) else 0.0
            assert st["cols_total"] == cols * st["pairs_total"], (kind, st)
        tp.profile_reset()
        assert all(tp.profile_get(k)["launches"] == 0 for k in range(4))
