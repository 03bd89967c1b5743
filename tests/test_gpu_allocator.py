"""Device memory through a registered allocator (tp_set_allocator): with PyTorch's caching
allocator registered, a resident problem's device buffers all come from it (the memory
PyTorch reports grows by the problem's device bytes and returns to its start once the
problem is destroyed; every allocation is matched by a free), and the results are the
same as with the library's own hipMalloc buffers."""
import numpy as np
import pytest

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


def _run(tp, m, u):
    V = torch.from_numpy(m.V).cuda()
    F = torch.from_numpy(m.F).cuda()
    with tp.Problem(V, F) as P:
        E, g = P.gradient()
        Lu = P.fractional_apply(u)
        x, _ = P.precond_apply(g)
        rep = P.step(tp.step_opts(tau0=1e-3, line_search=0))
        torch.cuda.synchronize()
        held = P.device_bytes()
        out = (E, g.cpu().numpy(), Lu.cpu().numpy(), x.cpu().numpy(), P.vertices().cpu().numpy(), rep.E_new)
    return out, held


def test_problem_allocates_through_registered_allocator(tp):
    m = mg.workload("small_sphere")
    u = torch.from_numpy(mg.random_columns(m.nV, 3, 1)).cuda()
    print("[allocator] hipMalloc run", flush=True)
    ref, _ = _run(tp, m, u)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    tp.allocator_calls.update(alloc=0, free=0)
    print("[allocator] torch caching allocator run", flush=True)
    tp.use_torch_allocator(True)
    try:
        V = torch.from_numpy(m.V).cuda()
        F = torch.from_numpy(m.F).cuda()
        inputs = torch.cuda.memory_allocated() - base
        with tp.Problem(V, F) as P:
            E, g = P.gradient()
            Lu = P.fractional_apply(u)
            x, _ = P.precond_apply(g)
            rep = P.step(tp.step_opts(tau0=1e-3, line_search=0))
            torch.cuda.synchronize()
            held = P.device_bytes()
            grown = torch.cuda.memory_allocated() - base - inputs
            got = (E, g.cpu().numpy(), Lu.cpu().numpy(), x.cpu().numpy(), P.vertices().cpu().numpy(), rep.E_new)
            outputs = sum(t.numel() * t.element_size() for t in (g, Lu, x))
        # everything the problem holds was allocated by torch (its block rounding aside)
        assert grown - outputs >= held, (grown, outputs, held)
        assert grown - outputs <= held + 512 * tp.allocator_calls["alloc"] + (1 << 20)
        del g, Lu, x
        torch.cuda.synchronize()
        assert tp.allocator_calls["alloc"] > 10
        assert tp.allocator_calls["alloc"] == tp.allocator_calls["free"]
        assert torch.cuda.memory_allocated() - base == inputs
        # a live buffer of the registered allocator blocks switching allocators
        with tp.Problem(V, F) as P2:
            P2.gradient()
            with pytest.raises(tp.TpError):
                tp.use_torch_allocator(False)
    finally:
        tp.use_torch_allocator(False)
    assert got[0] == ref[0] and got[5] == ref[5]
    for a, b in zip(got[1:5], ref[1:5]):
        assert np.array_equal(a, b)
