"""The C ABI's memory and bookkeeping entry points on the GPU.

* mbddc_set_allocator: every device buffer of a handle (and of its level-2 instance) comes
  from the caller's allocator (here PyTorch's caching allocator); once a handle has factored
  and solved, further Newton steps (set_tangent, factor, solve) allocate nothing; the results
  are bitwise those of the library's own hipMalloc path; every block is handed back.
* a failing allocator surfaces as MBDDC_ERR_OOM, the state rules hold;
* mbddc_release returns the buffers and the handle serves a new setup;
* a non-finite tangent entry is rejected on the device and leaves the factors usable;
* mbddc_get_iterations reports each (instance, right-hand side) system's own count.
"""
import numpy as np
import pytest

from paper_2208_06191_amd import mbddc
from tests.conftest import problem

pytestmark = pytest.mark.gpu


def run_steps(s, P, steps=3, levels=2, nrhs=2):
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                           mbddc.default_options(primal=3, symmetric_hint=1, levels=levels))
    out = []
    for k in range(steps):
        s.mbddc_set_tangent(P.Ke * (1.0 + 0.01 * k))
        s.mbddc_factor()
        x, _ = s.mbddc_solve(np.concatenate([P.rhs] * nrhs)[:nrhs])
        out.append(x)
        if k == 0:
            yield "warm"
    yield out


@pytest.mark.parametrize("name,levels", [("small_ve", 2), ("l3_nh", 3)])
def test_torch_allocator_supplies_every_buffer(name, levels):
    torch = pytest.importorskip("torch")
    P = problem(name)
    A = mbddc.TorchAllocator(0)
    s = mbddc.Solver(0, allocator=A)
    before = torch.cuda.memory_allocated()
    g = run_steps(s, P, levels=levels)
    assert next(g) == "warm"
    n_warm = A.n_alloc
    held = torch.cuda.memory_allocated() - before
    assert n_warm > 10 and held >= s.mbddc_footprint(2) * 0.9
    xs = next(g)
    print(f"{name} levels {levels}: {n_warm} blocks, {held / 1e6:.1f} MB from torch; "
          f"allocations after the first step: {A.n_alloc - n_warm}")
    assert A.n_alloc == n_warm, "a Newton step after the first allocated device memory"
    ref = mbddc.Solver(0)
    xr = list(run_steps(ref, P, levels=levels))[-1]
    ref.close()
    for a, b in zip(xs, xr):
        assert np.array_equal(a, b)
    s.close()
    assert A.n_free == A.n_alloc and not A.blocks


def test_allocator_rules_and_release():
    P = problem("small_ve")
    A = mbddc.TorchAllocator(0)
    s = mbddc.Solver(0)
    L = mbddc.lib()
    import ctypes
    f = ctypes.cast(A.c_alloc, ctypes.c_void_p)
    assert L.mbddc_set_allocator(s._h, f, None, None) == mbddc.MBDDC_ERR_ARG
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)], mbddc.default_options(primal=3))
    assert L.mbddc_set_allocator(s._h, f, ctypes.cast(A.c_free, ctypes.c_void_p), None) == mbddc.MBDDC_ERR_STATE
    s.mbddc_release()                      # back to the created state: the allocator may change
    assert L.mbddc_set_allocator(s._h, f, ctypes.cast(A.c_free, ctypes.c_void_p), None) == mbddc.MBDDC_OK
    s.allocator = A
    with pytest.raises(mbddc.MbddcError) as e:
        s.mbddc_factor()
    assert e.value.status == mbddc.MBDDC_ERR_STATE
    xs = list(run_steps(s, P, steps=1))[-1]
    assert A.n_alloc > 0
    s.mbddc_release()
    assert A.n_free == A.n_alloc and not A.blocks
    xs2 = list(run_steps(s, P, steps=1))[-1]   # the same handle set up again
    assert np.array_equal(xs[0], xs2[0])
    s.close()


class FailingAllocator(mbddc.TorchAllocator):
    def __init__(self, limit):
        super().__init__(0)
        self.limit = limit

    def _alloc(self, nbytes, user):
        if self.n_alloc >= self.limit:
            return None
        return super()._alloc(nbytes, user)


def test_failing_allocator_reports_oom_and_keeps_nothing():
    P = problem("small_ve")
    A = FailingAllocator(5)
    s = mbddc.Solver(0, allocator=A)
    with pytest.raises(mbddc.MbddcError) as e:
        s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)], mbddc.default_options(primal=3))
    assert e.value.status == mbddc.MBDDC_ERR_OOM
    assert A.n_free == A.n_alloc and not A.blocks
    s.close()


def test_nonfinite_tangent_rejected_on_device_keeps_factors():
    torch = pytest.importorskip("torch")
    P = problem("small_ve")
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)], mbddc.default_options(primal=3))
    s.mbddc_set_tangent(P.Ke)
    s.mbddc_factor()
    x0, _ = s.mbddc_solve(P.rhs)
    for bad_value in (np.nan, np.inf):
        bad = P.Ke.copy()
        bad[-1, 5, 7] = bad_value
        for Ke in (bad, torch.tensor(bad, device="cuda")):
            with pytest.raises(mbddc.MbddcError) as e:
                s.mbddc_set_tangent(Ke)
            assert e.value.status == mbddc.MBDDC_ERR_ARG
    x1, _ = s.mbddc_solve(P.rhs)              # operator and factors untouched
    assert np.array_equal(x0, x1)
    s.close()


def test_iterations_per_system():
    Pa, Pb = problem("small_ve"), problem("tiny_nh")
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(Pa), mbddc.mesh_from_problem(Pb)],
                           mbddc.default_options(primal=3, precision=mbddc.MBDDC_FP64))
    s.mbddc_set_tangent(np.concatenate([Pa.Ke.ravel(), Pb.Ke.ravel()]))
    s.mbddc_factor()
    rng = np.random.default_rng(2)
    b = rng.standard_normal((3, Pa.n_dofs + Pb.n_dofs))
    _, info = s.mbddc_solve(b)
    its = s.mbddc_get_iterations()
    assert its.shape == (2, 3) and its.max() == info.iterations
    for k in range(3):   # each system alone: the same count
        _, i1 = s.mbddc_solve(b[k])
        one = s.mbddc_get_iterations()
        assert one.shape == (2, 1) and list(one[:, 0]) == list(its[:, k])
        assert i1.iterations == its[:, k].max()
    s.close()
