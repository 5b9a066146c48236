"""The no-allocation entry point mbddc_matvec_noalloc (for callers that cannot allocate device
memory): the same operator product as mbddc_matvec, its staging blocks in the library's static
device buffer. Checked bitwise against mbddc_matvec on two calls in a row (the second with a
smaller input), on a second handle, and its size and state limits; no allocation is made."""
import numpy as np
import pytest

from paper_2208_06191_amd import mbddc
from paper_2208_06191_amd import workloads as W
from tests.conftest import problem

pytestmark = pytest.mark.gpu


def handle(P):
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)], mbddc.default_options(primal=3))
    s.mbddc_set_tangent(P.Ke)
    return s


def test_noalloc_matvec_equals_matvec_on_consecutive_calls():
    torch = pytest.importorskip("torch")
    P, Q = problem("q2_dense"), problem("small_ve")
    sp, sq = handle(P), handle(Q)
    rng = np.random.default_rng(4)
    cases = [(sp, P, 5), (sp, P, 2), (sq, Q, 1), (sp, P, 8), (sq, Q, 3)]   # each later call smaller or on another handle
    for s, R, nrhs in cases:
        x = torch.tensor(rng.standard_normal((nrhs, R.n_dofs)), device="cuda")
        ref = s.mbddc_matvec(x)
        out = torch.full_like(x, float("nan"))
        before = torch.cuda.memory_allocated()
        s.mbddc_matvec_noalloc(x, out)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert torch.equal(out, ref), (R.name, nrhs)
        # against the operator itself: clamped entries zero
        assert float(out[:, torch.as_tensor(R.dirichlet, device="cuda").long()].abs().max()) == 0.0
    sp.close()
    sq.close()


def test_noalloc_matvec_limits():
    torch = pytest.importorskip("torch")
    mesh = W.box_mesh(36, 36, 36, 1)                      # 151,959 DOFs
    part, nsub = W.block_partition(mesh, 4)
    m = mbddc._MeshArrays(mesh.coords, mesh.elem_nodes, mesh.elem_type, part, nsub, mesh.node_tags,
                          W.clamp_dofs(mesh, 1))
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([m], mbddc.default_options(primal=3))
    n = 3 * mesh.n_nodes
    x8 = torch.zeros((8, n), dtype=torch.float64, device="cuda")
    with pytest.raises(mbddc.MbddcError) as e:           # 2 x 8 x 151,959 doubles > 16 MiB
        s.mbddc_matvec_noalloc(x8, torch.empty_like(x8))
    assert e.value.status == mbddc.MBDDC_ERR_UNSUPPORTED
    x4 = torch.zeros((4, n), dtype=torch.float64, device="cuda")
    with pytest.raises(mbddc.MbddcError) as e:           # fits, but no tangent yet
        s.mbddc_matvec_noalloc(x4, torch.empty_like(x4))
    assert e.value.status == mbddc.MBDDC_ERR_STATE
    s.close()
