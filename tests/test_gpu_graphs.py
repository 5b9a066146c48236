"""Graph-replayed preconditioner application.

GMRES replays the BDDC apply (every phase, two and three levels) from an HIP graph
captured at the first iteration for each right-hand-side width. The graph runs the
same kernels in the same order as the eager launches, so every result must be
bitwise identical to the eager path: over many replays within one solve, across
solves with eager work in between, across widths (recapture after the apply
buffers move) and through the public apply entry point.
"""
import numpy as np
import pytest

from paper_2208_06191_amd import mbddc
from tests.conftest import problem

pytestmark = pytest.mark.gpu

CASES = [("small_ve", 3, 2), ("tiny_q2", 7, 2), ("l3_nh", 3, 3)]


def handle(P, primal, levels, graph, precision=mbddc.MBDDC_MIXED):
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                           mbddc.default_options(precision=precision, primal=primal, symmetric_hint=1,
                                                 levels=levels, graph_apply=graph))
    s.mbddc_set_tangent(P.Ke)
    s.mbddc_factor()
    return s


@pytest.mark.parametrize("name,primal,levels", CASES)
def test_graph_solves_equal_eager_bitwise(name, primal, levels):
    P = problem(name)
    g = handle(P, primal, levels, 1)
    e = handle(P, primal, levels, 0)
    rng = np.random.default_rng(5)
    for rep in range(3):
        b = P.rhs * (1.0 + rep) + (rep > 0) * 0.1 * rng.standard_normal(P.rhs.shape)
        b[:, P.dirichlet] = 0.0
        xg, ig = g.mbddc_solve(b)
        xe, ie = e.mbddc_solve(b)
        assert ig.applies > 2 and ig.applies_graphed == ig.applies
        assert ie.applies == ig.applies and ie.applies_graphed == 0
        assert ig.iterations == ie.iterations
        assert np.array_equal(xg, xe), f"replay {rep}: max diff {np.abs(xg - xe).max()}"
        assert ig.rel_res_true <= 1e-8
        # eager work on the same handle between the solves
        y = g.mbddc_matvec(xg)
        assert np.all(np.isfinite(y))


def test_width_changes_recapture():
    P = problem("small_ve")
    g = handle(P, 3, 2, 1)
    e = handle(P, 3, 2, 0)
    b = np.concatenate([P.rhs, 0.5 * P.rhs[::-1]], axis=0)      # 4 right-hand sides
    for rhs in (P.rhs[:1], b, P.rhs, P.rhs[:1], b):
        xg, ig = g.mbddc_solve(rhs)
        xe, _ = e.mbddc_solve(rhs)
        assert ig.applies_graphed == ig.applies
        assert np.array_equal(xg, xe)


@pytest.mark.parametrize("levels", [2, 3])
def test_public_apply_uses_the_graph(levels):
    P = problem("l3_nh")
    g = handle(P, 3, levels, 1)
    e = handle(P, 3, levels, 0)
    r = np.random.default_rng(11).standard_normal((3, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    for k in range(3):
        assert np.array_equal(g.mbddc_apply(r * (k + 1)), e.mbddc_apply(r * (k + 1)))


def test_profiled_applies_run_eagerly():
    P = problem("small_ve")
    g = handle(P, 3, 2, 1)
    bits = {n: i for i, n in enumerate(mbddc.profile_families())}
    g.mbddc_set_profiling(1 << bits["apply_C_interface"])
    x1, i1 = g.mbddc_solve(P.rhs)
    assert i1.applies_graphed == 0
    g.mbddc_set_profiling(1 << bits["spmv_bsr"])
    x2, i2 = g.mbddc_solve(P.rhs)
    assert i2.applies_graphed == i2.applies
    g.mbddc_set_profiling(0)
    assert np.array_equal(x1, x2)


@pytest.mark.parametrize("levels", [2, 3])
def test_overlapped_extraction_equals_sequential(levels):
    """The apply operators are extracted on a side stream while the coarse problem is factorised,
    except while the factorisation's families are profiled: both orders give identical results."""
    P = problem("l3_nh")
    a = handle(P, 3, levels, 1)
    b = mbddc.Solver(0)
    b.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                           mbddc.default_options(precision=mbddc.MBDDC_MIXED, primal=3, symmetric_hint=1,
                                                 levels=levels))
    b.mbddc_set_tangent(P.Ke)
    b.mbddc_set_profiling(0xFFFFFFFF)          # every family timed: sequential extraction
    b.mbddc_factor()
    b.mbddc_set_profiling(0)
    b.mbddc_get_profile()
    xa, ia = a.mbddc_solve(P.rhs)
    xb, ib = b.mbddc_solve(P.rhs)
    assert ia.iterations == ib.iterations and np.array_equal(xa, xb)
