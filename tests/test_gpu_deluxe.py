"""Deluxe scaling on the GPU against the oracle (paper §3.2: the more robust alternative to the
counting function; weights D_g^(i) = (sum_j S_g^(j))^-1 S_g^(i) computed in the factorisation and
folded into the stored operators).

Checkpoints as in the other parity tests: coarse matrix (unchanged by the scaling, 1e-12), one
application (FP64 max(1e-12, 100 x the oracle's own noise floor), mixed 1e-5), GMRES iterations
(FP64 +-1, mixed <= +2) and true residual; Q1 and Q2 boxes, a ragged partition, the curved Q2
shell, multi-panel subdomains (packed operators), three levels (deluxe on level 1) and deluxe
with near-null-space primals. On a stiff/soft checkerboard the device takes the oracle's
iterations, less than half of the counting function's.
"""
import functools

import numpy as np
import pytest

from oracle import bddc, gmres
from paper_2208_06191_amd import mbddc
from tests.conftest import problem
from tests.test_oracle_deluxe import checkerboard

pytestmark = pytest.mark.gpu

TOL_APPLY = {mbddc.MBDDC_FP64: 1e-12, mbddc.MBDDC_MIXED: 1e-5}
PRECS = [mbddc.MBDDC_FP64, mbddc.MBDDC_MIXED]
# (name, primal, levels, nnsp)
CASES = [("small_ve", 3, 2, 0), ("tiny_q2", 7, 2, 0), ("ragged", 3, 2, 0), ("vent", 7, 2, 0),
         ("large_q1", 3, 2, 0), ("l3_nh", 3, 3, 0), ("vent", 7, 2, 1)]


def _problem(name):
    return checkerboard() if name == "checkerboard" else problem(name)


@functools.lru_cache(maxsize=None)
def oracle(name, primal, levels=2, nnsp=0, scaling="deluxe"):
    P = _problem(name)
    dec = bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                             P.mesh.node_tags, primal=primal, coords=P.mesh.coords, nnsp=bool(nnsp))
    return P, dec, bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke, levels=levels, scaling=scaling)


@functools.lru_cache(maxsize=None)
def noise_floor(name, primal, levels, nnsp):
    P, dec, B = oracle(name, primal, levels, nnsp)
    E = np.random.default_rng(1).standard_normal(P.Ke.shape)
    E = 0.5 * (E + E.transpose(0, 2, 1))
    B2 = bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke * (1.0 + 2.2e-16 * E), levels=levels, scaling="deluxe")
    r = np.random.default_rng(3).standard_normal(P.n_dofs)[dec.free]
    z = B.apply(r)
    return float(np.linalg.norm(z - B2.apply(r)) / np.linalg.norm(z))


def solver(P, primal, precision, levels=2, nnsp=0, scaling=mbddc.MBDDC_SCALING_DELUXE):
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                           mbddc.default_options(primal=primal, precision=precision, symmetric_hint=1, levels=levels,
                                                 nnsp=nnsp, scaling=scaling, keep_coarse_matrix=1))
    s.mbddc_set_tangent(P.Ke)
    s.mbddc_factor()
    return s


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("name,primal,levels,nnsp", CASES)
def test_deluxe_matches_oracle(name, primal, levels, nnsp, precision):
    P, dec, B = oracle(name, primal, levels, nnsp)
    s = solver(P, primal, precision, levels, nnsp)
    if levels == 2:
        err_c = rel(s.mbddc_get_coarse_matrix(0, dec.n_coarse), B.Kc)
        assert err_c <= 1e-12
    r = np.random.default_rng(7).standard_normal((2, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    z = s.mbddc_apply(r)
    err = max(rel(z[k][dec.free], B.apply(r[k][dec.free])) for k in range(2))
    bound = TOL_APPLY[precision]
    if precision == mbddc.MBDDC_FP64:
        bound = max(bound, 100.0 * noise_floor(name, primal, levels, nnsp))
    b = P.rhs[0][dec.free]
    ref = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 1000)
    x, info = s.mbddc_solve(P.rhs[0])
    print(f"{name} levels {levels} nnsp {nnsp} prec {precision}: apply {err:.1e} (bound {bound:.1e}), "
          f"its {info.iterations} (oracle {ref.iterations})")
    assert err <= bound
    assert np.linalg.norm(b - B.A @ x[dec.free]) <= 1e-8 * np.linalg.norm(b)
    if precision == mbddc.MBDDC_FP64:
        assert abs(info.iterations - ref.iterations) <= 1
    else:
        assert info.iterations <= ref.iterations + 2
    s.close()


def test_deluxe_checkerboard_takes_the_oracles_iterations():
    P, dec, B = oracle("checkerboard", 3)
    b = P.rhs[0][dec.free]
    ref = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 2000)
    its = {}
    for scaling in (mbddc.MBDDC_SCALING_COUNTING, mbddc.MBDDC_SCALING_DELUXE):
        s = solver(P, 3, mbddc.MBDDC_FP64, scaling=scaling)
        _, info = s.mbddc_solve(P.rhs[0])
        assert info.rel_res_true <= 1e-8
        its[scaling] = info.iterations
        s.close()
    print(f"checkerboard: counting {its[0]} its, deluxe {its[1]} (oracle {ref.iterations})")
    assert abs(its[1] - ref.iterations) <= 1
    assert 2 * its[1] < its[0]
