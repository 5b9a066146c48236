"""The non-symmetric BDDC formulation on the GPU (general path, symmetric_hint = 0), against
the oracle's (paper §8: a tangent whose symmetry is broken, as by the base pressure of the
realistic simulation, needs the non-symmetric form of BDDC).

The tangents are the problems' element tangents plus a seeded skew-symmetric part (5 % of the
largest entry), as a follower load would add. Checkpoints: one application against the oracle
(FP64 max(1e-12, 100 x the oracle's own change under a relative-eps perturbation of K_e); mixed
1e-5), with the left coarse basis (nonsym_coarse = 1, the default) against the oracle's
non-symmetric form and with Psi = Phi against its symmetric form; GMRES iterations (FP64 +-1,
mixed <= +2) and true residuals; two and three levels; and the adjoint property of the
non-symmetric form on the device: the preconditioner built from K^T is the transpose of the one
built from K.
"""
import functools

import numpy as np
import pytest

from oracle import bddc, gmres
from paper_2208_06191_amd import mbddc
from paper_2208_06191_amd import workloads as W
from tests.conftest import problem

pytestmark = pytest.mark.gpu

TOL_APPLY = {mbddc.MBDDC_FP64: 1e-12, mbddc.MBDDC_MIXED: 1e-5}


def skew(Ke, seed=3, eps=0.05):
    S = np.random.default_rng(seed).standard_normal(Ke.shape)
    return Ke + eps * np.abs(Ke).max() * (S - np.transpose(S, (0, 2, 1)))


@functools.lru_cache(maxsize=None)
def case(name):
    P = problem(name)
    return P, skew(P.Ke)


@functools.lru_cache(maxsize=None)
def oracle(name, primal, nonsym, levels=2, group=8):
    P, Ke = case(name)
    dec = bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                             P.mesh.node_tags, primal=primal)
    return dec, bddc.BDDC(dec, P.mesh.elem_nodes, Ke, levels=levels, coarse_group=group, nonsymmetric=nonsym)


@functools.lru_cache(maxsize=None)
def floor(name, primal, levels=2, group=8):
    P, Ke = case(name)
    dec, B = oracle(name, primal, True, levels, group)
    E = np.random.default_rng(1).standard_normal(Ke.shape)
    B2 = bddc.BDDC(dec, P.mesh.elem_nodes, Ke * (1.0 + 2.2e-16 * E), levels=levels, coarse_group=group,
                   nonsymmetric=True)
    r = np.random.default_rng(3).standard_normal(P.n_dofs)[dec.free]
    z = B.apply(r)
    return float(np.linalg.norm(z - B2.apply(r)) / np.linalg.norm(z))


def solver(P, Ke, precision, primal, nonsym, levels=2, group=8):
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                           mbddc.default_options(precision=precision, primal=primal, symmetric_hint=0, levels=levels,
                                                 coarse_group=group, nonsym_coarse=nonsym))
    s.mbddc_set_tangent(Ke)
    s.mbddc_factor()
    return s


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


CASES = [("tiny", 1, 2, 8), ("small_ve", 3, 2, 8), ("tiny_q2", 7, 2, 8), ("ragged", 3, 2, 8),
         ("l3_ragged", 3, 3, 7), ("l3_nh", 3, 3, 8)]


@pytest.mark.parametrize("precision", [mbddc.MBDDC_FP64, mbddc.MBDDC_MIXED])
@pytest.mark.parametrize("name,primal,levels,group", CASES)
def test_nonsymmetric_apply_and_solve(name, primal, levels, group, precision):
    P, Ke = case(name)
    rng = np.random.default_rng(7)
    r = rng.standard_normal((2, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    for nonsym in (1, 0):
        dec, B = oracle(name, primal, bool(nonsym), levels, group)
        s = solver(P, Ke, precision, primal, nonsym, levels, group)
        z = s.mbddc_apply(r)
        err = max(rel(z[k][dec.free], B.apply(r[k][dec.free])) for k in range(2))
        bound = TOL_APPLY[precision]
        if precision == mbddc.MBDDC_FP64:
            bound = max(bound, 100.0 * floor(name, primal, levels, group))
        b = P.rhs[0][dec.free]
        ref = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 1000)
        x, info = s.mbddc_solve(P.rhs[0])
        print(f"{name} levels {levels} prec {precision} nonsym {nonsym}: apply {err:.2e} (bound {bound:.1e}), "
              f"its {info.iterations} (oracle {ref.iterations}), res {info.rel_res_true:.1e}")
        assert err <= bound
        assert np.linalg.norm(b - B.A @ x[dec.free]) <= 1e-8 * np.linalg.norm(b)
        if precision == mbddc.MBDDC_FP64:
            assert abs(info.iterations - ref.iterations) <= 1
        else:
            assert info.iterations <= ref.iterations + 2
        s.close()


@pytest.mark.parametrize("levels", [2, 3])
def test_preconditioner_of_transpose_is_transpose_on_device(levels):
    mesh = W.box_mesh(6, 6, 6, 1)
    part, nsub = W.block_partition(mesh, 3)
    dirichlet = W.clamp_dofs(mesh, 1)
    Ke = skew(W.element_tangents(mesh, W.linear_elastic(1.0, 0.3)))
    KeT = np.ascontiguousarray(np.transpose(Ke, (0, 2, 1)))
    m = mbddc._MeshArrays(mesh.coords, mesh.elem_nodes, mesh.elem_type, part, nsub, mesh.node_tags, dirichlet)
    free = np.setdiff1d(np.arange(3 * mesh.n_nodes), dirichlet)
    mats = []
    for K in (Ke, KeT):
        s = mbddc.Solver(0)
        s.mbddc_setup_symbolic([m], mbddc.default_options(precision=mbddc.MBDDC_FP64, primal=3, symmetric_hint=0,
                                                          levels=levels, coarse_group=2))
        s.mbddc_set_tangent(K)
        s.mbddc_factor()
        cols = []
        for j0 in range(0, len(free), 8):
            E = np.zeros((min(8, len(free) - j0), 3 * mesh.n_nodes))
            for q in range(E.shape[0]):
                E[q, free[j0 + q]] = 1.0
            cols.append(s.mbddc_apply(E)[:, free])
        mats.append(np.concatenate(cols, axis=0).T)   # column j = M e_j
        s.close()
    M, MT = mats
    d = np.abs(MT - M.T).max() / np.abs(M).max()
    print(f"levels {levels}: |M(K^T) - M(K)^T| / |M| = {d:.2e}")
    assert d <= 1e-12
