"""GPU parity for local matrices beyond the one-workgroup kernels.

Subdomains of 1k-2.2k DOFs (interior blocks K_II and interface blocks S + rho C^T C
of more than 304 rows) take the batched blocked sweep of the symmetric path, and
their apply stages the input vector in LDS a chunk of 1024 columns at a time. The
checkpoints and bounds are those of the small cases (paper §3.2 objects): coarse
matrix, one preconditioner application, GMRES iterations and solution against the
FP64 oracle, on a Q1 box, a box whose subdomains straddle the one-workgroup limit
(both kernels in one factorisation) and the Q2 ventricle-like shell. The FP32 local
factorisation (MBDDC_MIXED_F32FACT) sweeps the same blocks in FP32 on the matrix cores.
"""
import functools
import json

import numpy as np
import pytest

from oracle import bddc, gmres
from paper_2208_06191_amd import mbddc
from tests.conftest import apply_noise_floor, problem

pytestmark = pytest.mark.gpu

TOL_APPLY = {mbddc.MBDDC_FP64: 1e-12, mbddc.MBDDC_MIXED: 1e-5}
TOL_COARSE = 1e-12
PRECS = [mbddc.MBDDC_FP64, mbddc.MBDDC_MIXED]
# vent_parts6k: the Q2 shell at 1/16 of the full mesh (63.5k DOFs) whose RCB parts have the
# full-size shape (2k-5.7k DOFs, interiors up to 4.4k)
CASES = [("large_q1", 3), ("large_mixed", 3), ("vent_large", 7), ("vent_parts6k", 7)]
ONE_WG_MAX = 304          # largest matrix of the register-resident sweep


@functools.lru_cache(maxsize=None)
def oracle_of(name, primal, levels=2, group=8):
    P = problem(name)
    dec = bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                             P.mesh.node_tags, primal=primal)
    return dec, bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke, levels=levels, coarse_group=group, level2_primal=7)


def solver_for(P, precision, primal, sym=1, **kw):
    s = mbddc.Solver(0)
    o = mbddc.default_options(precision=precision, primal=primal, keep_coarse_matrix=1, symmetric_hint=sym, **kw)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)], o)
    s.mbddc_set_tangent(P.Ke)
    try:
        s.mbddc_factor()
    except mbddc.MbddcError as e:
        raise AssertionError(f"factor failed: {e}, subdomain {s.last_bad_subdomain()}") from e
    return s


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name,primal", CASES)
def test_local_blocks_exceed_one_workgroup(name, primal):
    dec, _ = oracle_of(name, primal)
    nI = np.array([s.n_interior for s in dec.subdomains])
    nG = np.array([len(s.dofs) for s in dec.subdomains]) - nI
    assert nI.max() > ONE_WG_MAX and nG.max() > ONE_WG_MAX
    if name == "large_q1":
        assert nI.max() > 1024            # more than one staged chunk in the apply
    if name == "vent_parts6k":
        assert nI.max() > 4000 and (nI + nG).max() > 5000
    if name == "large_mixed":             # both sweeps in one factorisation
        assert nI.min() <= ONE_WG_MAX and nG.min() <= ONE_WG_MAX


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("name,primal", CASES)
def test_coarse_matrix_and_apply(name, primal, precision):
    P = problem(name)
    dec, B = oracle_of(name, primal)
    s = solver_for(P, precision, primal)
    err_c = rel(s.mbddc_get_coarse_matrix(0, dec.n_coarse), B.Kc)
    r = np.random.default_rng(7).standard_normal((3, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    z = s.mbddc_apply(r)
    errs = [rel(z[k][dec.free], B.apply(r[k][dec.free])) for k in range(3)]
    clamped = np.setdiff1d(np.arange(P.n_dofs), dec.free)
    print(f"{name} prec={precision}: coarse {err_c:.2e} apply {max(errs):.2e}")
    assert err_c <= TOL_COARSE
    assert max(errs) <= max(TOL_APPLY[precision], 100.0 * apply_noise_floor(name, primal))
    assert np.abs(z[:, clamped]).max() == 0.0


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("name,primal", CASES)
def test_solve_matches_oracle(name, primal, precision):
    P = problem(name)
    dec, B = oracle_of(name, primal)
    s = solver_for(P, precision, primal)
    x, info = s.mbddc_solve(P.rhs)
    for k in range(P.rhs.shape[0]):
        b = P.rhs[k][dec.free]
        ref = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 1000)
        xr = x[k][dec.free]
        assert np.linalg.norm(b - B.A @ xr) / np.linalg.norm(b) <= 1e-8
        _, i1 = s.mbddc_solve(P.rhs[k])
        print(f"{name} prec={precision} rhs {k}: its {i1.iterations} (oracle {ref.iterations})")
        if precision == mbddc.MBDDC_FP64:
            assert abs(i1.iterations - ref.iterations) <= 1
        else:
            assert i1.iterations <= ref.iterations + 2
        assert i1.rel_res_true <= 1e-8


@pytest.mark.parametrize("precision", PRECS)
def test_three_levels_with_large_locals(precision):
    P = problem("large_q1")
    dec, B = oracle_of("large_q1", 3, levels=3, group=4)
    s = solver_for(P, precision, 3, levels=3, coarse_group=4, coarse_primal=7)
    r = np.random.default_rng(9).standard_normal((2, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    z = s.mbddc_apply(r)
    err = max(rel(z[k][dec.free], B.apply(r[k][dec.free])) for k in range(2))
    bound = max(TOL_APPLY[precision], 100.0 * apply_noise_floor("large_q1", 3, levels=3, group=4))
    print(f"three levels prec={precision}: apply {err:.2e} (bound {bound:.1e})")
    assert err <= bound
    x, info = s.mbddc_solve(P.rhs[0])
    assert info.rel_res_true <= 1e-8


# general path (symmetric_hint = 0): blocks above 512 rows go to the multi-workgroup pivoted
# inverse, the interface matrices augmented by rho C^T C around it
GENERAL = [("large_q1", 3), ("vent_parts6k", 7)]


@pytest.mark.parametrize("precision", PRECS)
@pytest.mark.parametrize("name,primal", GENERAL)
def test_general_path_large_locals(name, primal, precision):
    P = problem(name)
    dec, B = oracle_of(name, primal)
    nI = np.array([s.n_interior for s in dec.subdomains])
    m = np.array([len(s.dofs) - s.n_interior + s.C.shape[0] for s in dec.subdomains])
    assert nI.max() > 512 and m.max() > 512
    s = solver_for(P, precision, primal, sym=0)
    err_c = rel(s.mbddc_get_coarse_matrix(0, dec.n_coarse), B.Kc)
    r = np.random.default_rng(7).standard_normal((2, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    z = s.mbddc_apply(r)
    err = max(rel(z[k][dec.free], B.apply(r[k][dec.free])) for k in range(2))
    bound = max(TOL_APPLY[precision], 100.0 * apply_noise_floor(name, primal))
    b = P.rhs[0][dec.free]
    ref = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 1000)
    x, info = s.mbddc_solve(P.rhs[0])
    print(f"general {name} prec={precision}: coarse {err_c:.2e} apply {err:.2e} (bound {bound:.1e}) "
          f"its {info.iterations} (oracle {ref.iterations})")
    assert err_c <= 1e-11
    assert err <= bound
    assert np.linalg.norm(b - B.A @ x[dec.free]) <= 1e-8 * np.linalg.norm(b)
    if precision == mbddc.MBDDC_FP64:
        assert abs(info.iterations - ref.iterations) <= 1
    else:
        assert info.iterations <= ref.iterations + 2
    s.close()


def test_general_path_large_nonsymmetric():
    """Skew-perturbed tangents (5 % of the largest entry) on the large Q1 box against the
    oracle's non-symmetric formulation (left coarse basis)."""
    P = problem("large_q1")
    S = np.random.default_rng(3).standard_normal(P.Ke.shape)
    Ke = P.Ke + 0.05 * np.abs(P.Ke).max() * (S - np.transpose(S, (0, 2, 1)))
    dec = bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                             P.mesh.node_tags, primal=3)
    B = bddc.BDDC(dec, P.mesh.elem_nodes, Ke, nonsymmetric=True)
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                           mbddc.default_options(precision=mbddc.MBDDC_FP64, primal=3, symmetric_hint=0))
    s.mbddc_set_tangent(Ke)
    s.mbddc_factor()
    r = np.random.default_rng(7).standard_normal((2, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    z = s.mbddc_apply(r)
    err = max(rel(z[k][dec.free], B.apply(r[k][dec.free])) for k in range(2))
    b = P.rhs[0][dec.free]
    ref = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 1000)
    x, info = s.mbddc_solve(P.rhs[0])
    bound = max(1e-12, 100.0 * apply_noise_floor("large_q1", 3))
    print(f"general nonsymmetric large_q1: apply {err:.2e} (bound {bound:.1e}) its {info.iterations} "
          f"(oracle {ref.iterations})")
    assert err <= bound
    assert abs(info.iterations - ref.iterations) <= 1
    assert np.linalg.norm(b - B.A @ x[dec.free]) <= 1e-8 * np.linalg.norm(b)
    s.close()


def test_general_path_rejects_large_locals_in_fp32_factor():
    P = problem("large_q1")
    s = mbddc.Solver(0)
    with pytest.raises(mbddc.MbddcError) as e:
        s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                               mbddc.default_options(primal=3, symmetric_hint=0, precision=mbddc.MBDDC_MIXED_F32FACT))
    assert e.value.status == mbddc.MBDDC_ERR_UNSUPPORTED


def test_floating_large_subdomains_without_primals_are_singular():
    P = problem("large_q1")
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)], mbddc.default_options(primal=0, symmetric_hint=1,
                                                                              precision=mbddc.MBDDC_FP64))
    s.mbddc_set_tangent(P.Ke)
    with pytest.raises(mbddc.MbddcError) as e:
        s.mbddc_factor()
    assert e.value.status == mbddc.MBDDC_ERR_SINGULAR
    bad = s.last_bad_subdomain()
    elems = np.nonzero(P.elem_part == bad)[0]
    assert not np.any(P.mesh.node_tags[P.mesh.elem_nodes[elems]] & 1)   # a floating subdomain


# ------------------------------------------------------------------- FP32 local factorisations
EPS32_OVER_EPS64 = 1.1920929e-07 / 2.220446049250313e-16


@pytest.mark.parametrize("gemm", [1, 0])
@pytest.mark.parametrize("name,primal", CASES)
def test_fp32_blocked_sweep_on_the_matrix_cores(name, primal, gemm, tmp_path):
    """MBDDC_MIXED_F32FACT with every symmetric inversion forced onto the blocked sweep in FP32
    (panel products and trailing update on the FP32 matrix cores, FP32 accumulation) and the
    condensation GEMMs on the matrix cores (gemm 1) or the vector units (gemm 0). One application
    is held to the FP32 analogue of the FP64 bound: 100 x the oracle's change under a relative
    FP32-epsilon perturbation of K_e (first order in the epsilon, so the FP64 floor scaled by
    eps32 / eps64), at least 1e-2; the local coarse matrices, formed in FP32 as T^-1 - rho I, to the
    FP64 coarse bound scaled the same way (1e-12 eps32 / eps64, about 5e-4: the cancellation against
    rho costs no more than FP32 rounding); the solve reaches the FP64 true residual within the
    mode's allowance of oracle + 6 iterations."""
    P = problem(name)
    dec, B = oracle_of(name, primal)
    path = tmp_path / "fp32.json"
    path.write_text(json.dumps({"mbddc_tune": 1, "sym_fp64": [0, 0, 3, 3], "sym_fp32": [3, 3, 3, 3],
                                "apply_xchunk": 256, "apply_rows": [128, 128, 128, 128], "gemm_mfma": gemm}))
    s = solver_for(P, mbddc.MBDDC_MIXED_F32FACT, primal, tune_table=str(path))
    assert s.mbddc_get_tuning()["sym_fp32"] == [3, 3, 3, 3]
    err_c = rel(s.mbddc_get_coarse_matrix(0, dec.n_coarse), B.Kc)
    assert err_c <= TOL_COARSE * EPS32_OVER_EPS64, err_c
    r = np.random.default_rng(7).standard_normal((2, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    z = s.mbddc_apply(r)
    err = max(rel(z[k][dec.free], B.apply(r[k][dec.free])) for k in range(2))
    bound = max(1e-2, 100.0 * EPS32_OVER_EPS64 * apply_noise_floor(name, primal))
    b = P.rhs[0][dec.free]
    ref = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 1000)
    x, info = s.mbddc_solve(P.rhs[0])
    print(f"{name} gemm {gemm}: FP32 blocked sweep coarse {err_c:.2e}, apply {err:.2e} (bound {bound:.1e}), "
          f"its {info.iterations} (oracle {ref.iterations})")
    assert err <= bound
    assert info.rel_res_true <= 1e-8
    assert np.linalg.norm(b - B.A @ x[dec.free]) <= 1e-8 * np.linalg.norm(b)
    assert info.iterations <= ref.iterations + 6
    s.close()


def test_fp32_default_table_takes_the_blocked_sweep_for_large_blocks():
    """With the default table, FP32 blocks beyond 598 rows take the blocked sweep and the shell
    with full-size parts (interiors up to 4.4k rows, beyond every one-workgroup FP32 kernel)
    factorises and solves."""
    P = problem("vent_parts6k")
    dec, B = oracle_of("vent_parts6k", 7)
    s = solver_for(P, mbddc.MBDDC_MIXED_F32FACT, 7)
    assert s.mbddc_get_tuning()["sym_fp32"][3] == 3
    x, info = s.mbddc_solve(P.rhs[0])
    b = P.rhs[0][dec.free]
    assert info.rel_res_true <= 1e-8
    assert np.linalg.norm(b - B.A @ x[dec.free]) <= 1e-8 * np.linalg.norm(b)
    s.close()
