"""Autotuner: kernel variants per size bucket chosen on the handle's own matrices.

The tuned handle must give the oracle's iteration counts and a solution within 1e-10 of
the default handle's; a table written by one handle and read by another must select the
same kernels (bitwise equal results); and every symmetric-inversion variant, forced by a
table, must meet the same oracle bounds as the default choice (coarse matrix and one
application, paper §3.2 objects).
"""
import json

import numpy as np
import pytest

from oracle import bddc
from paper_2208_06191_amd import mbddc
from tests.conftest import apply_noise_floor, problem

pytestmark = pytest.mark.gpu


def handle(P, primal, precision, table=None, autotune=False, out=None):
    s = mbddc.Solver(0)
    kw = {} if table is None else {"tune_table": str(table)}
    s.mbddc_setup_symbolic([mbddc.mesh_from_problem(P)],
                           mbddc.default_options(precision=precision, primal=primal, symmetric_hint=1,
                                                 keep_coarse_matrix=1, **kw))
    s.mbddc_set_tangent(P.Ke)
    if autotune:
        s.mbddc_autotune(out)
    else:
        s.mbddc_factor()
    return s


@pytest.mark.parametrize("name,primal", [("small_ve", 3), ("large_mixed", 3)])
@pytest.mark.parametrize("precision", [mbddc.MBDDC_FP64, mbddc.MBDDC_MIXED])
def test_autotuned_handle_matches_default(name, primal, precision, tmp_path):
    P = problem(name)
    path = tmp_path / "tune.json"
    t = handle(P, primal, precision, autotune=True, out=path)
    d = handle(P, primal, precision)
    table = t.mbddc_get_tuning()
    on_disk = json.loads(path.read_text())
    assert on_disk["sym_fp64"] == table["sym_fp64"] and on_disk["apply_xchunk"] == table["apply_xchunk"]
    assert all(0 <= v <= 3 for v in table["sym_fp64"] + table["sym_fp32"])
    assert table["apply_xchunk"] in (128, 256, 512, 1024)
    assert all(r in (64, 128, 256) for r in table["apply_rows"]) and on_disk["apply_rows"] == table["apply_rows"]
    assert table["gemm_mfma"] in (0, 1) and on_disk["gemm_mfma"] == table["gemm_mfma"]
    xt, it = t.mbddc_solve(P.rhs)
    xd, idd = d.mbddc_solve(P.rhs)
    print(f"{name} prec={precision}: table {table}, its {it.iterations} vs {idd.iterations}")
    assert it.iterations == idd.iterations and it.rel_res_true <= 1e-8
    assert np.linalg.norm(xt - xd) <= 1e-10 * np.linalg.norm(xd)
    # a second handle reading the table selects the same kernels
    r = handle(P, primal, precision, table=path)
    assert r.mbddc_get_tuning() == table
    xr, _ = r.mbddc_solve(P.rhs)
    assert np.array_equal(xr, xt)


FORCED = {"lds16": [1, 1, 1, 3], "lds32": [2, 1, 1, 3], "blocked": [3, 3, 3, 3], "register": [0, 0, 1, 1]}


@pytest.mark.parametrize("variant", list(FORCED))
@pytest.mark.parametrize("name,primal", [("small_ve", 3), ("large_mixed", 3)])
def test_every_variant_meets_the_oracle_bounds(variant, name, primal, tmp_path):
    P = problem(name)
    path = tmp_path / "forced.json"
    rows = [128, 128, 128, 128] if variant in ("lds16", "blocked") else [256, 256, 256, 256]
    gemm = 1 if variant in ("lds16", "blocked") else 0      # matrix-core and vector GEMMs
    path.write_text(json.dumps({"mbddc_tune": 1, "sym_fp64": FORCED[variant], "sym_fp32": [2, 2, 1, 1],
                                "apply_xchunk": 256, "apply_rows": rows, "gemm_mfma": gemm}))
    s = handle(P, primal, mbddc.MBDDC_FP64, table=path)
    dec = bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                             P.mesh.node_tags, primal=primal)
    B = bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke)
    Kc = s.mbddc_get_coarse_matrix(0, dec.n_coarse)
    err_c = np.linalg.norm(Kc - B.Kc) / np.linalg.norm(B.Kc)
    r = np.random.default_rng(3).standard_normal((2, P.n_dofs))
    r[:, P.dirichlet] = 0.0
    z = s.mbddc_apply(r)
    err = max(np.linalg.norm(z[k][dec.free] - B.apply(r[k][dec.free])) / np.linalg.norm(B.apply(r[k][dec.free]))
              for k in range(2))
    print(f"{name} {variant}: coarse {err_c:.2e} apply {err:.2e}")
    assert err_c <= 1e-12
    assert err <= max(1e-12, 100.0 * apply_noise_floor(name, primal))
