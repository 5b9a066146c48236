"""CPU-side checks of the HIP library: it loads, exports every entry point that
``include/mbddc.h`` declares, and its host symbolic setup (interior/interface
split, vertex/edge/face globs, primal constraints; paper §3.2) is integer-exact
against the oracle's decomposition. No kernel runs here."""
import os
import re

import numpy as np
import pytest

from oracle import bddc
from paper_2208_06191_amd import mbddc
from paper_2208_06191_amd import workloads as W
from tests.conftest import problem

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mbddc.h")


def declared_entry_points():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(mbddc_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = mbddc.lib()
    names = declared_entry_points()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
        assert n in mbddc._SIGNATURES, f"binding lacks {n}"
    assert set(mbddc._SIGNATURES) == set(names)
    assert L.mbddc_strerror(mbddc.MBDDC_ERR_SINGULAR) == b"singular local or coarse problem"


def test_default_options():
    o = mbddc.default_options()
    assert (o.primal, o.levels, o.precision, o.restart, o.rtol, o.max_it) == (3, 2, 1, 30, 1e-8, 1000)
    assert (o.coarse_group, o.coarse_primal) == (8, 7)
    assert o.graph_apply == 1


def _compare_plan(P, primal):
    dec = bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                             P.mesh.node_tags, primal=primal)
    sz, node_glob, kind, cg, cc, sc = mbddc.mbddc_inspect_symbolic(mbddc.mesh_from_problem(P), primal)
    assert (sz.n_vertices, sz.n_edges, sz.n_faces) == dec.glob_counts()
    assert sz.n_coarse == dec.n_coarse
    assert sz.n_free == len(dec.free)
    np.testing.assert_array_equal(node_glob, dec.node_glob)
    np.testing.assert_array_equal(kind, [g[0] for g in dec.globs])
    np.testing.assert_array_equal(cg, [g for g, _ in dec.coarse])
    np.testing.assert_array_equal(cc, [c for _, c in dec.coarse])
    for s, sd in enumerate(dec.subdomains):
        assert tuple(sc[s]) == (sd.n_interior, len(sd.dofs) - sd.n_interior, len(sd.coarse))
    return sz


@pytest.mark.parametrize("name,primal", [("small", 1), ("small_ve", 3), ("small_ve", 7), ("small_ve", 6),
                                         ("tiny_q2", 7), ("ragged", 3), ("tiny", 1)])
def test_host_plan_equals_oracle(name, primal):
    _compare_plan(problem(name), primal)


def test_host_plan_equals_oracle_paper_scale_box():
    mesh = W.box_mesh(32, 32, 32, 1)
    part, nsub = W.block_partition(mesh, 4)
    P = W.Problem("box32", mesh, part, nsub, W.clamp_dofs(mesh), np.zeros((1, 1)), np.zeros((1, 1)), 3)
    sz = _compare_plan(P, 3)
    assert sz.n_coarse == 7140 and sz.n_sub == 512


def test_host_plan_rejects_bad_input():
    P = problem("tiny")
    m = mbddc.mesh_from_problem(P)
    bad = m.elem_part.copy()
    bad[0] = P.n_sub          # out of range
    m2 = mbddc._MeshArrays(P.mesh.coords, P.mesh.elem_nodes, P.mesh.elem_type, bad, P.n_sub, P.mesh.node_tags,
                           P.dirichlet)
    with pytest.raises(mbddc.MbddcError) as e:
        mbddc.mbddc_inspect_symbolic(m2, 1)
    assert e.value.status == mbddc.MBDDC_ERR_ARG
    with pytest.raises(mbddc.MbddcError):
        mbddc.mbddc_inspect_symbolic(m, 8)   # unknown primal bit


def test_footprint_estimate_is_host_only_and_grows_with_size():
    """The admission estimate needs no device and scales with the problem."""
    from paper_2208_06191_amd import workloads as W
    sizes = []
    for n in (4, 8, 12):
        mesh = W.box_mesh(n, n, n, 1)
        part, nsub = W.block_partition(mesh, 4)
        m = mbddc._MeshArrays(mesh.coords, mesh.elem_nodes, mesh.elem_type, part, nsub, mesh.node_tags,
                              W.clamp_dofs(mesh, 1))
        sizes.append(mbddc.mbddc_estimate_footprint([m], mbddc.default_options()))
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    # a three-level handle carries no dense level-1 coarse inverse (512 subdomains, V+E+F)
    mesh = W.box_mesh(24, 24, 24, 1)
    part, nsub = W.block_partition(mesh, 3, cluster=2)
    m = mbddc._MeshArrays(mesh.coords, mesh.elem_nodes, mesh.elem_type, part, nsub, mesh.node_tags,
                          W.clamp_dofs(mesh, 1))
    two = mbddc.mbddc_estimate_footprint([m], mbddc.default_options(primal=7))
    three = mbddc.mbddc_estimate_footprint([m], mbddc.default_options(primal=7, levels=3))
    assert three < two
    with pytest.raises(mbddc.MbddcError):
        mbddc.mbddc_estimate_footprint([m], mbddc.default_options(levels=5))


def test_tuning_table_is_read_and_checked(tmp_path):
    """Tables are read during setup (host only): valid ones are accepted, malformed,
    missing or out-of-range ones rejected with MBDDC_ERR_ARG."""
    from paper_2208_06191_amd import workloads as W
    m = mbddc.mesh_from_problem(W.linear_box(4, 2, 1, nrhs=1, primal=3, name="t"))
    good = tmp_path / "good.json"
    good.write_text('{"mbddc_tune": 1, "sym_fp64": [0, 1, 3, 3], "sym_fp32": [2, 2, 1, 1], "apply_xchunk": 512}\n')
    base = mbddc.mbddc_estimate_footprint([m], mbddc.default_options(symmetric_hint=1))
    assert mbddc.mbddc_estimate_footprint([m], mbddc.default_options(symmetric_hint=1, tune_table=str(good))) > 0
    assert base > 0
    rows = tmp_path / "rows_ok.json"   # every row block size the apply has (64, 128, 256; 0 = by size)
    rows.write_text('{"mbddc_tune": 1, "sym_fp64": [0, 1, 3, 3], "sym_fp32": [2, 2, 1, 1], "apply_xchunk": 256, '
                    '"apply_rows": [64, 128, 256, 0], "apply_rows2": [256, 64, 0, 128], "apply_groups": 0, '
                    '"gemm_mfma": 1}\n')
    assert mbddc.mbddc_estimate_footprint([m], mbddc.default_options(symmetric_hint=1, tune_table=str(rows))) > 0
    bad = {"garbage.json": "not a table",
           "range.json": '{"mbddc_tune": 1, "sym_fp64": [0, 1, 7, 3], "sym_fp32": [2, 2, 1, 1], "apply_xchunk": 512}',
           "chunk.json": '{"mbddc_tune": 1, "sym_fp64": [0, 1, 3, 3], "sym_fp32": [2, 2, 1, 1], "apply_xchunk": 100}',
           "short.json": '{"mbddc_tune": 1, "sym_fp64": [0, 1], "apply_xchunk": 512}',
           "rows.json": '{"mbddc_tune": 1, "sym_fp64": [0, 1, 3, 3], "sym_fp32": [2, 2, 1, 1], "apply_xchunk": 512, '
                        '"apply_rows": [128, 256, 96, 0]}',
           "gemm.json": '{"mbddc_tune": 1, "sym_fp64": [0, 1, 3, 3], "sym_fp32": [2, 2, 1, 1], "apply_xchunk": 512, '
                        '"gemm_mfma": 2}'}
    for name, text in bad.items():
        f = tmp_path / name
        f.write_text(text)
        with pytest.raises(mbddc.MbddcError) as e:
            mbddc.mbddc_estimate_footprint([m], mbddc.default_options(symmetric_hint=1, tune_table=str(f)))
        assert e.value.status == mbddc.MBDDC_ERR_ARG, name
    with pytest.raises(mbddc.MbddcError) as e:
        mbddc.mbddc_estimate_footprint([m], mbddc.default_options(tune_table=str(tmp_path / "missing.json")))
    assert e.value.status == mbddc.MBDDC_ERR_ARG


def test_nnsp_option_is_checked_on_the_host():
    """Near-null-space primals need node coordinates and two levels; the flag is 0 or 1."""
    P = problem("small_ve")
    m = mbddc.mesh_from_problem(P)
    bare = mbddc._MeshArrays(None, P.mesh.elem_nodes, P.mesh.elem_type, P.elem_part, P.n_sub, P.mesh.node_tags,
                             P.dirichlet)
    avg = mbddc.mbddc_estimate_footprint([m], mbddc.default_options(primal=7))
    rows = mbddc.mbddc_estimate_footprint([m], mbddc.default_options(primal=7, nnsp=1))
    assert rows > avg          # more coarse DOFs per edge and face
    for mesh, kw, status in ((bare, dict(nnsp=1), mbddc.MBDDC_ERR_ARG),
                             (m, dict(nnsp=2), mbddc.MBDDC_ERR_ARG),
                             (m, dict(nnsp=1, levels=3), mbddc.MBDDC_ERR_UNSUPPORTED)):
        with pytest.raises(mbddc.MbddcError) as e:
            mbddc.mbddc_estimate_footprint([mesh], mbddc.default_options(primal=7, **kw))
        assert e.value.status == status


def test_deluxe_option_is_checked_on_the_host():
    """Deluxe scaling: symmetric path with FP64 local factors; the flag is 0 or 1."""
    m = mbddc.mesh_from_problem(problem("small_ve"))
    base = mbddc.mbddc_estimate_footprint([m], mbddc.default_options(primal=3, symmetric_hint=1))
    dlx = mbddc.mbddc_estimate_footprint([m], mbddc.default_options(primal=3, symmetric_hint=1,
                                                                    scaling=mbddc.MBDDC_SCALING_DELUXE))
    assert dlx > base          # glob blocks and the scratch of the weighted operators
    for kw, status in ((dict(scaling=2, symmetric_hint=1), mbddc.MBDDC_ERR_ARG),
                       (dict(scaling=1, symmetric_hint=0), mbddc.MBDDC_ERR_UNSUPPORTED),
                       (dict(scaling=1, symmetric_hint=1, precision=mbddc.MBDDC_MIXED_F32FACT),
                        mbddc.MBDDC_ERR_UNSUPPORTED)):
        with pytest.raises(mbddc.MbddcError) as e:
            mbddc.mbddc_estimate_footprint([m], mbddc.default_options(primal=3, **kw))
        assert e.value.status == status
