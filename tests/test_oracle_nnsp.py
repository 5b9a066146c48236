"""Pins for the oracle's near-null-space primal constraints (paper §4: the rigid motions handed to
BDDC as extra primal degrees of freedom), against facts fixed by the geometry and the mathematics.

* row counts per glob equal closed forms on box partitions: a vertex keeps its 3 component rows,
  a straight edge 5 rigid-motion rows (the rotation about its own line vanishes on it), a planar
  face 6, so the coarse size is 3 V + 5 E + 6 F with the box's closed-form glob counts;
* every glob's rows are orthonormal, and every rigid motion (sampled by an independent routine)
  restricted to the glob lies in their span, on the curved shell too;
* lambda_min(M^-1 A) >= 1 and M = M^T: the BDDC lower bound holds for any primal set;
* on a slender clamped beam cut across its length (edge and face primals), the rigid-motion rows
  take fewer GMRES iterations than averages (they carry the bending and twisting of each
  cross-section, which averages miss);
* three levels with them are refused.
"""
import numpy as np
import pytest

from paper_2208_06191_amd import workloads as W
from oracle import bddc, fem, gmres
from tests.conftest import problem
from tests.test_oracle import closed_form_counts, dense_precond


def decomp(P, primal, nnsp=True):
    return bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                              P.mesh.node_tags, primal=primal, coords=P.mesh.coords, nnsp=nnsp)


@pytest.mark.parametrize("S,block", [(2, 4), (2, 3), (3, 3)])
def test_row_counts_closed_form(S, block):
    P = W.linear_box(S * block, block, 1, nrhs=1, primal=7)
    V, E, F = closed_form_counts(S)
    for mask, n in ((7, 3 * V + 5 * E + 6 * F), (6, 5 * E + 6 * F), (4, 6 * F), (1, 3 * V)):
        dec = decomp(P, mask)
        assert dec.glob_counts() == (V, E, F)
        assert dec.n_coarse == n, (mask, dec.n_coarse, n)
    dec = decomp(P, 7)
    for gi, (dd, B) in dec.glob_rows.items():
        assert B.shape[0] == {bddc.EDGE: 5, bddc.FACE: 6}[dec.globs[gi][0]]


@pytest.mark.parametrize("name", ["small", "vent"])
def test_rows_orthonormal_and_span_the_rigid_motions(name):
    P = problem(name)
    dec = decomp(P, 7)
    R = fem.rigid_body_modes(P.mesh.coords)
    assert dec.glob_rows
    for gi, (dd, B) in dec.glob_rows.items():
        assert 3 <= B.shape[0] <= 6
        assert np.abs(B @ B.T - np.eye(B.shape[0])).max() < 1e-12
        Rg = R[dd]
        resid = Rg - B.T @ (B @ Rg)
        assert np.linalg.norm(resid) <= 1e-10 * np.linalg.norm(Rg)
    # the constraint rows of a subdomain are those of its globs, placed on its local DOFs
    for sd, loc in zip(dec.subdomains, dec.local_dofs):
        pos = {int(d): k for k, d in enumerate(loc)}
        for row, cid in zip(sd.C, sd.coarse):
            gi, k = dec.coarse[cid]
            if gi in dec.glob_rows:
                dd, B = dec.glob_rows[gi]
                ref = np.zeros(len(loc))
                ref[[pos[int(d)] for d in dd]] = B[k]
                assert np.array_equal(row, ref)


@pytest.mark.parametrize("name,primal", [("tiny", 3), ("tiny", 4), ("tiny_q2", 7)])
def test_lower_bound_and_symmetry(name, primal):
    P = problem(name)
    dec = decomp(P, primal)
    assert dec.glob_rows
    B = bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke)
    n = len(dec.free)
    M = dense_precond(B, n)
    assert np.abs(M - M.T).max() < 1e-10 * np.abs(M).max()
    ev = np.linalg.eigvals(M @ B.A.toarray())
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() > 1 - 1e-10


def beam():
    """10 x 1 x 1 beam, 40 x 4 x 4 Q1 elements, x = 0 clamped, cut into 10 slabs along x: each cut
    has a face (the 3 x 3 inner nodes), 4 edges (3 nodes along each side) and 4 corner vertices."""
    mesh = W.box_mesh(40, 4, 4, 1, lengths=(10.0, 1.0, 1.0))
    part, nsub = W.block_partition(mesh, (4, 4, 4))
    dirichlet = W.clamp_dofs(mesh, 1)
    Ke = W.element_tangents(mesh, W.linear_elastic(1.0, 0.3))
    rhs = W._loads(mesh, dirichlet, 1, 1)
    return W.Problem("beam", mesh, part, nsub, dirichlet, Ke, rhs, 6, {})


def test_rigid_motion_rows_need_fewer_iterations_on_a_beam():
    P = beam()
    its = []
    for nnsp in (False, True):
        dec = decomp(P, bddc.EDGE | bddc.FACE, nnsp)
        assert dec.glob_counts() == (36, 36, 9)
        B = bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke)
        b = P.rhs[0][dec.free]
        res = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 1000)
        assert res.converged
        its.append(res.iterations)
    assert its[1] < its[0], its


def test_three_levels_refused():
    P = problem("tiny")
    with pytest.raises(NotImplementedError):
        bddc.BDDC(decomp(P, 3), P.mesh.elem_nodes, P.Ke, levels=3)
