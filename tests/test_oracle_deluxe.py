"""Pins for the oracle's deluxe scaling (paper §3.2: the more robust alternative to the counting
function), against facts fixed by its definition and by BDDC theory.

* partition of unity: over the subdomains sharing a glob the weight blocks add up to the
  identity;
* the extension is the S-weighted mean: for local values w_j on a glob, sum_j D_g^(j) w_j is the
  v minimising sum_j |S_g^(j)^(1/2) (w_j - v)|^2, computed here by a least-squares solve of the
  stacked square-root system (no use of the weight formula; fails for D transposed);
* with every interface DOF primal BDDC is exact whatever the scaling, and with a
  partition of unity it stays so;
* lambda_min(M^-1 A) >= 1 and M = M^T;
* on a checkerboard of stiff (E = 1e3) and soft (E = 1) subdomains, deluxe scaling takes less
  than half the GMRES iterations of the counting function;
* the non-symmetric formulation with deluxe scaling is refused.
"""
import numpy as np
import pytest

from paper_2208_06191_amd import workloads as W
from oracle import bddc, gmres
from tests.conftest import problem
from tests.test_oracle import dense_precond


def decomp(P, primal=None, **kw):
    return bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                              P.mesh.node_tags, primal=P.primal if primal is None else primal, **kw)


def glob_members(dec):
    members = {}
    for i, sp_ in enumerate(dec.subdomains):
        for g in np.unique(sp_.iglob):
            members.setdefault(int(g), []).append((i, np.nonzero(sp_.iglob == g)[0]))
    return members


def schur(K, nI):
    return K[nI:, nI:] - K[nI:, :nI] @ np.linalg.solve(K[:nI, :nI], K[:nI, nI:])


@pytest.mark.parametrize("name", ["small_ve", "tiny_q2", "vent"])
def test_partition_of_unity_and_weighted_mean(name):
    P = problem(name)
    dec = decomp(P)
    B = bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke, scaling="deluxe")
    Ks = bddc.local_matrices(dec, P.mesh.elem_nodes, P.Ke)
    S = [schur(K, sp_.n_interior) for K, sp_ in zip(Ks, dec.subdomains)]
    rng = np.random.default_rng(5)
    members = glob_members(dec)
    shared = [g for g, lst in members.items() if len(lst) >= 2]
    assert shared
    for g, lst in members.items():
        n = len(lst[0][1])
        total = sum(B.L1.D[i][np.ix_(p, p)] for i, p in lst)
        assert np.abs(total - np.eye(n)).max() < 1e-10
    for g in shared[:40]:
        lst = members[g]
        ws = [rng.standard_normal(len(p)) for _, p in lst]
        ext = sum(B.L1.D[i][np.ix_(p, p)] @ w for (i, p), w in zip(lst, ws))
        rows, rhs = [], []
        for (i, p), w in zip(lst, ws):
            ev, V = np.linalg.eigh(S[i][np.ix_(p, p)])
            assert ev.min() > 0
            R = (V * np.sqrt(ev)) @ V.T                      # S_g^(i)^(1/2)
            rows.append(R)
            rhs.append(R @ w)
        v = np.linalg.lstsq(np.vstack(rows), np.concatenate(rhs), rcond=None)[0]
        assert np.linalg.norm(ext - v) <= 1e-8 * np.linalg.norm(v)


def test_all_interface_primal_is_exact():
    P = problem("tiny_q2")
    dec = decomp(P, all_interface_vertices=True)
    B = bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke, scaling="deluxe")
    x = np.random.default_rng(2).standard_normal(len(dec.free))
    assert np.linalg.norm(B.apply(B.A @ x) - x) < 1e-9 * np.linalg.norm(x)


@pytest.mark.parametrize("name,primal", [("tiny", 1), ("tiny", 3), ("tiny_q2", 7)])
def test_lower_bound_and_symmetry(name, primal):
    P = problem(name)
    dec = decomp(P, primal)
    B = bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke, scaling="deluxe")
    M = dense_precond(B, len(dec.free))
    assert np.abs(M - M.T).max() < 1e-10 * np.abs(M).max()
    ev = np.linalg.eigvals(M @ B.A.toarray())
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() > 1 - 1e-10


def checkerboard(n=12, block=3, jump=1e3):
    """Unit cube, n^3 Q1 elements, x = 0 clamped, (n / block)^3 subdomains with E = jump on the
    odd cells of the subdomain checkerboard and E = 1 elsewhere (linear elasticity, nu = 0.3)."""
    mesh = W.box_mesh(n, n, n, 1)
    part, nsub = W.block_partition(mesh, block)
    s = n // block
    i, j, k = part % s, (part // s) % s, part // (s * s)
    E = np.where((i + j + k) % 2 == 1, jump, 1.0)
    Ke = W.element_tangents(mesh, W.linear_elastic(1.0, 0.3)) * E[:, None, None]
    dirichlet = W.clamp_dofs(mesh, 1)
    rhs = W._loads(mesh, dirichlet, 1, 1)
    return W.Problem("checkerboard", mesh, part, nsub, dirichlet, Ke, rhs, 3, {"jump": jump})


def test_deluxe_needs_fewer_iterations_across_coefficient_jumps():
    P = checkerboard()
    dec = decomp(P)
    its = {}
    for scaling in ("counting", "deluxe"):
        B = bddc.BDDC(dec, P.mesh.elem_nodes, P.Ke, scaling=scaling)
        b = P.rhs[0][dec.free]
        res = gmres.gmres(lambda v: B.A @ v, B.apply, b, 1e-8, 30, 2000)
        assert res.converged
        its[scaling] = res.iterations
    assert 2 * its["deluxe"] < its["counting"], its     # measured: 9 against 100


def test_nonsymmetric_deluxe_refused():
    P = problem("tiny")
    with pytest.raises(NotImplementedError):
        bddc.BDDC(decomp(P), P.mesh.elem_nodes, P.Ke, scaling="deluxe", nonsymmetric=True)
