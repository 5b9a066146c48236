"""Pins for the oracle's three-level construction with several level-2 subdomains
(paper §3.2 last paragraph: the coarse problem is itself solved by one BDDC application;
§7: level-2 subdomains are groups of 8 fine subdomains, primal V+E+F).

Facts fixed by the mathematics, independent of the oracle's code:

* on a box whose fine subdomains are numbered in 2x2x2 clusters, the level-2 subdomains
  are boxes too, so the level-2 globs are the corners / edges / face patches of an
  S x S x S box partition: the closed-form counts of the fine level hold with S level-2
  subdomains per axis, and a brute-force geometric classification of the fine globs
  (by which level-2 planes their nodes sit on) gives the same globs;
* with fine vertex primals only, every level-2 glob is a single fine vertex (edges and
  patches then hold one item each), and when every level-2 interface item is primal the
  level-2 BDDC is an exact solve of the coarse problem, so three levels equal two;
* BDDC's lower bound lambda_min(M^-1 A) >= 1 holds at level 2 on S_PiPi; therefore
  M_3^-1 - M_2^-1 = L^T diag(0, R_D^T Phi (M_c^-1 - S_PiPi^-1) Phi^T R_D) L is positive
  semidefinite (L the block elimination of the interior), so lambda_min(M_3^-1 A) >= 1 and
  M_3 is symmetric when A is.
A wrong level-2 weight, interior/interface split, constraint row or assembly position
breaks the partition of unity or the Galerkin coarse operator and fails one of these.
"""
import functools

import numpy as np
import pytest

from paper_2208_06191_amd import workloads as W
from oracle import bddc
from tests.test_oracle import closed_form_counts


@functools.lru_cache(maxsize=None)
def clustered(n, block, material="linear", ny=None, nz=None, cluster=2):
    """Q1 box, x = 0 clamped, subdomains of block^3 elements numbered in 2x2x2 clusters."""
    mesh = W.box_mesh(n, ny or n, nz or n, 1)
    part, nsub = W.block_partition(mesh, block, cluster)
    dirichlet = W.clamp_dofs(mesh, 1)
    if material == "linear":
        Ke = W.element_tangents(mesh, W.linear_elastic(1.0, 0.3))
    else:
        u = W.isochoric_field(mesh.coords, 4, 0.02)
        Ke = W.element_tangents(mesh, W.neo_hookean(1.0, 50.0), u)
    return mesh, part, nsub, dirichlet, Ke


def build(case, primal, levels=3, group=8, primal2=7):
    mesh, part, nsub, dirichlet, Ke = case
    dec = bddc.Decomposition(mesh.elem_nodes, mesh.n_nodes, part, nsub, dirichlet, mesh.node_tags,
                             primal=primal)
    return dec, bddc.BDDC(dec, mesh.elem_nodes, Ke, levels=levels, coarse_group=group, level2_primal=primal2)


def level2_counts(B):
    k = np.array([g[0] for g in B.L2.globs])
    return int((k == bddc.VERTEX).sum()), int((k == bddc.EDGE).sum()), int((k == bddc.FACE).sum())


@pytest.mark.parametrize("n,block,primal", [(12, 3, 3), (12, 3, 7), (16, 4, 3)])
def test_level2_glob_counts_closed_form(n, block, primal):
    dec, B = build(clustered(n, block), primal)
    V, E, F = closed_form_counts(n // block // 2)
    assert level2_counts(B) == (V, E, F)
    assert B.L2.n_coarse == 3 * (V + E + F)          # level-2 primal V+E+F, three components each


@pytest.mark.slow
def test_level2_glob_counts_closed_form_three_per_axis():
    dec, B = build(clustered(18, 3), 3)
    V, E, F = closed_form_counts(3)
    assert (V, E, F) == (44, 96, 54)
    assert level2_counts(B) == (V, E, F)
    assert B.L2.n_coarse == 3 * (V + E + F)


def test_level2_vertex_only_fine_primals_give_single_item_globs():
    dec, B = build(clustered(12, 3), 1)
    V, E, F = closed_form_counts(2)
    assert level2_counts(B) == (V + E + F, 0, 0)


@pytest.mark.parametrize("n,block,primal", [(12, 3, 3), (12, 3, 7)])
def test_level2_globs_equal_geometric_classification(n, block, primal):
    """Brute force: a fine glob lies on the level-2 interface when one of its nodes sits on an
    internal plane of the level-2 box grid; its level-2 entity is given, per axis, by the plane
    it sits on or the level-2 block it is inside; the kind by how many axes sit on a plane."""
    mesh, part, nsub, dirichlet, Ke = case = clustered(n, block)
    dec, B = build(case, primal)
    Nx = n + 1
    L = 2 * block                                    # nodes per level-2 block edge (Q1)
    items = sorted({gi for gi, _ in dec.coarse})      # level-2 items: fine globs with coarse DOFs
    geo = {}
    for k, gi in enumerate(items):
        keys = set()
        internal = False
        for nd in dec.globs[gi][1]:
            ijk = (nd % Nx, (nd // Nx) % Nx, nd // (Nx * Nx))
            on = [c % L == 0 for c in ijk]
            internal |= any(o and 0 < c < n for o, c in zip(on, ijk))
            keys.add(tuple(("c", c) if o else ("b", c // L) for c, o in zip(ijk, on)))
        assert len(keys) == 1, "a fine glob spans two level-2 entities"
        if internal:
            geo.setdefault(keys.pop(), []).append(k)
    kinds = {3: bddc.VERTEX, 2: bddc.EDGE, 1: bddc.FACE}
    expect = sorted((kinds[sum(c[0] == "c" for c in key)], tuple(v)) for key, v in geo.items())
    got = sorted((g[0], tuple(int(i) for i in g[1])) for g in B.L2.globs)
    assert got == expect


def test_all_level2_interface_items_primal_three_levels_equal_two():
    case = clustered(12, 3, "neo_hookean")
    dec, B3 = build(case, 1, primal2=1)
    assert all(g[0] == bddc.VERTEX and len(g[1]) == 1 for g in B3.L2.globs)
    assert len(B3.L2.spaces) == 8                    # eight level-2 subdomains
    _, B2 = build(case, 1, levels=2)
    r = np.random.default_rng(5).standard_normal(len(dec.free))
    z2, z3 = B2.apply(r), B3.apply(r)
    assert np.linalg.norm(z3 - z2) < 1e-12 * np.linalg.norm(z2)
    # and with edge primals at the fine level the level-2 solve is genuinely approximate
    dec, B3 = build(case, 3)
    _, B2 = build(case, 3, levels=2)
    z2, z3 = B2.apply(r), B3.apply(r)
    assert np.linalg.norm(z3 - z2) > 1e-3 * np.linalg.norm(z2)


def test_level2_lower_bound_and_symmetry_on_coarse_problem():
    """Level-2 BDDC applied to S_PiPi (972 coarse DOFs, 8 level-2 subdomains)."""
    dec, B = build(clustered(12, 3), 3)
    S = B.L1.Kc
    assert len(B.L2.spaces) == 8 and S.shape == (972, 972)
    Mc = np.stack([B.L2.apply(e) for e in np.eye(S.shape[0])], axis=1)
    assert np.abs(Mc - Mc.T).max() < 1e-12 * np.abs(Mc).max()
    ev = np.linalg.eigvals(Mc @ S)
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() > 1 - 1e-10
    assert ev.real.max() > 1.2                       # a genuine approximation of S_PiPi^-1


@pytest.mark.parametrize("dims,group,cluster,material,primal,primal2", [
    ((6, 6, 6), 2, 1, "linear", 3, 7),               # four slab groups of two subdomains
    ((6, 6, 6), 2, 1, "neo_hookean", 7, 3),
    ((12, 6, 6), 8, 2, "linear", 3, 7),              # two 2x2x2 clusters
])
def test_three_level_lower_bound_symmetry_and_order(dims, group, cluster, material, primal, primal2):
    nx, ny, nz = dims
    case = clustered(nx, 3, material, ny, nz, cluster)
    dec, B3 = build(case, primal, group=group, primal2=primal2)
    assert len(B3.L2.spaces) >= 2
    _, B2 = build(case, primal, levels=2)
    n = len(dec.free)
    A = B3.A.toarray()
    M3 = np.stack([B3.apply(e) for e in np.eye(n)], axis=1)
    M2 = np.stack([B2.apply(e) for e in np.eye(n)], axis=1)
    scale = np.abs(M3).max()
    assert np.abs(M3 - M3.T).max() < 1e-12 * scale
    ev = np.linalg.eigvals(M3 @ A)
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() > 1 - 1e-10
    D = M3 - M2
    assert np.linalg.eigvalsh(0.5 * (D + D.T)).min() > -1e-12 * scale
    assert np.abs(D).max() > 1e-6 * scale            # the level-2 solve is not exact here
