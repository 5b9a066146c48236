"""Shared fixtures. Tests marked ``gpu`` need an MI355X and the built HIP library."""
import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@functools.lru_cache(maxsize=None)
def problem(name: str):
    """Seeded problems shared across test modules (built once per session)."""
    from paper_2208_06191_amd import workloads as W
    if name == "small":            # 8^3 Q1 linear elasticity, 2x2x2 subdomains, primal V
        return W.config_small()
    if name == "small_ve":
        return W.linear_box(8, 4, 1, nrhs=2, primal=3, name="small_ve")
    if name == "tiny":             # 6^3 Q1, 2x2x2 subdomains of 3^3
        return W.linear_box(6, 3, 1, nrhs=1, primal=1, name="tiny")
    if name == "tiny_nh":          # neo-Hookean tangent on 8^3, 2x2x2 subdomains, VE
        return W.neo_hookean_box(8, 4, 1, nrhs=2, amplitude=0.02, primal=3, name="tiny_nh")
    if name == "tiny_q2":          # Q2 on 4^3 elements, 2x2x2 subdomains of 2^3
        return W.linear_box(4, 2, 2, nrhs=1, primal=3, name="tiny_q2")
    if name == "q2_dense":         # Q2 on 8^3 elements: node rows of 50+ 3x3 blocks on average
        return W.linear_box(8, 2, 2, nrhs=1, primal=3, name="q2_dense")
    if name == "l3_nh":            # neo-Hookean on 12^3, 4x4x4 subdomains of 3^3: three-level cases
        return W.neo_hookean_box(12, 3, 1, nrhs=2, amplitude=0.02, primal=3, name="l3_nh")
    if name == "l3_ragged":        # 7x6x9 Q1 box, blocks of 2 -> 4x3x5 uneven subdomains, linear elastic
        from paper_2208_06191_amd.workloads import Problem
        mesh = W.box_mesh(7, 6, 9, 1)
        part, nsub = W.block_partition(mesh, 2)
        dirichlet = W.clamp_dofs(mesh, 1)
        Ke = W.element_tangents(mesh, W.linear_elastic(1.0, 0.3))
        rhs = W._loads(mesh, dirichlet, 1, 11)
        return Problem("l3_ragged", mesh, part, nsub, dirichlet, Ke, rhs, 1, {})
    if name == "vent":             # Q2 ventricle-like shell, Guccione fibres, RCB parts <= 480 DOFs
        return W.ventricle(2, 16, 8, 2, target_dofs=480, nrhs=2, primal=7, name="vent")
    if name == "large_q1":         # 16^3 Q1, 2x2x2 subdomains of 8^3: local blocks of 600-1536 DOFs
        return W.linear_box(16, 8, 1, nrhs=2, primal=3, name="large_q1")
    if name == "large_mixed":      # 14x10x12 Q1 neo-Hookean, blocks of 8: interiors of 144-1344 DOFs
        from paper_2208_06191_amd.workloads import Problem
        mesh = W.box_mesh(14, 10, 12, 1)
        part, nsub = W.block_partition(mesh, 8)
        dirichlet = W.clamp_dofs(mesh, 1)
        u = W.isochoric_field(mesh.coords, 4, 0.02)
        Ke = W.element_tangents(mesh, W.neo_hookean(1.0, 50.0), u)
        rhs = W._loads(mesh, dirichlet, 2, 7)
        return Problem("large_mixed", mesh, part, nsub, dirichlet, Ke, rhs, 3, {})
    if name == "vent_large":       # Q2 ventricle-like shell, RCB parts <= 2500 DOFs
        return W.ventricle(2, 16, 8, 2, target_dofs=2500, nrhs=1, primal=7, name="vent_large")
    if name == "vent_parts6k":     # the shell at 1/16 of the full mesh, RCB parts of 2k-5.7k DOFs as at full size
        return W.ventricle(4, 24, 24, 2, target_dofs=6000, nrhs=1, primal=7, name="vent_parts6k")
    if name == "ragged":           # 6x5x7 Q1 box, blocks of 4 -> uneven subdomains
        from paper_2208_06191_amd.workloads import Problem
        mesh = W.box_mesh(6, 5, 7, 1)
        part, nsub = W.block_partition(mesh, 4)
        dirichlet = W.clamp_dofs(mesh, 1)
        u = W.isochoric_field(mesh.coords, 3, 0.02)
        Ke = W.element_tangents(mesh, W.neo_hookean(1.0, 50.0), u)
        rhs = W._loads(mesh, dirichlet, 2, 5)
        return Problem("ragged", mesh, part, nsub, dirichlet, Ke, rhs, 3, {})
    raise KeyError(name)


@pytest.fixture
def get_problem():
    return problem


@functools.lru_cache(maxsize=None)
def apply_noise_floor(name: str, primal: int, levels: int = 2, group: int = 8, primal2: int = 7) -> float:
    """How far the oracle's own FP64 preconditioner application moves when every element
    tangent entry is perturbed by a relative 2.2e-16 (seeded): no FP64 implementation of the
    same operator can be held closer to the oracle than this (the apply's condition)."""
    import numpy as np
    from oracle import bddc
    P = problem(name)
    dec = bddc.Decomposition(P.mesh.elem_nodes, P.mesh.n_nodes, P.elem_part, P.n_sub, P.dirichlet,
                             P.mesh.node_tags, primal=primal)
    E = np.random.default_rng(1).standard_normal(P.Ke.shape)
    E = 0.5 * (E + E.transpose(0, 2, 1))
    r = np.random.default_rng(3).standard_normal(P.n_dofs)[dec.free]
    out = []
    for Ke in (P.Ke, P.Ke * (1.0 + 2.2e-16 * E)):
        B = bddc.BDDC(dec, P.mesh.elem_nodes, Ke, levels=levels, coarse_group=group, level2_primal=primal2)
        out.append(B.apply(r))
    return float(np.linalg.norm(out[0] - out[1]) / np.linalg.norm(out[0]))
