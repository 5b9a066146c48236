"""Pins for the seeded input generators (element tangents, loads, meshes).

These check the generator against facts fixed by continuum mechanics and the
finite-element method, independent of any solver code:
* rigid motions are in the kernel of the unconstrained elastic stiffness;
* the consistent body-force load integrates to the body force times volume;
* the neo-Hookean tangent at zero displacement is the linear-elastic one with
  lambda = kappa - 2 mu / 3;
* every tangent is the derivative of its internal force (central differences);
* hyperelastic element tangents are symmetric.
"""
import numpy as np
import pytest

from paper_2208_06191_amd import workloads as W
from oracle import fem


@pytest.mark.parametrize("order", [1, 2])
def test_partition_of_unity_and_volume(order):
    pts, wts = W.gauss_rule(order + 1)
    N, dN = W.shape_functions(order, pts)
    assert np.allclose(N.sum(axis=1), 1.0, atol=1e-14)
    assert np.allclose(dN.sum(axis=1), 0.0, atol=1e-13)
    assert abs(wts.sum() - 1.0) < 1e-14
    mesh = W.box_mesh(2, 3, 2, order, lengths=(2.0, 1.5, 1.0))
    b = W.body_force_load(mesh, np.tile([0.0, 0.0, -1.0], (mesh.n_nodes, 1)))
    assert abs(b[2::3].sum() + 3.0) < 1e-12        # body force x volume (2 * 1.5 * 1)
    assert abs(b[0::3].sum()) < 1e-14


@pytest.mark.parametrize("order", [1, 2])
def test_rigid_motions_in_kernel(order):
    mesh = W.box_mesh(3, 2, 2, order)
    Ke = W.element_tangents(mesh, W.linear_elastic(1.0, 0.3))
    K = fem.assemble(mesh.elem_nodes, Ke, 3 * mesh.n_nodes)
    R = fem.rigid_body_modes(mesh.coords)
    scale = abs(K).max() * np.abs(R).max()
    assert np.abs(K @ R).max() < 1e-12 * scale
    # and nothing else: exactly 6 zero eigenvalues
    ev = np.linalg.eigvalsh(K.toarray())
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == 6


def test_translations_in_kernel_of_prestressed_tangent():
    mesh = W.box_mesh(3, 3, 2, 1)
    u = W.isochoric_field(mesh.coords, 7, 0.05)
    Ke = W.element_tangents(mesh, W.neo_hookean(1.0, 50.0), u)
    K = fem.assemble(mesh.elem_nodes, Ke, 3 * mesh.n_nodes)
    T = fem.rigid_body_modes(mesh.coords)[:, :3]
    assert np.abs(K @ T).max() < 1e-11 * abs(K).max()
    assert np.abs(Ke - np.transpose(Ke, (0, 2, 1))).max() < 1e-12 * np.abs(Ke).max()


def test_neo_hookean_at_rest_is_linear_elasticity():
    mesh = W.box_mesh(2, 2, 2, 1)
    mu, kappa = 1.3, 50.0
    lam = kappa - 2 * mu / 3
    E = mu * (3 * lam + 2 * mu) / (lam + mu)
    nu = lam / (2 * (lam + mu))
    K1 = W.element_tangents(mesh, W.neo_hookean(mu, kappa))
    K2 = W.element_tangents(mesh, W.linear_elastic(E, nu))
    assert np.abs(K1 - K2).max() < 1e-12 * np.abs(K2).max()


def test_isochoric_field_is_divergence_free_and_clamped():
    mesh = W.box_mesh(4, 4, 4, 2)
    u = W.isochoric_field(mesh.coords, 0, 0.05)
    assert abs(np.linalg.norm(u, axis=1).max() - 0.05) < 1e-15
    assert np.abs(u[mesh.node_tags & 1 == 1]).max() == 0.0
    # analytic divergence by central differences at random interior points (one call, so
    # the max-norm rescaling is shared by every evaluation point)
    rng = np.random.default_rng(0)
    X0 = rng.uniform(0.1, 0.9, size=(50, 3))
    h = 1e-5
    pts = [X0]
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        pts += [X0 + e, X0 - e]
    U = W.isochoric_field(np.concatenate(pts), 0, 1.0).reshape(7, 50, 3)
    div = sum((U[1 + 2 * i, :, i] - U[2 + 2 * i, :, i]) / (2 * h) for i in range(3))
    grad = np.abs(U[1] - U[2]).max() / (2 * h)
    assert np.abs(div).max() < 1e-8 * grad


def _fd_check(mesh, material, u, frames_fn=None, h=1e-6):
    rng = np.random.default_rng(11)
    d = rng.standard_normal(u.shape) * 1e-2
    Ke = W.element_tangents(mesh, material, u, frames_fn=frames_fn)
    fp = W.element_internal_forces(mesh, material, u + h * d, frames_fn=frames_fn)
    fm = W.element_internal_forces(mesh, material, u - h * d, frames_fn=frames_fn)
    de = d[mesh.elem_nodes].reshape(mesh.n_elems, -1)
    lin = np.einsum("eij,ej->ei", Ke, de)
    fd = (fp - fm) / (2 * h)
    return np.abs(lin - fd).max() / np.abs(lin).max()


@pytest.mark.parametrize("order", [1, 2])
def test_neo_hookean_tangent_is_derivative_of_internal_force(order):
    mesh = W.box_mesh(2, 2, 1, order)
    u = W.smooth_field(mesh.coords, 3, 0.05)
    assert _fd_check(mesh, W.neo_hookean(1.0, 50.0), u) < 1e-7


def test_guccione_tangent_is_derivative_of_internal_force():
    mesh = W.box_mesh(2, 1, 2, 1)
    u = W.smooth_field(mesh.coords, 4, 0.05)
    rng = np.random.default_rng(2)
    Qs = {}

    def frames(elems, q):
        key = (len(elems), q)
        if key not in Qs:
            A = rng.standard_normal((len(elems), 3, 3))
            Qs[key] = np.linalg.qr(A)[0].transpose(0, 2, 1)
        return Qs[key]
    assert _fd_check(mesh, W.guccione(), u, frames_fn=frames) < 1e-7


# ---------------------------------------------------------------- ventricle-like shell
def _shell_volume(a=1.0, c=2.5, w=0.3, phi0=np.deg2rad(10.0)):
    """Closed form of the mapped shell's volume: the map's Jacobian is
    w r1 sin(phi) (r3 sin^2(phi) + r1 cos^2(phi)) with r1 = a + w t, r3 = c + w t."""
    cp = np.cos(phi0)
    return 2 * np.pi * w * ((a * c + (a + c) * w / 2 + w * w / 3) * (cp - cp ** 3 / 3)
                            + (a * a + a * w + w * w / 3) * cp ** 3 / 3)


def test_ventricle_volume_tags_and_clamp():
    mesh, param = W.ventricle_mesh(2, 16, 8, 2)
    f = np.zeros((mesh.n_nodes, 3))
    f[:, 2] = 1.0
    vol = W.body_force_load(mesh, f).reshape(-1, 3)[:, 2].sum()   # sum of N_a |J| = volume
    assert abs(vol - _shell_volume()) < 2e-4 * _shell_volume()
    base = (mesh.node_tags & W.VENT_BASE) != 0
    assert np.allclose(mesh.coords[base, 2], 0.0, atol=1e-14) and base.sum() == 5 * 32
    endo = (mesh.node_tags & W.VENT_ENDO) != 0
    X = mesh.coords[endo]
    assert np.allclose((X[:, 0] ** 2 + X[:, 1] ** 2) / 1.0 + X[:, 2] ** 2 / 2.5 ** 2, 1.0)
    # periodic seam: every element's nodes are distinct and theta wraps around
    assert all(len(set(e)) == 27 for e in mesh.elem_nodes)


def test_ventricle_fibre_frames():
    mesh, param = W.ventricle_mesh(3, 12, 6, 2)
    Q = W.ventricle_frames(mesh, param)
    assert np.abs(np.einsum("eai,ebi->eab", Q, Q) - np.eye(3)).max() < 1e-12
    assert np.all(np.linalg.det(Q) > 0)
    # helix angle: +60 deg at the endocardial side decreasing to -60 deg, linear in t
    tc = W.ventricle_elem_param(mesh)[:, 0]
    Xc = mesh.coords[mesh.elem_nodes].mean(axis=1)
    th = np.arctan2(Xc[:, 1], Xc[:, 0])
    e_th = np.stack([-np.sin(th), np.cos(th), np.zeros_like(th)], axis=1)
    cos_a = np.einsum("ei,ei->e", Q[:, 0], e_th)
    assert np.allclose(cos_a, np.cos(np.deg2rad(60.0 - 120.0 * tc)), atol=1e-12)
    # the fibre turns from "upward" (towards the base) at the endocardium to downward outside
    up = Q[:, 0, 2]
    assert np.all(up[tc < 0.2] > 0) and np.all(up[tc > 0.8] < 0)


def test_rcb_parts_are_bounded_connected_and_cover():
    mesh, param = W.ventricle_mesh(2, 16, 8, 2)
    part, nsub = W.rcb_partition(mesh, param, 480, 3)
    assert part.min() == 0 and part.max() == nsub - 1
    for i in range(nsub):
        el = np.nonzero(part == i)[0]
        assert 3 * len(np.unique(mesh.elem_nodes[el])) <= 480
        # connectivity through shared nodes
        seen, front = {el[0]}, [el[0]]
        nodes_of = {e: set(mesh.elem_nodes[e]) for e in el}
        while front:
            e = front.pop()
            for f_ in el:
                if f_ not in seen and nodes_of[e] & nodes_of[f_]:
                    seen.add(f_)
                    front.append(f_)
        assert len(seen) == len(el)


def test_ventricle_guccione_tangent_is_derivative_of_internal_force():
    mesh, param = W.ventricle_mesh(1, 4, 2, 2)
    Q = W.ventricle_frames(mesh, param)
    u = W.isochoric_field(mesh.coords, 2, 0.015)
    assert _fd_check(mesh, W.guccione(), u, frames_fn=lambda e, q: Q[e]) < 1e-7


def test_ventricle_newton_request_shapes_and_first_step():
    """A serving request on the shell: RCB parts within the bound, base clamped, and step 0's
    tangents are those of the first iterate u0 (the steps differ)."""
    mesh, part, nsub, dirichlet, Ks = W.ventricle_newton(1.2e4, 3, 41, part_dofs=2000)
    assert Ks.shape == (3, mesh.n_elems, 81, 81)
    assert part.min() == 0 and part.max() == nsub - 1
    for i in range(nsub):
        nodes = np.unique(mesh.elem_nodes[part == i])
        assert 3 * len(nodes) <= 2000
    assert len(dirichlet) > 0 and np.all(mesh.node_tags[np.asarray(dirichlet) // 3] & W.VENT_BASE)
    assert np.allclose(Ks[0], Ks[0].transpose(0, 2, 1), atol=1e-10 * np.abs(Ks[0]).max())
    assert np.abs(Ks[2] - Ks[0]).max() > 1e-6 * np.abs(Ks[0]).max()


# ------------------------------------------------------------------ boundary conditions (§2)
@pytest.mark.parametrize("kind,params", [("robin", (2.0, 0.5)), ("pressure", (0.7,))])
def test_boundary_tangent_is_derivative_of_boundary_force(kind, params):
    mesh, param = W.ventricle_mesh(2, 8, 6, 2)
    faces = W.boundary_faces(mesh, W.VENT_ENDO if kind == "pressure" else W.VENT_EPI)
    assert len(faces) == 8 * 6
    u = W.isochoric_field(mesh.coords, 5, 0.02)
    du = W.smooth_field(mesh.coords, 6, 1.0)
    K, f0 = W.boundary_terms(mesh, faces, kind, params, u)
    h = 1e-6
    _, fp = W.boundary_terms(mesh, faces, kind, params, u + h * du)
    _, fm = W.boundary_terms(mesh, faces, kind, params, u - h * du)
    fd = (fp - fm) / (2 * h)
    due = du[mesh.elem_nodes].reshape(mesh.n_elems, -1)
    lin = np.einsum("eij,ej->ei", K, due)
    assert np.abs(fd - lin).max() <= 1e-7 * np.abs(lin).max()
    if kind == "robin":   # linear in u, symmetric
        assert np.abs(K - np.transpose(K, (0, 2, 1))).max() <= 1e-14 * np.abs(K).max()
    else:                 # a follower load: not symmetric
        assert np.abs(K - np.transpose(K, (0, 2, 1))).max() > 1e-3 * np.abs(K).max()


def test_pressure_on_a_closed_surface_has_no_resultant():
    """Piola: the integral of J F^-T N over a closed reference surface is the integral of the
    current normal over the closed deformed surface, zero for any deformation."""
    mesh = W.box_mesh(3, 2, 2, 2)
    faces = np.concatenate([W.boundary_faces(mesh, bit) for bit in (1, 2, 4, 8, 16, 32)])
    u = W.isochoric_field(mesh.coords, 7, 0.05) + 0.03 * W.smooth_field(mesh.coords, 8, 1.0)
    _, f = W.boundary_terms(mesh, faces, "pressure", (1.3,), u)
    tot = f.reshape(mesh.n_elems, -1, 3).sum(axis=(0, 1))
    area = 2 * (1 + 1 + 1)
    assert np.abs(tot).max() <= 1e-12 * area
    # and the reference outward normals of a box: the resultant of a uniform unit pressure on one
    # face is its area along the outward normal
    _, f1 = W.boundary_terms(mesh, W.boundary_faces(mesh, 2), "pressure", (1.0,))
    assert np.allclose(f1.reshape(mesh.n_elems, -1, 3).sum(axis=(0, 1)), [1.0, 0.0, 0.0], atol=1e-13)


def test_active_stress_tangent_is_derivative_and_stress_is_along_the_fibre():
    """§2 active part P_act = gamma (F f) (x) f / |F f|: the tangent with it is still the derivative
    of the internal force, and at u = 0 it adds exactly gamma f (x) f to the stress (|f| = 1)."""
    mesh, param = W.ventricle_mesh(2, 8, 6, 2)
    Q = W.ventricle_frames(mesh, param)
    u = W.isochoric_field(mesh.coords, 3, 0.02)
    assert _fd_check(mesh, W.guccione(gamma=0.4), u, frames_fn=lambda e, q: Q[e]) < 1e-7
    F = np.broadcast_to(np.eye(3), (5, 3, 3)).copy()
    mat = dict(W.guccione(gamma=0.4), frames=Q[:5])
    S1, _ = W._stress_tangent(mat, F)
    S0, _ = W._stress_tangent(dict(W.guccione(), frames=Q[:5]), F)
    assert np.abs(S1 - S0 - 0.4 * np.einsum("mi,mj->mij", Q[:5, 0], Q[:5, 0])).max() < 1e-14
