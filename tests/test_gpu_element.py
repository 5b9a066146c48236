"""Device element tangents and internal forces (mbddc_set_material / mbddc_set_displacement)
against the host generator of the same quantities (workloads.element_tangents and
element_internal_forces, whose material laws are pinned by finite differences and closed
forms in tests/test_workloads.py), and a Newton iteration run on the device.

Paper §2: the tangent problem of the hyperelastic balance law (Guccione law with its
volumetric term on the ventricle-like shell; compressible neo-Hookean and Saint
Venant-Kirchhoff on boxes). Bounds: element matrices and forces within 1e-13 of the host's
(relative to their largest entry; only the summation order differs), the assembled operator
within 1e-14, and the Newton iterates within 1e-9 of a host Newton iteration with direct solves.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
from paper_2208_06191_amd import mbddc
from paper_2208_06191_amd import workloads as W

pytestmark = pytest.mark.gpu


def mat_params(material):
    k = material["kind"]
    if k == "svk":
        return (mbddc.MBDDC_MAT_SVK, (material["lam"], material["mu"]))
    if k == "neo_hookean":
        return (mbddc.MBDDC_MAT_NEO_HOOKEAN, (material["mu"], material["lam"]))
    return (mbddc.MBDDC_MAT_GUCCIONE, (material["C"], material["bf"], material["bt"], material["bfs"], material["B"],
                                       material.get("gamma", 0.0)))


def case(name):
    """(mesh, part, nsub, dirichlet, material, u, frames) of one test problem."""
    if name in ("q1_linear", "q1_nh", "q2_nh"):
        order = 2 if name == "q2_nh" else 1
        mesh = W.box_mesh(6, 5, 4, order)
        part, nsub = W.block_partition(mesh, 2 if order == 2 else 3)
        mat = W.linear_elastic(1.0, 0.3) if name == "q1_linear" else W.neo_hookean(1.3, 40.0)
        u = W.isochoric_field(mesh.coords, 7, 0.05) + 0.02 * W.smooth_field(mesh.coords, 8, 1.0)
        return mesh, part, nsub, W.clamp_dofs(mesh, 1), mat, u, None
    mesh, param = W.ventricle_mesh(2, 12, 8, 2)
    part, nsub = W.rcb_partition(mesh, param, 900, 3)
    frames = W.ventricle_frames(mesh, param)
    u = W.isochoric_field(mesh.coords, 2, 0.015)
    mat = W.guccione(gamma=0.3) if name == "shell_guccione_active" else W.guccione()
    return mesh, part, nsub, W.clamp_dofs(mesh, W.VENT_BASE), mat, u, frames


def host_forces(mesh, mat, u, frames, dirichlet):
    fe = W.element_internal_forces(mesh, mat, u, frames_fn=None if frames is None else (lambda el, q: frames[el]))
    f = np.zeros(3 * mesh.n_nodes)
    dofs = (3 * mesh.elem_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(mesh.n_elems, -1)
    np.add.at(f, dofs.ravel(), fe.ravel())
    f[dirichlet] = 0.0
    return f


def handle(mesh, part, nsub, dirichlet):
    m = mbddc._MeshArrays(mesh.coords, mesh.elem_nodes, mesh.elem_type, part, nsub, mesh.node_tags, dirichlet)
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([m], mbddc.default_options(primal=7 if mesh.order == 2 else 3, symmetric_hint=1))
    return s


@pytest.mark.parametrize("name", ["q1_linear", "q1_nh", "q2_nh", "shell_guccione", "shell_guccione_active"])
def test_element_tangents_and_forces_match_host(name):
    torch = pytest.importorskip("torch")
    mesh, part, nsub, dirichlet, mat, u, frames = case(name)
    ffn = None if frames is None else (lambda el, q: frames[el])
    Kh = W.element_tangents(mesh, mat, u, frames_fn=ffn)
    fh = host_forces(mesh, mat, u, frames, dirichlet)
    s = handle(mesh, part, nsub, dirichlet)
    s.mbddc_set_material([mat_params(mat)], frames)
    f = s.mbddc_set_displacement(u.ravel(), f_int=True)
    Kd = s.mbddc_get_element_tangents().reshape(Kh.shape)
    ek = np.abs(Kd - Kh).max() / np.abs(Kh).max()
    ef = np.abs(f - fh).max() / np.abs(fh).max()
    print(f"{name}: element tangents {ek:.2e}, internal forces {ef:.2e}")
    assert ek <= 1e-13 and ef <= 1e-13
    assert np.abs(f[dirichlet]).max() == 0.0
    # device inputs and outputs give the same, and the operator equals the one assembled from K_e
    ud = torch.tensor(u.ravel(), device="cuda")
    fd = s.mbddc_set_displacement(ud, f_int=True)
    assert np.array_equal(fd.cpu().numpy(), f)
    x = np.random.default_rng(1).standard_normal((2, 3 * mesh.n_nodes))
    y1 = s.mbddc_matvec(x)
    ref = handle(mesh, part, nsub, dirichlet)
    ref.mbddc_set_tangent(Kh)
    y2 = ref.mbddc_matvec(x)
    assert np.abs(y1 - y2).max() <= 1e-13 * np.abs(y2).max()
    s.close()
    ref.close()


def test_batch_of_two_materials_and_orders():
    c1, c2 = case("q1_nh"), case("q2_nh")
    m1 = mbddc._MeshArrays(c1[0].coords, c1[0].elem_nodes, c1[0].elem_type, c1[1], c1[2], c1[0].node_tags, c1[3])
    m2 = mbddc._MeshArrays(c2[0].coords, c2[0].elem_nodes, c2[0].elem_type, c2[1], c2[2], c2[0].node_tags, c2[3])
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([m1, m2], mbddc.default_options(primal=3, symmetric_hint=1))
    mat2 = W.linear_elastic(2.0, 0.25)
    s.mbddc_set_material([mat_params(c1[4]), mat_params(mat2)])
    u = np.concatenate([c1[5].ravel(), c2[5].ravel()])
    f = s.mbddc_set_displacement(u, f_int=True)
    K = s.mbddc_get_element_tangents()
    Kh = np.concatenate([W.element_tangents(c1[0], c1[4], c1[5]).ravel(), W.element_tangents(c2[0], mat2, c2[5]).ravel()])
    fh = np.concatenate([host_forces(c1[0], c1[4], c1[5], None, c1[3]), host_forces(c2[0], mat2, c2[5], None, c2[3])])
    assert np.abs(K - Kh).max() <= 1e-13 * np.abs(Kh).max()
    assert np.abs(f - fh).max() <= 1e-13 * np.abs(fh).max()
    s.close()


def test_inverted_element_is_rejected_and_factors_kept():
    mesh, part, nsub, dirichlet, mat, u, _ = case("q1_nh")
    s = handle(mesh, part, nsub, dirichlet)
    s.mbddc_set_material([mat_params(mat)])
    s.mbddc_set_displacement(u.ravel())
    s.mbddc_factor()
    b = W._loads(mesh, dirichlet, 1, 3)
    x0, _ = s.mbddc_solve(b)
    bad = -2.0 * mesh.coords          # F = -I: J = -1
    with pytest.raises(mbddc.MbddcError) as e:
        s.mbddc_set_displacement(bad.ravel())
    assert e.value.status == mbddc.MBDDC_ERR_ARG
    x1, _ = s.mbddc_solve(b)          # operator and factors untouched
    assert np.array_equal(x0, x1)
    with pytest.raises(mbddc.MbddcError) as e:   # but no factorisation of the rejected tangent
        s.mbddc_factor()
    assert e.value.status == mbddc.MBDDC_ERR_STATE
    s.mbddc_set_displacement(u.ravel())
    s.mbddc_factor()
    s.close()


@pytest.mark.parametrize("name", ["q1_nh", "shell_guccione"])
def test_newton_on_device_matches_host_newton(name):
    """u_{k+1} = u_k + K(u_k)^-1 (f_ext - f_int(u_k)), tangents and forces on the device, BDDC-GMRES
    solves to rtol 1e-12; against the same iteration on the host with direct solves."""
    mesh, part, nsub, dirichlet, mat, _, frames = case(name)
    ffn = None if frames is None else (lambda el, q: frames[el])
    fext = 0.05 * W._loads(mesh, dirichlet, 1, 3)[0]
    free = np.setdiff1d(np.arange(3 * mesh.n_nodes), dirichlet)
    s = mbddc.Solver(0)
    m = mbddc._MeshArrays(mesh.coords, mesh.elem_nodes, mesh.elem_type, part, nsub, mesh.node_tags, dirichlet)
    s.mbddc_setup_symbolic([m], mbddc.default_options(primal=7 if mesh.order == 2 else 3, symmetric_hint=1,
                                                      rtol=1e-12, precision=mbddc.MBDDC_FP64))
    s.mbddc_set_material([mat_params(mat)], frames)
    ud = np.zeros(3 * mesh.n_nodes)
    uh = np.zeros(3 * mesh.n_nodes)
    res = []
    for k in range(5):
        fint = s.mbddc_set_displacement(ud, f_int=True)
        s.mbddc_factor()
        r = fext - fint
        res.append(np.linalg.norm(r[free]))
        du, info = s.mbddc_solve(r)
        ud = ud + du
        # host
        Kh = W.element_tangents(mesh, mat, uh.reshape(-1, 3), frames_fn=ffn)
        A = fem.reduce_to_free(fem.assemble(mesh.elem_nodes, Kh, 3 * mesh.n_nodes), free)
        rh = fext - host_forces(mesh, mat, uh.reshape(-1, 3), frames, dirichlet)
        uh[free] += spla.spsolve(A.tocsc(), rh[free])
        e = np.linalg.norm(ud - uh) / np.linalg.norm(uh)
        print(f"{name} Newton step {k}: residual {res[-1]:.3e}, its {info.iterations}, |u_dev - u_host| / |u| = {e:.2e}")
        assert e <= 1e-9
    # Newton's quadratic convergence: once close, each residual is about the square of the last
    assert res[4] <= 1e-7 * res[0]
    assert res[3] <= 10.0 * res[2] ** 2 / res[0] and res[4] < res[3] < res[2]
    s.close()


# ------------------------------------------------------------------ boundary conditions (§2)
def shell_with_bcs():
    mesh, param = W.ventricle_mesh(2, 12, 8, 2)
    part, nsub = W.rcb_partition(mesh, param, 480, 3)
    frames = W.ventricle_frames(mesh, param)
    return mesh, part, nsub, W.clamp_dofs(mesh, W.VENT_BASE), frames


BCS = [(mbddc.MBDDC_BC_ROBIN, W.VENT_EPI, -1, (2.0, 0.5)), (mbddc.MBDDC_BC_PRESSURE, W.VENT_ENDO, -1, (0.05, 0.0))]


def host_boundary(mesh, u):
    K = np.zeros((mesh.n_elems, 81, 81))
    f = np.zeros((mesh.n_elems, 81))
    for kind, tag, _, params in BCS:
        name = "robin" if kind == mbddc.MBDDC_BC_ROBIN else "pressure"
        Kb, fb = W.boundary_terms(mesh, W.boundary_faces(mesh, tag), name, params[:2] if name == "robin" else params[:1],
                                  u)
        K += Kb
        f += fb
    return K, f


def test_boundary_terms_match_host():
    mesh, part, nsub, dirichlet, frames = shell_with_bcs()
    mat = W.guccione()
    u = W.isochoric_field(mesh.coords, 2, 0.015)
    Kv = W.element_tangents(mesh, mat, u, frames_fn=lambda el, q: frames[el])
    Kb, fb = host_boundary(mesh, u)
    fe = W.element_internal_forces(mesh, mat, u, frames_fn=lambda el, q: frames[el]) + fb
    fh = np.zeros(3 * mesh.n_nodes)
    dofs = (3 * mesh.elem_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(mesh.n_elems, -1)
    np.add.at(fh, dofs.ravel(), fe.ravel())
    fh[dirichlet] = 0.0
    s = handle(mesh, part, nsub, dirichlet)
    s.mbddc_set_material([mat_params(mat)], frames)
    s.mbddc_set_boundary(BCS)
    f = s.mbddc_set_displacement(u.ravel(), f_int=True)
    Kd = s.mbddc_get_element_tangents().reshape(Kv.shape)
    Kh = Kv + Kb
    ek = np.abs(Kd - Kh).max() / np.abs(Kh).max()
    ef = np.abs(f - fh).max() / np.abs(fh).max()
    eb = np.abs((Kd - Kv) - Kb).max() / np.abs(Kb).max()
    print(f"shell with Robin and pressure: element tangents {ek:.2e} (boundary part {eb:.2e}), forces {ef:.2e}")
    # the boundary part is isolated by subtracting the much larger volume part: its floor is the
    # total's 1e-13 scaled by their ratio
    assert ek <= 1e-13 and ef <= 1e-13 and eb <= 1e-13 * np.abs(Kh).max() / np.abs(Kb).max()
    s.close()


def test_realistic_shell_newton_nonsymmetric():
    """The realistic setting of §8 in miniature: Guccione shell, base clamped, Robin epicardium,
    follower pressure on the endocardium (a non-symmetric tangent), Newton on the device with the
    non-symmetric BDDC formulation on the pivoted path, against a host Newton with direct solves."""
    mesh, part, nsub, dirichlet, frames = shell_with_bcs()
    mat = W.guccione()
    free = np.setdiff1d(np.arange(3 * mesh.n_nodes), dirichlet)
    m = mbddc._MeshArrays(mesh.coords, mesh.elem_nodes, mesh.elem_type, part, nsub, mesh.node_tags, dirichlet)
    s = mbddc.Solver(0)
    s.mbddc_setup_symbolic([m], mbddc.default_options(primal=7, symmetric_hint=0, rtol=1e-12,
                                                      precision=mbddc.MBDDC_FP64))
    s.mbddc_set_material([mat_params(mat)], frames)
    s.mbddc_set_boundary(BCS)
    ud = np.zeros(3 * mesh.n_nodes)
    uh = np.zeros(3 * mesh.n_nodes)
    dofs = (3 * mesh.elem_nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(mesh.n_elems, -1)
    res = []
    for k in range(5):
        fint = s.mbddc_set_displacement(ud, f_int=True)
        s.mbddc_factor()
        r = -fint
        res.append(np.linalg.norm(r[free]))
        du, info = s.mbddc_solve(r)
        ud = ud + du
        U = uh.reshape(-1, 3)
        Kb, fb = host_boundary(mesh, U)
        Kh = W.element_tangents(mesh, mat, U, frames_fn=lambda el, q: frames[el]) + Kb
        A = fem.reduce_to_free(fem.assemble(mesh.elem_nodes, Kh, 3 * mesh.n_nodes), free)
        fe = W.element_internal_forces(mesh, mat, U, frames_fn=lambda el, q: frames[el]) + fb
        fh = np.zeros(3 * mesh.n_nodes)
        np.add.at(fh, dofs.ravel(), fe.ravel())
        uh[free] += spla.spsolve(A.tocsc(), -fh[free])
        e = np.linalg.norm(ud - uh) / np.linalg.norm(uh)
        print(f"realistic Newton step {k}: residual {res[-1]:.3e}, its {info.iterations}, |u_dev - u_host| / |u| = {e:.2e}")
        assert e <= 1e-9
    assert res[4] <= 1e-7 * res[0]
    s.close()
