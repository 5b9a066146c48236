"""Seeded synthetic workloads: meshes, partitions, element tangents and loads.

This module only synthesises *inputs* to the solver: structured Q1/Q2 hexahedral
box meshes (paper §2, "Space discretization": H1-conforming hexahedral elements of
order 1 and 2), element-by-element tangent matrices of hyperelastic materials
linearised at a given displacement (the Newton tangent of §2, eq. "tangent
problem"), consistent body-force load vectors, homogeneous Dirichlet clamps and
structured subdomain partitions (§3.2, non-overlapping decomposition).

It holds none of the domain-decomposition arithmetic: no assembly of a global
operator, no interface classification, no factorisation and no Krylov method.
Both the solver library and the FP64 checker consume what it produces.

Conventions
-----------
* Nodes of an ``nx x ny x nz`` element box of order ``p`` are numbered
  lexicographically with x fastest: ``node(i, j, k) = i + Nx*(j + Ny*k)`` with
  ``Nx = p*nx + 1``.
* Element-local node ``(a, b, c)`` (each in ``0..p``) has local index
  ``a + (p+1)*b + (p+1)**2*c``.
* Degree of freedom ``3*node + comp`` (the strided block-size-3 layout of §4).
* Element matrices are ``[n_el, 3*npe, 3*npe]`` in that local DOF order.
* Boundary tag bits per node: 1:x=0, 2:x=Lx, 4:y=0, 8:y=Ly, 16:z=0, 32:z=Lz.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import concurrent.futures
import os

import numpy as np

HEX8 = 1
HEX27 = 2


# ----------------------------------------------------------------------------
# reference element (tensor-product Lagrange on [0,1]^3) and Gauss rules
# ----------------------------------------------------------------------------
def _lagrange_1d(order: int, x: np.ndarray):
    """Values and derivatives of the 1D Lagrange basis on equispaced points of [0,1]."""
    x = np.asarray(x, dtype=np.float64)
    if order == 1:
        v = np.stack([1.0 - x, x])
        d = np.stack([-np.ones_like(x), np.ones_like(x)])
    elif order == 2:
        v = np.stack([2.0 * (x - 0.5) * (x - 1.0), -4.0 * x * (x - 1.0), 2.0 * x * (x - 0.5)])
        d = np.stack([4.0 * x - 3.0, -8.0 * x + 4.0, 4.0 * x - 1.0])
    else:
        raise ValueError("order must be 1 or 2")
    return v, d  # [p+1, len(x)]


def gauss_rule(npts: int):
    """Tensor Gauss-Legendre rule on [0,1]^3: points [q,3], weights [q]."""
    g, w = np.polynomial.legendre.leggauss(npts)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    for k in range(npts):
        for j in range(npts):
            for i in range(npts):
                pts.append((g[i], g[j], g[k]))
                wts.append(w[i] * w[j] * w[k])
    return np.array(pts), np.array(wts)


def shape_functions(order: int, pts: np.ndarray):
    """N [q, npe] and dN/dxi [q, npe, 3] at reference points, lexicographic local order."""
    p1 = order + 1
    vx, dx = _lagrange_1d(order, pts[:, 0])
    vy, dy = _lagrange_1d(order, pts[:, 1])
    vz, dz = _lagrange_1d(order, pts[:, 2])
    q = pts.shape[0]
    N = np.empty((q, p1 ** 3))
    dN = np.empty((q, p1 ** 3, 3))
    for c in range(p1):
        for b in range(p1):
            for a in range(p1):
                l = a + p1 * b + p1 * p1 * c
                N[:, l] = vx[a] * vy[b] * vz[c]
                dN[:, l, 0] = dx[a] * vy[b] * vz[c]
                dN[:, l, 1] = vx[a] * dy[b] * vz[c]
                dN[:, l, 2] = vx[a] * vy[b] * dz[c]
    return N, dN


# ----------------------------------------------------------------------------
# meshes and partitions
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Mesh:
    coords: np.ndarray        # [n_nodes, 3] float64
    elem_nodes: np.ndarray    # [n_el, npe] int32
    order: int                # 1 (HEX8) or 2 (HEX27)
    node_tags: np.ndarray     # [n_nodes] uint32 boundary-surface bitmask
    shape: tuple = ()         # element counts per direction for boxes

    @property
    def elem_type(self) -> int:
        return HEX8 if self.order == 1 else HEX27

    @property
    def n_nodes(self) -> int:
        return self.coords.shape[0]

    @property
    def n_elems(self) -> int:
        return self.elem_nodes.shape[0]

    @property
    def npe(self) -> int:
        return self.elem_nodes.shape[1]


def box_mesh(nx: int, ny: int, nz: int, order: int = 1, lengths=(1.0, 1.0, 1.0)) -> Mesh:
    p = order
    Nx, Ny, Nz = p * nx + 1, p * ny + 1, p * nz + 1
    i = np.arange(Nx)
    j = np.arange(Ny)
    k = np.arange(Nz)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    coords = np.stack([I.ravel() * lengths[0] / (p * nx),
                       J.ravel() * lengths[1] / (p * ny),
                       K.ravel() * lengths[2] / (p * nz)], axis=1)
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    tags = ((I == 0) * 1 | (I == Nx - 1) * 2 | (J == 0) * 4 | (J == Ny - 1) * 8
            | (K == 0) * 16 | (K == Nz - 1) * 32).astype(np.uint32)
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    p1 = p + 1
    en = np.empty((nx * ny * nz, p1 ** 3), dtype=np.int64)
    for c in range(p1):
        for b in range(p1):
            for a in range(p1):
                en[:, a + p1 * b + p1 * p1 * c] = (p * ex + a) + Nx * ((p * ey + b) + Ny * (p * ez + c))
    return Mesh(coords=coords, elem_nodes=en.astype(np.int32), order=order,
                node_tags=tags, shape=(nx, ny, nz))


def block_partition(mesh: Mesh, block, cluster: int = 1) -> tuple[np.ndarray, int]:
    """Element -> subdomain map for axis-aligned blocks of ``block`` elements per direction.

    Subdomains are numbered lexicographically; with ``cluster`` > 1 they are numbered
    cluster by cluster instead (clusters of cluster^3 neighbouring subdomains, each
    lexicographic inside), so that consecutive groups of cluster^3 subdomain ids are
    compact clusters (the grouping of fine subdomains into level-2 subdomains)."""
    nx, ny, nz = mesh.shape
    bx, by, bz = (block, block, block) if np.isscalar(block) else block
    sx, sy, sz = -(-nx // bx), -(-ny // by), -(-nz // bz)
    e = np.arange(nx * ny * nz)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    part = (ex // bx) + sx * ((ey // by) + sy * (ez // bz))
    if cluster > 1:
        s = np.arange(sx * sy * sz)
        i, j, k = s % sx, (s // sx) % sy, s // (sx * sy)
        c = cluster
        cx, cy = -(-sx // c), -(-sy // c)
        key = ((i // c) + cx * ((j // c) + cy * (k // c))) * c ** 3 + (i % c) + c * ((j % c) + c * (k % c))
        rank = np.empty_like(s)
        rank[np.argsort(key, kind="stable")] = s
        part = rank[part]
    return part.astype(np.int32), sx * sy * sz


def clamp_dofs(mesh: Mesh, tag_bit: int = 1) -> np.ndarray:
    """All three DOFs of every node carrying ``tag_bit`` (default: face x=0)."""
    nodes = np.nonzero(mesh.node_tags & tag_bit)[0]
    return np.sort((3 * nodes[:, None] + np.arange(3)[None, :]).ravel()).astype(np.int32)


# ----------------------------------------------------------------------------
# seeded smooth fields
# ----------------------------------------------------------------------------
def smooth_field(X: np.ndarray, seed: int, amplitude: float, n_modes: int = 8) -> np.ndarray:
    """u(X) = sum_m a_m sin(pi k_m.X + phi_m), k_m in {1,2}^3, a_m ~ N(0, I3),
    phi_m ~ U[0, 2pi), rescaled so that max_nodes |u| = amplitude."""
    rng = np.random.default_rng(seed)
    kvec = rng.integers(1, 3, size=(n_modes, 3)).astype(np.float64)
    amp = rng.standard_normal((n_modes, 3))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    arg = np.pi * X @ kvec.T + phase[None, :]          # [n, m]
    u = np.sin(arg) @ amp                               # [n, 3]
    mx = np.max(np.linalg.norm(u, axis=1))
    return u * (amplitude / mx) if mx > 0 else u


def isochoric_field(X: np.ndarray, seed: int, amplitude: float, n_modes: int = 8) -> np.ndarray:
    """Divergence-free displacement u = curl(x^2 psi), psi the seeded 8-mode sine field,
    rescaled to max_nodes |u| = amplitude. It vanishes on the clamped face x = 0 and keeps
    J = 1 + O(|grad u|^2), the natural state of a nearly incompressible solid."""
    rng = np.random.default_rng(seed)
    kvec = rng.integers(1, 3, size=(n_modes, 3)).astype(np.float64)
    amp = rng.standard_normal((n_modes, 3))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    arg = np.pi * X @ kvec.T + phase[None, :]
    psi = np.sin(arg) @ amp                                             # [n, 3]
    gpsi = np.einsum("nm,mj,mi->nji", np.cos(arg), amp, np.pi * kvec)   # d psi_j / d X_i
    curl = np.stack([gpsi[:, 2, 1] - gpsi[:, 1, 2], gpsi[:, 0, 2] - gpsi[:, 2, 0],
                     gpsi[:, 1, 0] - gpsi[:, 0, 1]], axis=1)
    x = X[:, 0]
    gx2 = np.zeros_like(X)
    gx2[:, 0] = 2.0 * x
    u = np.cross(gx2, psi) + (x * x)[:, None] * curl
    mx = np.max(np.linalg.norm(u, axis=1))
    return u * (amplitude / mx) if mx > 0 else u


# ----------------------------------------------------------------------------
# materials: second Piola-Kirchhoff stress S and material tangent C = dS/dE
# (the Newton tangent of a hyperelastic potential, paper §2)
# ----------------------------------------------------------------------------
def _eye3():
    return np.eye(3)


def linear_elastic(E: float = 1.0, nu: float = 0.3):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return {"kind": "svk", "lam": lam, "mu": mu}


def neo_hookean(mu: float = 1.0, kappa: float = 50.0):
    return {"kind": "neo_hookean", "mu": mu, "lam": kappa - 2.0 * mu / 3.0}


def _stress_tangent(mat, F):
    """F [m,3,3] -> S [m,3,3], CC [m,3,3,3,3] (dS/dE, major-symmetric)."""
    I = _eye3()
    m = F.shape[0]
    if mat["kind"] == "svk":
        # Saint Venant-Kirchhoff: the linear-elastic law written on E.
        lam, mu = mat["lam"], mat["mu"]
        C = np.einsum("mki,mkj->mij", F, F)
        E = 0.5 * (C - I)
        trE = np.trace(E, axis1=1, axis2=2)
        S = lam * trE[:, None, None] * I + 2 * mu * E
        CC = (lam * np.einsum("ij,kl->ijkl", I, I)
              + mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I)))
        CC = np.broadcast_to(CC, (m, 3, 3, 3, 3)).copy()
        return S, CC
    if mat["kind"] == "neo_hookean":
        # Psi = mu/2 (I1 - 3) - mu ln J + lam/2 (ln J)^2
        lam, mu = mat["lam"], mat["mu"]
        C = np.einsum("mki,mkj->mij", F, F)
        J = np.linalg.det(F)
        if np.any(J <= 0):
            raise ValueError("non-positive Jacobian at a quadrature point")
        Ci = np.linalg.inv(C)
        lnJ = np.log(J)
        S = mu * (I - Ci) + (lam * lnJ)[:, None, None] * Ci
        CC = (lam * np.einsum("mij,mkl->mijkl", Ci, Ci)
              + (mu - lam * lnJ)[:, None, None, None, None]
              * (np.einsum("mik,mjl->mijkl", Ci, Ci) + np.einsum("mil,mjk->mijkl", Ci, Ci)))
        return S, CC
    if mat["kind"] == "guccione":
        return _guccione(mat, F)
    raise ValueError(mat["kind"])


def guccione(C: float = 0.88, bf: float = 8.0, bt: float = 2.0, bfs: float = 2.0, B: float = 50.0,
             gamma: float = 0.0):
    """Guccione law; gamma > 0 adds the active stress of §2, P_act = gamma (F f) (x) f / |F f|."""
    return {"kind": "guccione", "C": C, "bf": bf, "bt": bt, "bfs": bfs, "B": B, "gamma": gamma}


def _guccione(mat, F):
    """Guccione exponential law in the fibre frame plus B/2 (J-1) ln J (paper §2).
    ``mat['frames']`` holds the per-point rotation Q [m,3,3] whose rows are f, s, n."""
    I = _eye3()
    Q = mat["frames"]
    Cm, bf, bt, bfs, B = mat["C"], mat["bf"], mat["bt"], mat["bfs"], mat["B"]
    Cg = np.einsum("mki,mkj->mij", F, F)
    E = 0.5 * (Cg - I)
    Ef = np.einsum("mai,mij,mbj->mab", Q, E, Q)           # E in the fibre frame
    b = np.array([[bf, bfs, bfs], [bfs, bt, bt], [bfs, bt, bt]])
    Qv = np.einsum("ab,mab->m", b, Ef * Ef)
    eQ = np.exp(Qv)
    # S_frame = C e^Q b.E_frame ; C_frame = C e^Q (2 (b.E)(b.E) + diag-b)
    bE = b[None] * Ef
    S_f = Cm * eQ[:, None, None] * bE
    Cf = Cm * eQ[:, None, None, None, None] * (2.0 * np.einsum("mab,mcd->mabcd", bE, bE)
                                              + 0.5 * (np.einsum("ab,ac,bd->abcd", b, I, I)
                                                       + np.einsum("ab,ad,bc->abcd", b, I, I))[None])
    S = np.einsum("mai,mab,mbj->mij", Q, S_f, Q)
    CC = np.einsum("mai,mbj,mck,mdl,mabcd->mijkl", Q, Q, Q, Q, Cf, optimize=True)
    # volumetric part W(J) = B/2 (J-1) ln J:  S_vol = J W'(J) C^-1
    J = np.linalg.det(F)
    if np.any(J <= 0):
        raise ValueError("non-positive Jacobian at a quadrature point")
    Ci = np.linalg.inv(Cg)
    lnJ = np.log(J)
    W1 = 0.5 * B * (lnJ + (J - 1.0) / J)
    W2 = 0.5 * B * (1.0 / J + 1.0 / (J * J))
    a1 = J * W1
    a2 = J * W1 + J * J * W2
    S = S + a1[:, None, None] * Ci
    CC = CC + (a2[:, None, None, None, None] * np.einsum("mij,mkl->mijkl", Ci, Ci)
               - a1[:, None, None, None, None]
               * (np.einsum("mik,mjl->mijkl", Ci, Ci) + np.einsum("mil,mjk->mijkl", Ci, Ci)))
    gamma = mat.get("gamma", 0.0)
    if gamma != 0.0:
        # active stress P_act = gamma (F f) (x) f / |F f|: S_act = gamma f (x) f / sqrt(f.C f),
        # CC_act = 2 dS_act/dC = -gamma f (x) f (x) f (x) f / (f.C f)^(3/2)
        f = Q[:, 0, :]
        lam2 = np.einsum("mi,mij,mj->m", f, Cg, f)
        ff = np.einsum("mi,mj->mij", f, f)
        S = S + (gamma / np.sqrt(lam2))[:, None, None] * ff
        CC = CC - (gamma / lam2 ** 1.5)[:, None, None, None, None] * np.einsum("mij,mkl->mijkl", ff, ff)
    return S, CC


# ----------------------------------------------------------------------------
# element tangents / internal forces / loads (Gauss quadrature, isoparametric)
# ----------------------------------------------------------------------------
def _elem_geometry(mesh: Mesh, elems: np.ndarray, dNq: np.ndarray):
    """For one quadrature point: dN/dX [e, npe, 3] and det J [e]."""
    Xe = mesh.coords[mesh.elem_nodes[elems]]                 # [e, npe, 3]
    Jm = np.einsum("eai,aj->eij", Xe, dNq)                   # dX/dxi
    det = np.linalg.det(Jm)
    if np.any(det <= 0):
        raise ValueError("inverted element")
    Jinv = np.linalg.inv(Jm)
    dNX = np.einsum("aj,eji->eai", dNq, Jinv)
    return dNX, det


def element_tangents(mesh: Mesh, material, u: Optional[np.ndarray] = None,
                     chunk: int = 4096, frames_fn=None) -> np.ndarray:
    """K_e[(a,i),(b,k)] = sum_q w |J| dN_a/dX_J A_iJkL dN_b/dX_L with
    A_iJkL = delta_ik S_JL + F_iI F_kK C_IJKL, for every element (float64)."""
    order = mesh.order
    pts, wts = gauss_rule(order + 1)
    _, dN = shape_functions(order, pts)
    npe = mesh.npe
    nd = 3 * npe
    out = np.zeros((mesh.n_elems, nd, nd))
    I = _eye3()

    def one_chunk(e0):
        elems = np.arange(e0, min(mesh.n_elems, e0 + chunk))
        ue = None if u is None else u[mesh.elem_nodes[elems]]   # [e, npe, 3]
        Ke = np.zeros((len(elems), npe, 3, npe, 3))
        for q in range(len(wts)):
            dNX, det = _elem_geometry(mesh, elems, dN[q])
            if ue is None:
                F = np.broadcast_to(I, (len(elems), 3, 3)).copy()
            else:
                F = I + np.einsum("eai,eaJ->eiJ", ue, dNX)
            mat = material
            if frames_fn is not None:
                mat = dict(material)
                mat["frames"] = frames_fn(elems, q)
            S, CC = _stress_tangent(mat, F)
            A = (np.einsum("ik,mJL->miJkL", I, S)
                 + np.einsum("miI,mkK,mIJKL->miJkL", F, F, CC, optimize=True))
            wdet = wts[q] * det
            m = len(elems)
            # B[e,a,(i,k,L)] = sum_J dN_a/dX_J A_iJkL, then K[e,(a,i,k),b] = sum_L B dN_b/dX_L
            A2 = np.ascontiguousarray(A.transpose(0, 2, 1, 3, 4)).reshape(m, 3, 27)
            Bm = np.matmul(dNX, A2).reshape(m, npe * 9, 3)
            Kq = np.matmul(Bm, dNX.transpose(0, 2, 1)).reshape(m, npe, 3, 3, npe)
            Ke += wdet[:, None, None, None, None] * Kq.transpose(0, 1, 2, 4, 3)
        out[elems] = Ke.reshape(len(elems), nd, nd)

    # chunks are independent (each writes its own elements): run them on a thread pool, the
    # arithmetic of every chunk is the same as in a sequential loop
    starts = list(range(0, mesh.n_elems, chunk))
    workers = min(len(starts), max(1, min(16, os.cpu_count() or 1)))
    if workers > 1:
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            list(ex.map(one_chunk, starts))
    else:
        for e0 in starts:
            one_chunk(e0)
    return out


def element_internal_forces(mesh: Mesh, material, u: np.ndarray, frames_fn=None) -> np.ndarray:
    """f_e[(a,i)] = sum_q w |J| P_iJ dN_a/dX_J with P = F S (used to check tangents)."""
    order = mesh.order
    pts, wts = gauss_rule(order + 1)
    _, dN = shape_functions(order, pts)
    elems = np.arange(mesh.n_elems)
    ue = u[mesh.elem_nodes]
    fe = np.zeros((mesh.n_elems, mesh.npe, 3))
    for q in range(len(wts)):
        dNX, det = _elem_geometry(mesh, elems, dN[q])
        F = np.eye(3) + np.einsum("eai,eaJ->eiJ", ue, dNX)
        mat = material
        if frames_fn is not None:
            mat = dict(material)
            mat["frames"] = frames_fn(elems, q)
        S, _ = _stress_tangent(mat, F)
        P = np.einsum("miI,mIJ->miJ", F, S)
        fe += (wts[q] * det)[:, None, None] * np.einsum("eiJ,eaJ->eai", P, dNX)
    return fe.reshape(mesh.n_elems, 3 * mesh.npe)


def boundary_faces(mesh: Mesh, tag_bit: int) -> np.ndarray:
    """Element faces on a tagged surface: rows (element, d, side) of every face xi_d = side
    (reference cube [0,1]^3) whose nodes all carry tag_bit, sorted."""
    p1 = mesh.order + 1
    out = []
    for d in range(3):
        for side in (0, 1):
            idx = [a + p1 * b + p1 * p1 * c for c in range(p1) for b in range(p1) for a in range(p1)
                   if (a, b, c)[d] == side * (p1 - 1)]
            on = np.all((mesh.node_tags[mesh.elem_nodes[:, idx]] & tag_bit) != 0, axis=1)
            out += [(int(e), d, side) for e in np.nonzero(on)[0]]
    return np.array(sorted(out), dtype=np.int64).reshape(-1, 3)


def boundary_terms(mesh: Mesh, faces: np.ndarray, kind: str, params, u: Optional[np.ndarray] = None):
    """Element-matrix and element-force contributions [n_el, nd, nd], [n_el, nd] of a boundary
    condition on `faces` (paper §2, boundary conditions), by the (p+1)^2 Gauss rule of each face:
    * "robin" (params a_perp, a_par): g = (N (x) N) a_perp u + (I - N (x) N) a_par u, the epicardial
      condition with the stiffness and damping terms combined into a_perp, a_par;
      force int N_a g dS, tangent int N_a N_b (a_perp N N^T + a_par (I - N N^T)) dS;
    * "pressure" (params p): g = p J F^-T N (follower pressure on the endocardium), force
      int N_a g dS, tangent int N_a p J (F^-T_iJ F^-T_kL - F^-T_iL F^-T_kJ) N_J dN_b/dX_L dS
      (not symmetric).
    N is the outward unit normal and dS the area element of the reference configuration."""
    order = mesh.order
    p1 = order + 1
    npe = mesh.npe
    nd = 3 * npe
    K = np.zeros((mesh.n_elems, nd, nd))
    f = np.zeros((mesh.n_elems, nd))
    g1, w1 = np.polynomial.legendre.leggauss(p1)
    g1, w1 = 0.5 * (g1 + 1.0), 0.5 * w1
    for e, d, side in faces:
        Xe = mesh.coords[mesh.elem_nodes[e]]
        ue = np.zeros((npe, 3)) if u is None else u[mesh.elem_nodes[e]]
        d1, d2 = (d + 1) % 3, (d + 2) % 3
        for q1 in range(p1):
            for q2 in range(p1):
                xi = np.zeros(3)
                xi[d], xi[d1], xi[d2] = float(side), g1[q1], g1[q2]
                Nq, dNq = shape_functions(order, xi[None, :])
                Nq, dNq = Nq[0], dNq[0]
                Jm = Xe.T @ dNq                                   # dX_i / dxi_j
                nvec = np.cross(Jm[:, d1], Jm[:, d2]) * (1.0 if side == 1 else -1.0) * w1[q1] * w1[q2]
                dS = np.linalg.norm(nvec)
                Nn = nvec / dS
                dNX = dNq @ np.linalg.inv(Jm)                     # dN_a / dX_L
                if kind == "robin":
                    ap, al = params
                    Bm = ap * np.outer(Nn, Nn) + al * (np.eye(3) - np.outer(Nn, Nn))
                    g = Bm @ (ue.T @ Nq)
                    f[e] += dS * np.einsum("a,i->ai", Nq, g).ravel()
                    K[e] += dS * np.einsum("a,b,ik->aibk", Nq, Nq, Bm).reshape(nd, nd)
                elif kind == "pressure":
                    (pr,) = params
                    F = np.eye(3) + ue.T @ dNX
                    J = np.linalg.det(F)
                    Fi = np.linalg.inv(F).T                       # F^-T
                    g = pr * J * Fi @ nvec
                    f[e] += np.einsum("a,i->ai", Nq, g).ravel()
                    T = pr * J * (np.einsum("iJ,kL->iJkL", Fi, Fi) - np.einsum("iL,kJ->iJkL", Fi, Fi))
                    TN = np.einsum("iJkL,J->ikL", T, nvec)
                    K[e] += np.einsum("a,ikL,bL->aibk", Nq, TN, dNX).reshape(nd, nd)
                else:
                    raise ValueError(kind)
    return K, f


def body_force_load(mesh: Mesh, force_at_nodes: np.ndarray) -> np.ndarray:
    """Consistent load b_(a,i) = sum_e sum_q w |J| N_a f_i(X_q), f interpolated from nodal
    values [n_nodes, 3]; returned as a full DOF vector [3*n_nodes]."""
    order = mesh.order
    pts, wts = gauss_rule(order + 1)
    N, dN = shape_functions(order, pts)
    elems = np.arange(mesh.n_elems)
    fnod = force_at_nodes[mesh.elem_nodes]                     # [e, npe, 3]
    fe = np.zeros((mesh.n_elems, mesh.npe, 3))
    for q in range(len(wts)):
        _, det = _elem_geometry(mesh, elems, dN[q])
        fq = np.einsum("a,eai->ei", N[q], fnod)
        fe += (wts[q] * det)[:, None, None] * N[q][None, :, None] * fq[:, None, :]
    b = np.zeros(3 * mesh.n_nodes)
    np.add.at(b, (3 * mesh.elem_nodes[:, :, None] + np.arange(3)[None, None, :]).ravel(), fe.ravel())
    return b


# ----------------------------------------------------------------------------
# complete problem instances
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """One tangent system: mesh, partition, clamps, element tangents and right-hand sides."""
    name: str
    mesh: Mesh
    elem_part: np.ndarray     # [n_el] int32
    n_sub: int
    dirichlet: np.ndarray     # [n_dir] int32 DOF ids (homogeneous)
    Ke: np.ndarray            # [n_el, 3npe, 3npe] float64
    rhs: np.ndarray           # [nrhs, 3*n_nodes] float64, zero on Dirichlet DOFs
    primal: int               # bitmask V=1, E=2, F=4
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_dofs(self) -> int:
        return 3 * self.mesh.n_nodes


def _loads(mesh: Mesh, dirichlet: np.ndarray, nrhs: int, seed: int) -> np.ndarray:
    f0 = np.zeros((mesh.n_nodes, 3))
    f0[:, 2] = -1.0
    out = [body_force_load(mesh, f0)]
    for j in range(1, nrhs):
        fj = smooth_field(mesh.coords, seed + j, 1.0)
        out.append(body_force_load(mesh, fj))
    rhs = np.stack(out)
    rhs[:, dirichlet] = 0.0
    return rhs


def linear_box(n: int = 8, block: int = 4, order: int = 1, nrhs: int = 1, E: float = 1.0,
               nu: float = 0.3, primal: int = 1, seed: int = 1, name: str = "linear_box") -> Problem:
    """Linear elasticity on the unit cube, x=0 clamped, body force (0,0,-1)."""
    mesh = box_mesh(n, n, n, order)
    part, nsub = block_partition(mesh, block)
    dirichlet = clamp_dofs(mesh, 1)
    Ke = element_tangents(mesh, linear_elastic(E, nu))
    rhs = _loads(mesh, dirichlet, nrhs, seed)
    return Problem(name, mesh, part, nsub, dirichlet, Ke, rhs, primal,
                   {"material": "linear", "E": E, "nu": nu, "n": n, "block": block, "order": order})


def neo_hookean_box(n: int = 32, block: int = 4, order: int = 1, nrhs: int = 4, mu: float = 1.0,
                    kappa: float = 50.0, amplitude: float = 0.05, field_seed: int = 0,
                    rhs_seed: int = 1, primal: int = 3, name: str = "neo_hookean_box",
                    cluster: int = 1) -> Problem:
    """Compressible neo-Hookean tangent linearised at a seeded isochoric 8-mode field."""
    mesh = box_mesh(n, n, n, order)
    part, nsub = block_partition(mesh, block, cluster)
    dirichlet = clamp_dofs(mesh, 1)
    u = isochoric_field(mesh.coords, field_seed, amplitude)
    Ke = element_tangents(mesh, neo_hookean(mu, kappa), u)
    rhs = _loads(mesh, dirichlet, nrhs, rhs_seed)
    return Problem(name, mesh, part, nsub, dirichlet, Ke, rhs, primal,
                   {"material": "neo_hookean", "mu": mu, "kappa": kappa, "n": n, "block": block,
                    "order": order, "amplitude": amplitude, "field_seed": field_seed})


def newton_tangents(mesh: Mesh, material, u0: np.ndarray, du: np.ndarray, n_steps: int) -> np.ndarray:
    """Element tangents of n_steps Newton iterates u_k = u0 + (k / n_steps) du, k = 0..n_steps-1
    ([n_steps, n_el, 3npe, 3npe]): the sequence of tangent systems one request of the serving
    loop solves, its factors computed at u0 and reused (lagged) for the later steps."""
    return np.stack([element_tangents(mesh, material, u0 + (k / n_steps) * du) for k in range(n_steps)])


def _nh_basis(mesh: Mesh, u: np.ndarray):
    """The compressible neo-Hookean tangent is linear in (mu, lambda) at a fixed deformation:
    K = mu K_mu + lambda K_lambda. Returns (K_mu, K_lambda)."""
    return (element_tangents(mesh, {"kind": "neo_hookean", "mu": 1.0, "lam": 0.0}, u),
            element_tangents(mesh, {"kind": "neo_hookean", "mu": 0.0, "lam": 1.0}, u))


def batched_instances(n_inst: int = 64, seed: int = 100, dof_min: float = 5e3, dof_max: float = 2e5,
                      nrhs: int = 4, amplitude: float = 0.02, progress=None) -> list:
    """Independent neo-Hookean box tangents solved together: element type Q1 or Q2 with
    probability 1/2, DOF count log-uniform in [dof_min, dof_max] (Q1 boxes n^3 with n a multiple
    of 4 and subdomains of 4^3 elements, Q2 boxes with n a multiple of 2 and subdomains of 2^3,
    both 375 DOFs per subdomain, numbered in 2x2x2 clusters), (mu, kappa) = (1, 50) times
    independent U[0.5, 2] factors,
    x = 0 clamped, primal V+E, nrhs right-hand sides. Instances of the same mesh share the
    linearisation field (seed per mesh) and differ by their material factors."""
    rng = np.random.default_rng(seed)
    cache = {}
    out = []
    for i in range(n_inst):
        q2 = rng.random() < 0.5
        N = float(np.exp(rng.uniform(np.log(dof_min), np.log(dof_max))))
        side = (N / 3.0) ** (1.0 / 3.0)                     # nodes per edge
        if q2:
            ne = max(2, 2 * int(round((side - 1.0) / 2.0 / 2.0)))
            order, block = 2, 2
        else:
            ne = max(4, 4 * int(round((side - 1.0) / 4.0)))
            order, block = 1, 4
        fmu, fk = rng.uniform(0.5, 2.0, size=2)
        key = (order, ne)
        if key not in cache:
            mesh = box_mesh(ne, ne, ne, order)
            part, nsub = block_partition(mesh, block, cluster=2)
            dirichlet = clamp_dofs(mesh, 1)
            u = isochoric_field(mesh.coords, seed + len(cache), amplitude)
            Kmu, Klam = _nh_basis(mesh, u)
            rhs = _loads(mesh, dirichlet, nrhs, seed + 1000 + len(cache))
            cache[key] = (mesh, part, nsub, dirichlet, Kmu, Klam, rhs)
            if progress is not None:
                progress(f"mesh Q{order} {ne}^3: {3 * mesh.n_nodes} DOFs")
        mesh, part, nsub, dirichlet, Kmu, Klam, rhs = cache[key]
        mu, kappa = fmu, 50.0 * fk
        lam = kappa - 2.0 * mu / 3.0
        out.append(Problem(f"inst{i}", mesh, part, nsub, dirichlet, mu * Kmu + lam * Klam, rhs, 3,
                           {"order": order, "n": ne, "mu": mu, "kappa": kappa}))
    return out


# ----------------------------------------------------------------------------
# ventricle-like shell: mapped truncated half-ellipsoid, fibre frames, RCB partition
# ----------------------------------------------------------------------------
VENT_BASE, VENT_ENDO, VENT_EPI, VENT_APEX = 1, 2, 4, 8


def ventricle_mesh(n_t: int, n_theta: int, n_phi: int, order: int = 2, wall: float = 0.3,
                   a_endo: float = 1.0, c_endo: float = 2.5, phi0_deg: float = 10.0):
    """Thick-walled truncated half-ellipsoid (endocardial semi-axes a, a, c; wall thickness
    `wall` along each axis), mapped isoparametrically from the parametric box
    (t, theta, phi) in [0,1] x [0, 2 pi) x [phi0, pi/2]:
        X = ((a + wall t) sin(phi) cos(theta), (a + wall t) sin(phi) sin(theta), -(c + wall t) cos(phi)).
    theta is periodic; the base is the plane z = 0 (phi = pi/2), a small apical opening at
    phi0 avoids degenerate elements. Node tags: base, endocardium (t = 0), epicardium
    (t = 1), apex rim. Returns the mesh and the parametric node coordinates
    (t, theta / 2 pi, meridian fraction)."""
    p = order
    Nt, Nth, Nph = p * n_t + 1, p * n_theta, p * n_phi + 1
    phi0 = np.deg2rad(phi0_deg)
    it, ith, iph = np.meshgrid(np.arange(Nt), np.arange(Nth), np.arange(Nph), indexing="ij")
    it, ith, iph = it.ravel(order="F"), ith.ravel(order="F"), iph.ravel(order="F")
    # node id = it + Nt (ith + Nth iph)
    order_ids = it + Nt * (ith + Nth * iph)
    t = np.empty(Nt * Nth * Nph)
    th = np.empty_like(t)
    ph = np.empty_like(t)
    t[order_ids] = it / (Nt - 1)
    th[order_ids] = 2.0 * np.pi * ith / Nth
    ph[order_ids] = phi0 + (0.5 * np.pi - phi0) * iph / (Nph - 1)
    r_xy = a_endo + wall * t
    r_z = c_endo + wall * t
    coords = np.stack([r_xy * np.sin(ph) * np.cos(th), r_xy * np.sin(ph) * np.sin(th), -r_z * np.cos(ph)], axis=1)
    IT = np.empty(Nt * Nth * Nph, dtype=np.int64)
    IPH = np.empty_like(IT)
    IT[order_ids] = it
    IPH[order_ids] = iph
    tags = ((IPH == Nph - 1) * VENT_BASE | (IT == 0) * VENT_ENDO | (IT == Nt - 1) * VENT_EPI
            | (IPH == 0) * VENT_APEX).astype(np.uint32)
    ep, eth, et = np.meshgrid(np.arange(n_phi), np.arange(n_theta), np.arange(n_t), indexing="ij")
    et, eth, ep = et.ravel(), eth.ravel(), ep.ravel()
    p1 = p + 1
    en = np.empty((n_t * n_theta * n_phi, p1 ** 3), dtype=np.int64)
    for c in range(p1):
        for b in range(p1):
            for a in range(p1):
                en[:, a + p1 * b + p1 * p1 * c] = ((p * et + a) + Nt * (((p * eth + b) % Nth) + Nth * (p * ep + c)))
    mesh = Mesh(coords=coords, elem_nodes=en.astype(np.int32), order=order, node_tags=tags,
                shape=(n_t, n_theta, n_phi))
    param = np.stack([t, th / (2.0 * np.pi), (ph - phi0) / (0.5 * np.pi - phi0)], axis=1)
    return mesh, param


def ventricle_elem_param(mesh: Mesh) -> np.ndarray:
    """Parametric centroid (t, theta / 2 pi, meridian fraction) of every element, from the
    structured element numbering (element = et + n_t (eth + n_theta ep)), so that elements
    on the periodic seam are not averaged across it."""
    n_t, n_th, n_ph = mesh.shape
    e = np.arange(mesh.n_elems)
    et, eth, ep = e % n_t, (e // n_t) % n_th, e // (n_t * n_th)
    return np.stack([(et + 0.5) / n_t, (eth + 0.5) / n_th, (ep + 0.5) / n_ph], axis=1)


def ventricle_frames(mesh: Mesh, param: np.ndarray, helix_endo_deg: float = 60.0, helix_epi_deg: float = -60.0):
    """Per-element fibre frames (rows f, s, n) at the element centroid: helix angle linear in
    the transmural coordinate from helix_endo at t = 0 to helix_epi at t = 1; f = cos(a) e_theta
    + sin(a) e_phi, s the transmural direction made orthogonal to f, n = f x s."""
    pc = ventricle_elem_param(mesh)
    Xc = mesh.coords[mesh.elem_nodes].mean(axis=1)
    theta = np.arctan2(Xc[:, 1], Xc[:, 0])
    e_th = np.stack([-np.sin(theta), np.cos(theta), np.zeros_like(theta)], axis=1)
    # transmural and meridian directions from the element's own geometry
    npe = mesh.npe
    p1 = mesh.order + 1
    Xe = mesh.coords[mesh.elem_nodes]
    a_hi = [i for i in range(npe) if i % p1 == p1 - 1]
    a_lo = [i for i in range(npe) if i % p1 == 0]
    c_hi = [i for i in range(npe) if i // (p1 * p1) == p1 - 1]
    c_lo = [i for i in range(npe) if i // (p1 * p1) == 0]
    e_t = Xe[:, a_hi].mean(axis=1) - Xe[:, a_lo].mean(axis=1)
    e_ph = Xe[:, c_hi].mean(axis=1) - Xe[:, c_lo].mean(axis=1)
    e_ph -= np.sum(e_ph * e_th, axis=1, keepdims=True) * e_th
    e_ph /= np.linalg.norm(e_ph, axis=1, keepdims=True)
    alpha = np.deg2rad(helix_endo_deg + (helix_epi_deg - helix_endo_deg) * pc[:, 0])
    f = np.cos(alpha)[:, None] * e_th + np.sin(alpha)[:, None] * e_ph
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    s = e_t - np.sum(e_t * f, axis=1, keepdims=True) * f
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    n = np.cross(f, s)
    return np.stack([f, s, n], axis=1)


def rcb_partition(mesh: Mesh, param: np.ndarray, target_dofs: int, seed: int = 3,
                  scale=(0.3, 7.2, 2.5)) -> tuple[np.ndarray, int]:
    """Recursive coordinate bisection of the element centroids in scaled parametric
    coordinates (transmural, circumferential, meridian extents): the longest extent of a part
    is split at a seeded quantile q ~ U[0.2, 0.8] (elements with equal coordinates on the
    same side, so every part is a box of the structured parameter grid) until a part has at
    most target_dofs DOFs (3 x its distinct nodes). Parts are numbered in recursion order
    (neighbours get neighbouring ids). Returns (elem_part, n_parts)."""
    rng = np.random.default_rng(seed)
    cen = ventricle_elem_param(mesh) * np.asarray(scale)[None, :]
    part = np.zeros(mesh.n_elems, dtype=np.int32)
    stack = [np.arange(mesh.n_elems)]
    leaves = []
    while stack:
        el = stack.pop()
        ndof = 3 * len(np.unique(mesh.elem_nodes[el]))
        if ndof <= target_dofs or len(el) < 2:
            leaves.append(el)
            continue
        ext = cen[el].max(axis=0) - cen[el].min(axis=0)
        d = int(np.argmax(ext))
        q = rng.uniform(0.2, 0.8)
        key = cen[el, d]
        cut = np.quantile(key, q)
        if cut >= key.max():                     # all elements with equal coordinates stay together
            cut = key[key < key.max()].max() if np.any(key < key.max()) else cut
        lo, hi = el[key <= cut], el[key > cut]
        if len(lo) == 0 or len(hi) == 0:
            leaves.append(el)
            continue
        stack.append(hi)
        stack.append(lo)
    for i, el in enumerate(leaves):
        part[el] = i
    return part, len(leaves)


def ventricle(n_t: int = 4, n_theta: int = 96, n_phi: int = 96, order: int = 2, target_dofs: int = 6000,
              nrhs: int = 1, amplitude: float = 0.015, field_seed: int = 2, part_seed: int = 3,
              rhs_seed: int = 5, primal: int = 7, name: str = "ventricle") -> Problem:
    """Guccione tangent (C = 0.88, bf = 8, bt = bfs = 2, B = 50) on the ventricle-like shell,
    fibres rotating from +60 to -60 degrees transmurally, linearised at the seeded isochoric
    8-mode field of the physical coordinates (max |u| = amplitude = 0.05 x wall thickness),
    base clamped, RCB partition into parts of at most target_dofs DOFs."""
    mesh, param = ventricle_mesh(n_t, n_theta, n_phi, order)
    part, nsub = rcb_partition(mesh, param, target_dofs, part_seed)
    dirichlet = clamp_dofs(mesh, VENT_BASE)
    u = isochoric_field(mesh.coords, field_seed, amplitude)
    frames = ventricle_frames(mesh, param)
    Ke = element_tangents(mesh, guccione(), u, frames_fn=lambda elems, q: frames[elems])
    rhs = _loads(mesh, dirichlet, nrhs, rhs_seed)
    return Problem(name, mesh, part, nsub, dirichlet, Ke, rhs, primal,
                   {"material": "guccione", "n": (n_t, n_theta, n_phi), "order": order,
                    "target_dofs": target_dofs, "amplitude": amplitude})


def config_small() -> Problem:
    """8^3 Q1 unit cube, linear elasticity E=1 nu=0.3, 2x2x2 subdomains of 4^3, primal V."""
    return linear_box(8, 4, 1, nrhs=1, primal=1, name="linear_8cube_2x2x2_V")


def config_nh32(nrhs: int = 4) -> Problem:
    """32^3 Q1 neo-Hookean (mu=1, kappa=50) at the 8-mode field, 512 subdomains of 4^3, primal VE."""
    return neo_hookean_box(32, 4, 1, nrhs=nrhs, primal=3, name="neo_hookean_32cube_512sub_VE")


def ventricle_newton(target_dofs: float, n_steps: int, seed: int, part_dofs: int = 2000, amplitude: float = 0.015):
    """One serving request on the ventricle-like shell: the mesh (two Q2 elements through the
    wall, n_theta = n_phi chosen for about target_dofs DOFs), an RCB partition into parts of at
    most part_dofs DOFs, and the Guccione element tangents of n_steps Newton iterates
    u_k = u0 + (k / n_steps) du (isochoric fields of the physical coordinates, seeds seed and
    seed + 1). Returns (mesh, part, n_sub, dirichlet, Ks [n_steps, n_el, 81, 81])."""
    m = max(6, int(round(np.sqrt(target_dofs / 60.0))))
    mesh, param = ventricle_mesh(2, m, m, 2)
    part, nsub = rcb_partition(mesh, param, part_dofs, seed)
    dirichlet = clamp_dofs(mesh, VENT_BASE)
    frames = ventricle_frames(mesh, param)
    u0 = isochoric_field(mesh.coords, seed, amplitude)
    du = isochoric_field(mesh.coords, seed + 1, 0.5 * amplitude)
    Ks = np.stack([element_tangents(mesh, guccione(), u0 + (k / n_steps) * du,
                                    frames_fn=lambda elems, q: frames[elems]) for k in range(n_steps)])
    return mesh, part, nsub, dirichlet, Ks
