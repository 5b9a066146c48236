"""Oracle: two- and three-level BDDC for unassembled finite-element tangents.

Follows paper §3.2 ("BDDC preconditioner"):

* non-overlapping decomposition Omega = U Omega_i, interface
  Gamma = U dOmega_i minus dOmega, local spaces V^(i) = V_I^(i) (+) V_Gamma^(i);
* primal degrees of freedom associated with subdomain vertices, edges and/or
  faces (edge and face primals are averages, §3.2 and §6.2);
* counting-function scaling delta_i^dagger = 1 / #{subdomains sharing x}, or the
  deluxe scaling the paper names as the more robust option (§3.2, remark after
  the counting function; ``scaling="deluxe"``): per glob g and subdomain i,
  D_g^(i) = (sum_j S_g^(j))^-1 S_g^(i) with S_g^(j) the glob block of subdomain
  j's interface Schur complement; the extension averages the local interface
  values with these weights (the S-weighted mean), the restriction applies
  their transposes;
* the exact block factorisation of A^-1 through the interface Schur complement
  S_Gamma, in which BDDC replaces S_Gamma^-1 by
  M^-1_BDDC = R_{D,Gamma}^T S~_Gamma^-1 R_{D,Gamma};
* S~_Gamma^-1 = local constrained problems + Phi S_PiPi^-1 Phi^T, with Phi the
  minimum-energy extension of the primal constraints (the columns of the
  coarse basis) and S_PiPi = sum_i R_Pi^T Phi_i^T A^(i) Phi_i R_Pi;
* multilevel BDDC: the coarse problem is itself approximated by one BDDC
  application (§3.2 last paragraph; §7, coarse problem on a group of 8);
* near-null-space primals (§4, rigid motions given to BDDC as extra primal
  degrees of freedom): on every primal edge and face the constraint rows span
  the six rigid motions restricted to the glob (``nnsp=True``);
* the non-symmetric formulation (§8, realistic simulation: the base pressure
  breaks the symmetry of the tangent and BDDC is told to use its non-symmetric
  form): a left coarse basis Psi from the transposed constrained problems
  N_i^T [Psi_i; Lambda'_i] = [0; I], coarse matrix S_PiPi = sum Psi^T A Phi and
  coarse right-hand side Psi^T R_D r, so that the preconditioner of A^T is the
  transpose of the preconditioner of A.

The primal constraints are enforced with Lagrange multipliers in the local
problems (the constrained Neumann matrices N_i = [A^(i) C_i^T; C_i 0]); for
primal sets made of single DOFs this is the same operator as the paper's
explicit-primal formula (checked by a test). All arithmetic is float64.

Readings of the paper used here (the paper is silent on them):
* glob classification: key N'(x) = {subdomains containing node x} united
  with the node's boundary-surface tags; each key class is split into
  element-connected components; a one-node component is a vertex, otherwise
  |N'| >= 3 makes an edge and |N'| = 2 a face;
* an edge/face constraint is the plain mean of one displacement component
  over the glob's nodes; a vertex constraint selects one component;
* near-null-space rows (the paper names the option, not the construction): the
  candidates are the translations along x, y, z, then the rotations about the
  x, y, z axes through the centroid of the glob's nodes, restricted to the
  glob's free DOFs; they are orthonormalised in that order by modified
  Gram-Schmidt with one re-orthogonalisation pass, and a candidate whose norm
  after projection is at most 1e-8 of its norm before is dropped (a straight
  edge keeps 5 rows, a planar face 6); vertices keep their component rows;
* vertices are weighted by delta^dagger like every interface DOF (primal
  values are single-valued, so this equals the paper's unweighted R_GammaPi);
* clamped DOFs are eliminated from every matrix;
* three levels: the level-2 "elements" are the fine subdomains with matrices
  Phi_i^T A^(i) Phi_i, the level-2 "nodes" are the fine primal globs (a coarse
  DOF is a (glob, component) pair), fine subdomain i belongs to level-2
  subdomain i // group, and the level-2 globs follow the same rule with the
  fine glob's boundary tags in the key.

Test infrastructure only; see the package docstring.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

from . import fem

VERTEX, EDGE, FACE = 1, 2, 4
NNSP_DROP = 1e-8     # relative norm below which a rigid-motion candidate is dependent


def rigid_motion_rows(X: np.ndarray, free: np.ndarray) -> np.ndarray:
    """Orthonormal rows spanning the rigid motions of the nodes X (nn x 3) restricted to the free
    entries (``free``: nn x 3 mask, entries ordered node-major), candidates in the order
    translations x, y, z, rotations about x, y, z through the nodes' centroid (§4)."""
    d = X - X.mean(axis=0)
    cand = np.zeros((6, X.shape[0], 3))
    for a in range(3):
        cand[a, :, a] = 1.0                              # translation along axis a
        w = np.zeros(3)
        w[a] = 1.0
        cand[3 + a] = np.cross(w, d)                     # rotation about axis a: w x (x - centroid)
    Q = []
    for v in cand.reshape(6, -1)[:, free.ravel()]:
        n0 = np.linalg.norm(v)
        if n0 == 0.0:
            continue
        for _ in range(2):
            for q in Q:
                v = v - (q @ v) * q
        n1 = np.linalg.norm(v)
        if n1 <= NNSP_DROP * n0:
            continue
        Q.append(v / n1)
    return np.array(Q) if Q else np.zeros((0, int(free.sum())))


def classify_globs(n_items: int, item_subs: list, item_tags: np.ndarray, is_interface: np.ndarray,
                   adjacency_pairs: np.ndarray, all_vertices: bool = False):
    """Split interface items (nodes, or fine globs at level 2) into globs.

    Items with equal key (subdomain set, boundary tags) that are connected through
    ``adjacency_pairs`` [k, 2] form one glob. Returns a list of (kind, items, subs),
    sorted by smallest item id."""
    key_of = {}
    key_id = -np.ones(n_items, dtype=np.int64)
    for it in np.nonzero(is_interface)[0]:
        key_id[it] = key_of.setdefault((item_subs[it], int(item_tags[it])), len(key_of))
    if all_vertices:
        comp = np.arange(n_items)
    else:
        a, b = adjacency_pairs[:, 0], adjacency_pairs[:, 1]
        same = (key_id[a] >= 0) & (key_id[a] == key_id[b])
        g = sp.coo_matrix((np.ones(int(same.sum())), (a[same], b[same])), shape=(n_items, n_items))
        _, comp = csgraph.connected_components(g, directed=False)
    members = {}
    for it in np.nonzero(is_interface)[0]:
        members.setdefault(int(comp[it]), []).append(int(it))
    globs = []
    for items in members.values():
        items = np.array(sorted(items))
        subs = item_subs[items[0]]
        nprime = len(subs) + bin(int(item_tags[items[0]])).count("1")
        if len(items) == 1 or all_vertices:
            kind = VERTEX
        elif nprime >= 3:
            kind = EDGE
        else:
            kind = FACE
        globs.append((kind, items, subs))
    globs.sort(key=lambda t: t[1][0])
    return globs


@dataclasses.dataclass
class LocalSpace:
    dofs: np.ndarray          # global indices (level's index space), interior first, then interface
    n_interior: int
    weights: np.ndarray       # counting-function weights on the interface entries
    coarse: np.ndarray        # global coarse ids of the local primal constraints
    C: np.ndarray             # [n_c, n_i] constraint rows
    iglob: Optional[np.ndarray] = None   # glob id of each interface entry (deluxe scaling)


class Decomposition:
    """Index sets of paper §3.2 on a mesh: interior / interface, globs, primal constraints,
    weights. The level index space is the free-DOF vector (positions in ``free``)."""

    def __init__(self, elem_nodes, n_nodes, elem_part, n_sub, dirichlet, node_tags=None,
                 primal: int = VERTEX, all_interface_vertices: bool = False, coords=None, nnsp: bool = False):
        elem_nodes = np.asarray(elem_nodes, dtype=np.int64)
        elem_part = np.asarray(elem_part, dtype=np.int64)
        self.n_nodes = int(n_nodes)
        self.n_dofs = 3 * self.n_nodes
        self.n_sub = int(n_sub)
        self.primal = primal
        self.nnsp = nnsp
        if nnsp and coords is None:
            raise ValueError("near-null-space primals need the node coordinates")
        free_mask = np.ones(self.n_dofs, dtype=bool)
        free_mask[np.asarray(dirichlet, dtype=np.int64)] = False
        self.free_mask = free_mask
        self.free = np.nonzero(free_mask)[0]
        self.free_pos = -np.ones(self.n_dofs, dtype=np.int64)
        self.free_pos[self.free] = np.arange(len(self.free))
        tags = np.zeros(self.n_nodes, dtype=np.int64) if node_tags is None else np.asarray(node_tags, np.int64)
        self.node_tags = tags

        node_subs = [set() for _ in range(self.n_nodes)]
        for e in range(elem_nodes.shape[0]):
            for nd in elem_nodes[e]:
                node_subs[nd].add(int(elem_part[e]))
        self.node_subs = [tuple(sorted(s)) for s in node_subs]
        has_free = free_mask.reshape(-1, 3).any(axis=1)
        self.interface_node = np.array([len(s) >= 2 for s in self.node_subs]) & has_free

        npe = elem_nodes.shape[1]
        ia, ib = np.triu_indices(npe, 1)
        pairs = np.stack([elem_nodes[:, ia].ravel(), elem_nodes[:, ib].ravel()], axis=1)
        self.globs = classify_globs(self.n_nodes, self.node_subs, tags, self.interface_node, pairs,
                                    all_interface_vertices)
        self.node_glob = -np.ones(self.n_nodes, dtype=np.int64)
        for gi, (_, nodes, _) in enumerate(self.globs):
            self.node_glob[nodes] = gi

        sel = (VERTEX | EDGE | FACE) if all_interface_vertices else primal
        self.coarse = []                       # (glob, component) per coarse DOF; (glob, row) for nnsp globs
        self.glob_rows = {}                    # nnsp glob -> (its free DOFs, orthonormal rows over them)
        for gi, (kind, nodes, _) in enumerate(self.globs):
            if not kind & sel:
                continue
            if nnsp and kind != VERTEX:
                fm = free_mask[(3 * nodes[:, None] + np.arange(3)[None, :])]
                B = rigid_motion_rows(np.asarray(coords, dtype=np.float64)[nodes], fm)
                dd = (3 * nodes[:, None] + np.arange(3)[None, :])[fm]
                self.glob_rows[gi] = (dd, B)
                self.coarse.extend((gi, k) for k in range(B.shape[0]))
                continue
            for c in range(3):
                if free_mask[3 * nodes + c].any():
                    self.coarse.append((gi, c))
        self.n_coarse = len(self.coarse)

        sub_coarse = [[] for _ in range(self.n_sub)]
        for cid, (gi, c) in enumerate(self.coarse):
            for i in self.globs[gi][2]:
                sub_coarse[i].append(cid)
        self.subdomains = []
        self.sub_elems = []
        for i in range(self.n_sub):
            elems = np.nonzero(elem_part == i)[0]
            nodes = np.unique(elem_nodes[elems])
            dofs = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
            dofs = dofs[free_mask[dofs]]
            is_if = self.interface_node[dofs // 3]
            local = np.concatenate([dofs[~is_if], dofs[is_if]])
            w = np.array([1.0 / len(self.node_subs[d // 3]) for d in dofs[is_if]])
            pos = {int(d): k for k, d in enumerate(local)}
            rows, cids = [], []
            for cid in sub_coarse[i]:
                gi, c = self.coarse[cid]
                row = np.zeros(len(local))
                if gi in self.glob_rows:               # row c of the glob's rigid-motion basis
                    dd, B = self.glob_rows[gi]
                    for d, b in zip(dd, B[c]):
                        row[pos[int(d)]] = b
                else:                                  # mean of component c over the glob
                    gnodes = self.globs[gi][1]
                    dd = 3 * gnodes + c
                    dd = dd[free_mask[dd]]
                    for d in dd:
                        row[pos[int(d)]] = 1.0 / len(dd)
                rows.append(row)
                cids.append(cid)
            C = np.array(rows) if rows else np.zeros((0, len(local)))
            self.subdomains.append(LocalSpace(self.free_pos[local], int((~is_if).sum()), w,
                                              np.array(cids, dtype=np.int64), C,
                                              self.node_glob[dofs[is_if] // 3]))
            self.sub_elems.append(elems)
        self.local_dofs = [self.free[s.dofs] for s in self.subdomains]   # global DOF ids

    def glob_counts(self):
        k = np.array([g[0] for g in self.globs])
        return int((k == VERTEX).sum()), int((k == EDGE).sum()), int((k == FACE).sum())


class Level:
    """One BDDC level on an index space of size n with assembled operator A (n x n).

    ``spaces[i]`` gives subdomain i's local index set, interior-first; ``Ks[i]`` its
    unassembled matrix A^(i) on that set. ``coarse_solver`` (optional) replaces the exact
    coarse solve (multilevel BDDC)."""

    def __init__(self, A, spaces: list, Ks: list, n_coarse: int,
                 coarse_solver: Optional[Callable] = None, build_coarse: bool = True, nonsymmetric: bool = False,
                 scaling: str = "counting"):
        if scaling not in ("counting", "deluxe"):
            raise ValueError("scaling is 'counting' or 'deluxe'")
        if scaling == "deluxe" and nonsymmetric:
            raise NotImplementedError("deluxe scaling of the non-symmetric formulation")
        self.A = A
        self.spaces = spaces
        self.n = A.shape[0]
        self.n_coarse = n_coarse
        self.loc = []
        Kc = np.zeros((n_coarse, n_coarse))
        interior = []
        for sp_, Ki in zip(spaces, Ks):
            nI = sp_.n_interior
            nc = sp_.C.shape[0]
            ni = len(sp_.dofs)
            KII_lu = sla.lu_factor(Ki[:nI, :nI]) if nI > 0 else None
            Ni = np.block([[Ki, sp_.C.T], [sp_.C, np.zeros((nc, nc))]])
            N_lu = sla.lu_factor(Ni)
            rhs = np.zeros((ni + nc, nc))
            rhs[ni:, :] = np.eye(nc)
            sol = sla.lu_solve(N_lu, rhs)                      # N_i [Phi_i; Lambda_i] = [0; I]
            Phi, Lam = sol[:ni], sol[ni:]
            # left basis: N_i^T [Psi_i; Lambda'_i] = [0; I] (non-symmetric form), else Psi = Phi
            Psi = sla.lu_solve(N_lu, rhs, trans=1)[:ni] if nonsymmetric else Phi
            Kci = Psi.T @ Ki @ Phi                              # Psi_i^T A^(i) Phi_i
            Kc[np.ix_(sp_.coarse, sp_.coarse)] += Kci
            self.loc.append(dict(K=Ki, KII_lu=KII_lu, N_lu=N_lu, Phi=Phi, Psi=Psi, Lam=Lam, Kc=Kci))
            interior.append(sp_.dofs[:nI])
        self.Kc = Kc
        # interface weights: R_D restricts with D_i^T and R_D^T extends with D_i
        self.D = [np.diag(sp_.weights) for sp_ in spaces] if scaling == "counting" else deluxe_weights(spaces, Ks)
        self.coarse_solver = coarse_solver
        self.Kc_lu = sla.lu_factor(Kc) if (n_coarse and coarse_solver is None and build_coarse) else None
        I = np.sort(np.concatenate(interior)) if interior else np.zeros(0, np.int64)
        is_if = np.ones(self.n, dtype=bool)
        is_if[I] = False
        self.I = I
        self.G = np.nonzero(is_if)[0]
        A_csr = sp.csr_matrix(A)
        self.A_GI = A_csr[self.G][:, self.I]
        self.A_IG = A_csr[self.I][:, self.G]

    def interior_solve(self, v: np.ndarray) -> np.ndarray:
        """A_II^-1 v on the level's interior entries (block diagonal by subdomain);
        ``v`` and the result live on the full level index space."""
        out = np.zeros(self.n)
        for sp_, L in zip(self.spaces, self.loc):
            nI = sp_.n_interior
            if nI:
                d = sp_.dofs[:nI]
                out[d] = sla.lu_solve(L["KII_lu"], v[d])
        return out

    def coarse_solve(self, gc: np.ndarray) -> np.ndarray:
        if self.coarse_solver is not None:
            return self.coarse_solver(gc)
        return sla.lu_solve(self.Kc_lu, gc)

    def interface_precond(self, r: np.ndarray) -> np.ndarray:
        """M^-1_BDDC r on the interface entries of ``r`` (full level vector in and out)."""
        gc = np.zeros(self.n_coarse)
        ws = []
        for sp_, L, D in zip(self.spaces, self.loc, self.D):
            nI, ni, nc = sp_.n_interior, len(sp_.dofs), sp_.C.shape[0]
            ri = np.zeros(ni)
            ri[nI:] = D.T @ r[sp_.dofs[nI:]]                      # R_D restriction
            sol = sla.lu_solve(L["N_lu"], np.concatenate([ri, np.zeros(nc)]))
            ws.append(sol[:ni])                                   # constrained local solve
            gc[sp_.coarse] += L["Psi"].T @ ri                     # Psi^T R_D r (Psi = Phi: symmetric form)
        uc = self.coarse_solve(gc) if self.n_coarse else gc
        z = np.zeros(self.n)
        for sp_, L, w, D in zip(self.spaces, self.loc, ws, self.D):
            nI = sp_.n_interior
            w = w + L["Phi"] @ uc[sp_.coarse]
            np.add.at(z, sp_.dofs[nI:], D @ w[nI:])               # R_D^T
        return z

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = [I -A_II^-1 A_IG; 0 I] diag(A_II^-1, M^-1_BDDC) [I 0; -A_GI A_II^-1 I] r
        (the block factorisation of A^-1 in §3.2 with S_Gamma^-1 replaced by BDDC)."""
        u0 = self.interior_solve(r)
        g = np.zeros(self.n)
        g[self.G] = r[self.G] - self.A_GI @ u0[self.I]
        zG = self.interface_precond(g)
        v = np.zeros(self.n)
        v[self.I] = r[self.I] - self.A_IG @ zG[self.G]
        z = self.interior_solve(v)
        z[self.G] = zG[self.G]
        return z


def deluxe_weights(spaces: list, Ks: list) -> list:
    """Deluxe scaling (§3.2 remark): per subdomain the block-diagonal matrix D_i on its interface
    entries with blocks D_g^(i) = (sum_j S_g^(j))^-1 S_g^(i), S_g^(j) the rows and columns of glob g
    in subdomain j's interface Schur complement S^(j) = A_GG - A_GI A_II^-1 A_IG. The entries of a
    glob appear in the same (ascending DOF) order in every subdomain that shares it."""
    S = []
    for sp_, K in zip(spaces, Ks):
        nI = sp_.n_interior
        S.append(K[nI:, nI:] - K[nI:, :nI] @ np.linalg.solve(K[:nI, :nI], K[:nI, nI:]) if nI else K.copy())
    members = {}
    for i, sp_ in enumerate(spaces):
        for g in np.unique(sp_.iglob):
            members.setdefault(int(g), []).append((i, np.nonzero(sp_.iglob == g)[0]))
    D = [np.zeros_like(Si) for Si in S]
    for g, lst in members.items():
        T = sum(S[i][np.ix_(p, p)] for i, p in lst)
        for i, p in lst:
            D[i][np.ix_(p, p)] = np.linalg.solve(T, S[i][np.ix_(p, p)])
    return D


def local_matrices(dec: Decomposition, elem_nodes, Ke) -> list:
    """A^(i) = sum of the subdomain's element matrices on its local free DOFs."""
    out = []
    for elems, dofs in zip(dec.sub_elems, dec.local_dofs):
        Ki = fem.assemble(elem_nodes, Ke, dec.n_dofs, elems=elems)
        out.append(Ki[dofs][:, dofs].toarray())
    return out


class BDDC:
    """Two-level (``levels=2``) or three-level (``levels=3``) BDDC on the free-DOF operator."""

    def __init__(self, dec: Decomposition, elem_nodes, Ke, levels: int = 2, coarse_group: int = 8,
                 level2_primal: int = VERTEX | EDGE | FACE, nonsymmetric: bool = False, scaling: str = "counting"):
        self.dec = dec
        K = fem.assemble(elem_nodes, Ke, dec.n_dofs)
        self.A = fem.reduce_to_free(K, dec.free)
        Ks = local_matrices(dec, elem_nodes, Ke)
        self.levels = levels
        if levels == 2:
            self.L1 = Level(self.A, dec.subdomains, Ks, dec.n_coarse, nonsymmetric=nonsymmetric, scaling=scaling)
            self.L2 = None
        elif levels == 3:
            if dec.nnsp:
                raise NotImplementedError("three levels with near-null-space primals")
            self.L1 = Level(self.A, dec.subdomains, Ks, dec.n_coarse, build_coarse=False, nonsymmetric=nonsymmetric,
                            scaling=scaling)
            self.L2 = coarse_level(dec, self.L1, coarse_group, level2_primal, nonsymmetric)
            self.L1.coarse_solver = self.L2.apply
        else:
            raise ValueError("levels must be 2 or 3")
        self.Kc = self.L1.Kc

    def apply(self, r_free: np.ndarray) -> np.ndarray:
        return self.L1.apply(r_free)


def coarse_level(dec: Decomposition, L1: Level, group: int, primal: int, nonsymmetric: bool = False) -> Level:
    """Level-2 BDDC on S_PiPi: fine subdomains are its elements (matrices Psi_i^T A^(i) Phi_i),
    fine primal globs its nodes, level-2 subdomain of fine subdomain i is i // group."""
    nsub = dec.n_sub
    part2 = np.arange(nsub) // group
    glob_ids = sorted({gi for gi, _ in dec.coarse})
    gpos = {g: k for k, g in enumerate(glob_ids)}
    ng = len(glob_ids)
    cdof = {(gpos[gi], c): k for k, (gi, c) in enumerate(dec.coarse)}
    sub_globs = [sorted({gpos[dec.coarse[c][0]] for c in dec.subdomains[i].coarse}) for i in range(nsub)]
    g_subs = [set() for _ in range(ng)]
    for i in range(nsub):
        for g in sub_globs[i]:
            g_subs[g].add(int(part2[i]))
    g_subs = [tuple(sorted(s)) for s in g_subs]
    g_tags = np.array([dec.node_tags[dec.globs[gi][1][0]] for gi in glob_ids], dtype=np.int64)
    is_if = np.array([len(s) >= 2 for s in g_subs])
    pairs = []
    for gs in sub_globs:
        for a in range(len(gs)):
            for b in range(a + 1, len(gs)):
                pairs.append((gs[a], gs[b]))
    pairs = np.array(pairs, dtype=np.int64).reshape(-1, 2)
    globs2 = classify_globs(ng, g_subs, g_tags, is_if, pairs)
    coarse2 = []
    for k2, (kind, items, _) in enumerate(globs2):
        if kind & primal:
            for c in range(3):
                if any((g, c) in cdof for g in items):
                    coarse2.append((k2, c))
    spaces, Ks = [], []
    for j in range(int(part2.max()) + 1):
        fines = np.nonzero(part2 == j)[0]
        gl = sorted({g for i in fines for g in sub_globs[i]})
        cd = [(cdof[(g, c)], g) for g in gl for c in range(3) if (g, c) in cdof]
        cd_int = [d for d, g in cd if not is_if[g]]
        cd_if = [d for d, g in cd if is_if[g]]
        w = np.array([1.0 / len(g_subs[g]) for d, g in cd if is_if[g]])
        local = np.array(cd_int + cd_if, dtype=np.int64)
        pos = {int(d): k for k, d in enumerate(local)}
        Kj = np.zeros((len(local), len(local)))
        for i in fines:
            p = [pos[int(d)] for d in dec.subdomains[i].coarse]
            Kj[np.ix_(p, p)] += L1.loc[i]["Kc"]
        rows, cids = [], []
        for cid, (k2, c) in enumerate(coarse2):
            _, items, subs = globs2[k2]
            if j not in subs:
                continue
            dd = [cdof[(g, c)] for g in items if (g, c) in cdof]
            row = np.zeros(len(local))
            for d in dd:
                row[pos[d]] = 1.0 / len(dd)
            rows.append(row)
            cids.append(cid)
        C = np.array(rows) if rows else np.zeros((0, len(local)))
        spaces.append(LocalSpace(local, len(cd_int), w, np.array(cids, dtype=np.int64), C))
        Ks.append(Kj)
    lvl = Level(L1.Kc, spaces, Ks, len(coarse2), nonsymmetric=nonsymmetric)
    lvl.globs = globs2
    return lvl
