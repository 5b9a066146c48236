"""Oracle: assembly of element tangents and clamped-DOF elimination.

The global operator is the sum of the unassembled subdomain matrices,
A = sum_i A^(i), each of which is the sum of its element matrices (paper §3.2,
"unassembled matrix corresponding to subdomain Omega_i"; §4, MATIS storage).
Homogeneous Dirichlet DOFs are removed from rows and columns (the increment of
a clamped displacement is zero).

Test infrastructure only; see the package docstring.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def element_dofs(elem_nodes: np.ndarray) -> np.ndarray:
    """[n_el, 3*npe] global DOF ids, node-major / component-minor (DOF = 3 node + comp)."""
    return (3 * elem_nodes[:, :, None].astype(np.int64) + np.arange(3)[None, None, :]).reshape(
        elem_nodes.shape[0], -1)


def assemble(elem_nodes: np.ndarray, Ke: np.ndarray, n_dofs: int, elems=None) -> sp.csr_matrix:
    """Sum of element matrices K_e scattered to global DOFs (all DOFs, no clamps)."""
    if elems is not None:
        elem_nodes = elem_nodes[elems]
        Ke = Ke[elems]
    d = element_dofs(elem_nodes)
    nd = d.shape[1]
    rows = np.repeat(d, nd, axis=1).ravel()
    cols = np.tile(d, (1, nd)).ravel()
    K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(n_dofs, n_dofs)).tocsr()
    K.sum_duplicates()
    return K


def free_dofs(n_dofs: int, dirichlet: np.ndarray) -> np.ndarray:
    mask = np.ones(n_dofs, dtype=bool)
    mask[np.asarray(dirichlet, dtype=np.int64)] = False
    return np.nonzero(mask)[0]


def reduce_to_free(K: sp.csr_matrix, free: np.ndarray) -> sp.csr_matrix:
    return K[free][:, free].tocsr()


def rigid_body_modes(coords: np.ndarray) -> np.ndarray:
    """The six infinitesimal rigid motions sampled at the nodes, [3 n_nodes, 6]."""
    n = coords.shape[0]
    R = np.zeros((n, 3, 6))
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    for c in range(3):
        R[:, c, c] = 1.0
    R[:, 0, 3], R[:, 1, 3] = -y, x          # rotation about z
    R[:, 1, 4], R[:, 2, 4] = -z, y          # rotation about x
    R[:, 0, 5], R[:, 2, 5] = z, -x          # rotation about y
    return R.reshape(3 * n, 6)
