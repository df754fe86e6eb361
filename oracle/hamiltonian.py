"""Assembled FE Hamiltonian H^k and its symmetric scaling (paper eqn:FEHloc,
eqn:FEHnloc, eqn:CMat, eqn:OvlapMap, eqn:GHEP; Sec. III.B.2 for M_D).

H^k_{2I+a, 2J+b} = int [ 1/2 grad N_I . grad N_J - i N_I k.grad N_J
                         + |k|^2/2 N_I N_J + V N_I N_J ] delta_ab
                   + sum_d int B_d N_I N_J sigma^d_ab
                   + sum_atoms sum_{chi chi'} P_{I chi} Delta_{2chi+a, 2chi'+b} conj(P_{J chi'})
The filter works on M_D^{-1} H; the oracle uses the similar matrix
H_hat = M_D^{-1/2} H M_D^{-1/2} so that orthonormality is Euclidean.
Cell integrals use the mesh's quadrature (eqn:cellIntegrals); the global
sparse matrix is assembled cell by cell and summed (the restriction form of
Sec. IV.B written out as index arithmetic).  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import projectors
from .fe import Mesh

PAULI = projectors.PAULI


def mesh_for(system) -> Mesh:
    return Mesh(system.n_cells, system.box, system.p, system.quad, system.n_q)


def fields_at_quadrature(mesh: Mesh, system, veff_fn, bxc_fn):
    """V [E][nq^3] and B [E][nq^3][3] evaluated at the oracle's own points."""
    pts = mesh.all_quad_points().reshape(-1, 3)
    V = veff_fn(system, pts).reshape(mesh.n_cell_total, -1)
    B = bxc_fn(system, pts).reshape(mesh.n_cell_total, -1, 3)
    return V, B


def cell_reference_matrices(mesh: Mesh, k):
    """Kinetic, consistent-mass and k-gradient cell matrices.  All cells of the
    uniform mesh have the same h, so these are computed once:
       K[i,j] = 1/2 sum_q w_q J grad N_i . grad N_j
       Mc[i,j] = sum_q w_q J N_i N_j
       C[i,j] = sum_q w_q J N_i (k . grad N_j)."""
    wJ = mesh.wq * mesh.J
    K = 0.5 * sum((mesh.dNt[d] * wJ) @ mesh.dNt[d].T for d in range(3))
    Mc = (mesh.Nt * wJ) @ mesh.Nt.T
    kgrad = sum(k[d] * mesh.dNt[d] for d in range(3))
    C = (mesh.Nt * wJ) @ kgrad.T
    return K, Mc, C


def projector_matrix(mesh: Mesh, atom, k, box):
    """P[I, chi] = sum_e sum_q w_q J N_i(r_q) beta_chi(r_q) (eqn:CMat), dense [M][n_pj]."""
    wJ = mesh.wq * mesh.J
    P = np.zeros((mesh.n_nodes, projectors.n_orbitals(atom)), dtype=np.complex128)
    for e in range(mesh.n_cell_total):
        beta = projectors.bloch_projector(atom, mesh.quad_points(e), k, box)
        if not np.any(beta):
            continue
        contrib = (mesh.Nt * wJ) @ beta           # [n^3][n_pj]
        np.add.at(P, mesh.cell_nodes(e), contrib)
    return P


def assemble_local(mesh: Mesh, V, B, k):
    """Global sparse complex128 H^{k,loc} (2M x 2M), CSR (eqn:FEHloc)."""
    k = np.asarray(k, dtype=np.float64)
    K, Mc, C = cell_reference_matrices(mesh, k)
    wJ = mesh.wq * mesh.J
    n = mesh.Nt.shape[0]
    k2 = float(k @ k)
    rows, cols, vals = [], [], []
    I2 = np.eye(2)
    for e in range(mesh.n_cell_total):
        MV = (mesh.Nt * (wJ * V[e])) @ mesh.Nt.T
        H0 = K - 1j * C + 0.5 * k2 * Mc + MV
        Hc = np.kron(H0, I2)
        for d in range(3):
            MB = (mesh.Nt * (wJ * B[e, :, d])) @ mesh.Nt.T
            Hc = Hc + np.kron(MB, PAULI[d])
        g = mesh.cell_nodes(e)
        dof = (2 * g[:, None] + np.arange(2)[None, :]).ravel()
        rows.append(np.repeat(dof, 2 * n))
        cols.append(np.tile(dof, 2 * n))
        vals.append(Hc.ravel())
    nd = 2 * mesh.n_nodes
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nd, nd)).tocsr()


def spinor_projectors(mesh: Mesh, atoms, k, box):
    """Per atom: Ps [2M][2 n_pj] sparse with Ps[2I+a, 2chi+b] = P[I,chi] delta_ab, and Delta."""
    out = []
    for atom in atoms:
        P = projector_matrix(mesh, atom, k, box)
        Ps = sp.kron(sp.csr_matrix(P), sp.identity(2, format="csr"), format="csr")
        out.append((Ps, projectors.delta_matrix(atom)))
    return out


class Operator:
    """H_hat = M_D^{-1/2} (H^loc + sum_a Ps_a Delta_a Ps_a^H) M_D^{-1/2}, with the
    local part assembled as a sparse matrix and each atom's nonlocal term kept
    as the product of eqn:FEHnloc (assembling it would fill whole blocks)."""

    def __init__(self, Hloc, projs, M_D):
        s = np.repeat(1.0 / np.sqrt(M_D), 2)
        S = sp.diags(s)
        self.loc = (S @ Hloc @ S).tocsr()
        self.projs = [((S @ Ps).tocsr(), D) for Ps, D in projs]
        self.shape = self.loc.shape
        self.dtype = np.complex128

    def __matmul__(self, X):
        Y = self.loc @ X
        for Ps, D in self.projs:
            Y = Y + Ps @ (D @ (Ps.conj().T @ X))
        return Y

    def toarray(self):
        A = self.loc.toarray()
        for Ps, D in self.projs:
            Pd = Ps.toarray()
            A = A + Pd @ D @ Pd.conj().T
        return A


def build(system, veff_fn, bxc_fn, ik=0, V=None, B=None, atoms=None):
    """Mesh, fields and H_hat for k-point ik.  Returns (mesh, H_hat, M_D, V, B)."""
    mesh = mesh_for(system)
    if V is None or B is None:
        V, B = fields_at_quadrature(mesh, system, veff_fn, bxc_fn)
    k = system.kpts[ik]
    Hloc = assemble_local(mesh, V, B, k)
    projs = spinor_projectors(mesh, system.atoms if atoms is None else atoms, k, system.box)
    M_D = mesh.lumped_mass()
    return mesh, Operator(Hloc, projs, M_D), M_D, V, B
