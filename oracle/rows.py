"""Selected rows of H_hat X for meshes too large to assemble (test
infrastructure).  Same definitions as hamiltonian.py (eqn:FEHloc, eqn:FEHnloc,
eqn:CMat; M_D of Sec. III.B.2), evaluated only for the cells that contain the
sampled nodes and for the atoms whose projector support contains them:

  (H_hat X)[2I + a] = s_I [ sum_{e containing I} sum_j H_e[(i,a),(j,b)] s_J X[2J + b]
                            + sum_atoms sum_chi P[I,chi] (Delta C)[2 chi + a] ],
  C = sum over the atom's support of conj(P[J,chi]) s_J X[2J + b],   s = M_D^{-1/2}.

Cells outside an atom's reach are skipped in the projector sums: their terms are
exactly zero (the projectors vanish beyond r_c).
"""
from __future__ import annotations

import math

import numpy as np

from . import projectors
from .fe import Mesh
from .hamiltonian import PAULI, cell_reference_matrices


def cells_of_node(mesh: Mesh, I: int):
    """(cell, local index) pairs of every cell containing global node I."""
    Nx, Ny, _ = mesh.N
    idx = [I % Nx, (I // Nx) % Ny, I // (Nx * Ny)]
    per_dir = []
    for d in range(3):
        c, a = divmod(idx[d], mesh.p)
        opts = [(c, a)]
        if a == 0:
            opts.append(((c - 1) % mesh.n_cells[d], mesh.p))
        per_dir.append(opts)
    out = []
    n = mesh.np1
    for cx, ax in per_dir[0]:
        for cy, ay in per_dir[1]:
            for cz, az in per_dir[2]:
                e = cx + mesh.n_cells[0] * (cy + mesh.n_cells[1] * cz)
                out.append((e, ax + n * (ay + n * az)))
    return out


def atom_cells(mesh: Mesh, atom, box):
    """Cells whose box lies within r_c of some periodic image of the atom."""
    L = np.asarray(box, dtype=np.float64)
    R = np.asarray(atom.pos, dtype=np.float64)
    nimg = [int(math.ceil(atom.rcut / L[d])) for d in range(3)]
    lo = np.stack([mesh.cell_origin(e) for e in range(mesh.n_cell_total)])
    hi = lo + mesh.h
    hit = np.zeros(mesh.n_cell_total, dtype=bool)
    for ix in range(-nimg[0], nimg[0] + 1):
        for iy in range(-nimg[1], nimg[1] + 1):
            for iz in range(-nimg[2], nimg[2] + 1):
                c = R + np.array([ix, iy, iz]) * L
                g = np.maximum(0.0, np.maximum(lo - c, c - hi))
                hit |= np.einsum("ij,ij->i", g, g) < atom.rcut ** 2
    return np.nonzero(hit)[0].tolist()


def projector_support(mesh: Mesh, atom, k, box):
    """(support nodes, P[node][chi]) of eqn:CMat over the atom's cells."""
    wJ = mesh.wq * mesh.J
    cells = atom_cells(mesh, atom, box)
    allnodes = np.concatenate([mesh.cell_nodes(e) for e in cells])
    nodes = np.unique(allnodes)
    P = np.zeros((nodes.size, projectors.n_orbitals(atom)), dtype=np.complex128)
    for e in cells:
        beta = projectors.bloch_projector(atom, mesh.quad_points(e), k, box)
        np.add.at(P, np.searchsorted(nodes, mesh.cell_nodes(e)), (mesh.Nt * wJ) @ beta)
    return nodes, P


def apply_rows(system, nodes, x_rows, veff_fn, bxc_fn, ik=0):
    """(H_hat X)[2I + a, :] for I in `nodes` -> [len(nodes)][2][n_cols].
    x_rows(dof_rows) returns X at those rows (any order)."""
    mesh = Mesh(system.n_cells, system.box, system.p, system.quad, system.n_q)
    k = np.asarray(system.kpts[ik], dtype=np.float64)
    M_D = mesh.lumped_mass()
    s = 1.0 / np.sqrt(M_D)
    K, Mc, C = cell_reference_matrices(mesh, k)
    wJ = mesh.wq * mesh.J
    k2 = float(k @ k)
    nodes = np.asarray(nodes)
    out = None
    for t, I in enumerate(nodes):
        for e, i in cells_of_node(mesh, int(I)):
            pts = mesh.quad_points(e)
            V = veff_fn(system, pts)
            B = bxc_fn(system, pts)
            g = mesh.cell_nodes(e)
            Ni = mesh.Nt[i]
            H0 = K[i] - 1j * C[i] + 0.5 * k2 * Mc[i] + (Ni * wJ * V) @ mesh.Nt.T
            MB = [(Ni * wJ * B[:, d]) @ mesh.Nt.T for d in range(3)]
            Xc = x_rows((2 * g[:, None] + np.arange(2)[None, :]).ravel())
            if out is None:
                out = np.zeros((len(nodes), 2, Xc.shape[1]), dtype=np.complex128)
            Xc = Xc.reshape(len(g), 2, -1) * s[g][:, None, None]
            for a in range(2):
                row = H0 @ Xc[:, a, :]
                for d in range(3):
                    for b in range(2):
                        if PAULI[d][a, b] != 0:
                            row = row + PAULI[d][a, b] * (MB[d] @ Xc[:, b, :])
                out[t, a] += s[I] * row
    # coordinates of the sampled nodes, to skip atoms whose support cannot reach them
    Nx, Ny, _ = mesh.N
    idx = np.stack([nodes % Nx, (nodes // Nx) % Ny, nodes // (Nx * Ny)], axis=1)
    xyz = np.stack([(idx[:, d] // mesh.p) * mesh.h[d] + (mesh.xi[idx[:, d] % mesh.p] + 1) * mesh.h[d] / 2
                    for d in range(3)], axis=1)
    Lb = np.asarray(system.box, dtype=np.float64)
    reach = np.linalg.norm(mesh.h)
    for atom in system.atoms:
        dmin = xyz - np.asarray(atom.pos)
        dmin = dmin - Lb * np.round(dmin / Lb)
        if np.all(np.linalg.norm(dmin, axis=1) > atom.rcut + reach):
            continue
        sup, P = projector_support(mesh, atom, k, system.box)
        supset = set(sup.tolist())
        hit = [t for t, I in enumerate(nodes) if int(I) in supset]
        if not hit:
            continue
        Xs = x_rows((2 * sup[:, None] + np.arange(2)[None, :]).ravel()).reshape(len(sup), 2, -1)
        Xs = Xs * s[sup][:, None, None]
        Cvec = np.einsum("jx,jbn->xbn", P.conj(), Xs).reshape(2 * P.shape[1], -1)   # index 2 chi + b
        DC = (projectors.delta_matrix(atom) @ Cvec).reshape(P.shape[1], 2, -1)
        pos = {int(I): r for r, I in enumerate(sup)}
        for t in hit:
            I = int(nodes[t])
            out[t] += s[I] * np.einsum("x,xan->an", P[pos[I]], DC)
    return out
