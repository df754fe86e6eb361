"""Self-consistent field iteration, plain FP64 -- TEST INFRASTRUCTURE ONLY.

The nonlinear problem is the fixed point F[(rho, m)] = (rho, m) of Sec. III.B
(eqn:fixedpointmap): from input densities build V_eff and B_xc, solve the linear
eigenproblem by ChFSI, and form the output densities (eqn:rho, eqn:mag) with
Fermi-Dirac occupations.  Inputs for the next iteration come from Anderson mixing
(Sec. III.B, "Density Mixing"): with the last n inputs x_j and residuals
f_j = F(x_j) - x_j, coefficients b_j with sum_j b_j = 1 minimise
|| sum_j b_j f_j || in the norm of eqn:innerPdt,
    <(rho1, m1), (rho2, m2)> = (1/2) (int rho1 rho2 + int m1 . m2),
and the next input is sum_j b_j (x_j + alpha f_j), the charge part of the residual
passed through the Kerker preconditioner K.  The two-grid strategy (Sec. IV.A,
eqn:FEWfnsCMesh) iterates first with degree p - 1 elements on the same cells and
moves the subspace to degree p by interpolation.

Readings (the map itself needs electrostatics and an XC functional that this
build leaves out; these stand-ins keep its structure):
* V_eff = V_ext + V_H[rho] + V_x[rho, |m|],  B_xc = B_ext + B_x[rho, m], where
  V_ext, B_ext are the synthetic external fields, V_H solves the periodic
  Poisson problem -lap V_H = 4 pi (rho - rho_bar) (the uniform background rho_bar
  stands in for the smeared nuclear charges of eqn:poissonEl; V_H has zero mean
  under the lumped GLL mass), and V_x, B_x are the LSDA (Dirac) exchange under the
  locally collinear substitution rho_up,dn = (rho +- |m|)/2 of Sec. II.B:
  e_x = -(3/4)(6/pi)^(1/3) (rho_up^(4/3) + rho_dn^(4/3)), v_s = -(6/pi)^(1/3) rho_s^(1/3),
  V_x = (v_up + v_dn)/2, B_x = (v_up - v_dn)/2 m/|m| (zero where m = 0).
* Kerker: K rho = rho - k0^2 w with (k0^2 - lap) w = rho (Fourier factor
  G^2/(G^2 + k0^2)), applied to the charge part of the mixed residual; the
  Anderson coefficients use the unpreconditioned residuals.
* Field equations are solved in the FE space of the eigenproblem: for
  (kappa^2 - lap) u = g the Galerkin system (K_s + kappa^2 M_c) u = b with
  K_s = int grad N_I . grad N_J, M_c = int N_I N_J and b_I = int N_I g, all with the
  cell quadrature; u at a point is sum_I N_I u_I.
* The output densities are scaled to hold exactly N_e electrons: the eigenvectors
  are normalised in the lumped (GLL) mass, while int rho uses the cell quadrature,
  and the two differ at the level of the discretisation error.  Without the
  scaling that uniform charge residual would never be mixed away (the Kerker
  factor vanishes at G = 0).
* ChFSI per SCF iteration: Lanczos bound (40 steps, seeded), a prologue CholGS +
  Rayleigh-Ritz on the first iteration of each grid, then `passes_first` passes on
  the first iteration and `passes` on the later ones, bounds from the previous
  Rayleigh-Ritz.  The Anderson history is cleared when the grid changes.
* Brillouin-zone sampling (Sec. II.C: the sum over states becomes the sum over n
  of the zone average over k): every k-point of the system carries its own block
  and ChFSI passes, with weights w_k summing to one (equal by default); the
  occupations f_nk are Fermi-Dirac numbers with one Fermi level for all (n, k),
  fixed by sum_k w_k sum_n f_nk = N_e, and the densities are
  rho = sum_k w_k sum_n f_nk |u_nk|^2 (likewise m) of the periodic parts u.  The
  start block of k-point ik is the seeded block of seed + 7919 ik.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import chfsi as och, density as oden, hamiltonian as ham
from .fe import Mesh, lagrange_tables

C_X = (6.0 / np.pi) ** (1.0 / 3.0)


# ---------------------------------------------------------------- fields at quadrature points
def integrate(mesh: Mesh, f):
    """int f over the box with the cell quadrature; f is [E][nq^3] (or [E][nq^3][d])."""
    wJ = mesh.wq * mesh.J
    f = np.asarray(f)
    if f.ndim == 2:
        return float(np.sum(f * wJ[None, :]))
    return float(np.sum(f * wJ[None, :, None]))


def inner(mesh: Mesh, r1, m1, r2, m2):
    """eqn:innerPdt."""
    return 0.5 * (integrate(mesh, r1 * r2) + integrate(mesh, np.sum(m1 * m2, axis=-1)))


def scalar_operator(mesh: Mesh, kappa2):
    """Sparse K_s + kappa^2 M_c (M x M) assembled from the cell matrices."""
    K, Mc, _ = ham.cell_reference_matrices(mesh, np.zeros(3))
    A = 2.0 * K + kappa2 * Mc
    rows, cols, vals = [], [], []
    for e in range(mesh.n_cell_total):
        g = mesh.cell_nodes(e)
        rows.append(np.repeat(g, g.size))
        cols.append(np.tile(g, g.size))
        vals.append(A.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()


def project(mesh: Mesh, g):
    """b_I = int N_I g (cell quadrature)."""
    wJ = mesh.wq * mesh.J
    b = np.zeros(mesh.n_nodes)
    for e in range(mesh.n_cell_total):
        np.add.at(b, mesh.cell_nodes(e), mesh.Nt @ (wJ * g[e]))
    return b


def interpolate(mesh: Mesh, u):
    """u(e, q) = sum_i N_i(r_q) u_{I(e,i)}."""
    return np.stack([mesh.Nt.T @ u[mesh.cell_nodes(e)] for e in range(mesh.n_cell_total)])


def hartree(mesh: Mesh, rho):
    """V_H at the quadrature points: -lap V_H = 4 pi (rho - rho_bar), periodic,
    zero mean under the lumped mass.  The singular system is solved with node 0
    held at zero (a direct sparse solve), then the mean is removed."""
    vol = float(np.prod(mesh.box))
    rho_bar = integrate(mesh, rho) / vol
    b = 4.0 * np.pi * project(mesh, rho - rho_bar)
    A = scalar_operator(mesh, 0.0)
    keep = np.arange(1, mesh.n_nodes)
    u = np.zeros(mesh.n_nodes)
    u[keep] = spla.spsolve(A[keep][:, keep].tocsc(), b[keep])
    MD = mesh.lumped_mass()
    u -= np.dot(MD, u) / MD.sum()
    return interpolate(mesh, u)


def kerker(mesh: Mesh, rho, k0):
    """K rho = rho - k0^2 w, (k0^2 - lap) w = rho in the FE space."""
    if k0 <= 0.0:
        return rho.copy()
    A = scalar_operator(mesh, k0 * k0)
    w = spla.spsolve(A.tocsc(), project(mesh, rho))
    return rho - k0 * k0 * interpolate(mesh, w)


def exchange(rho, m):
    """(V_x, B_x, e_x) pointwise: LSDA Dirac exchange with rho_s = (rho +- |m|)/2."""
    mabs = np.linalg.norm(m, axis=-1)
    r_up = np.maximum(0.5 * (rho + mabs), 0.0)
    r_dn = np.maximum(0.5 * (rho - mabs), 0.0)
    v_up = -C_X * np.cbrt(r_up)
    v_dn = -C_X * np.cbrt(r_dn)
    e_x = -0.75 * C_X * (r_up ** (4.0 / 3.0) + r_dn ** (4.0 / 3.0))
    V = 0.5 * (v_up + v_dn)
    with np.errstate(invalid="ignore", divide="ignore"):
        unit = np.where(mabs[..., None] > 0.0, m / mabs[..., None], 0.0)
    B = 0.5 * (v_up - v_dn)[..., None] * unit
    return V, B, e_x


def potentials(mesh: Mesh, rho, m, vext, bext):
    """(V_eff, B_xc) of the input densities (the map's first step)."""
    vx, bx, _ = exchange(rho, m)
    return vext + hartree(mesh, rho) + vx, bext + bx


# ---------------------------------------------------------------- mixing
def anderson_coefficients(mesh: Mesh, res):
    """b_j, sum b_j = 1, minimising || sum_j b_j f_j || (eqn:innerPdt norm):
    A b = lambda 1 with A_jk = <f_j, f_k>."""
    n = len(res)
    A = np.array([[inner(mesh, res[j][0], res[j][1], res[k][0], res[k][1]) for k in range(n)]
                  for j in range(n)])
    c = np.linalg.solve(A, np.ones(n))
    return c / c.sum()


def anderson_next(mesh: Mesh, xs, fs, alpha, k0):
    """sum_j b_j x_j + alpha (K f_rho, f_m), f = sum_j b_j f_j."""
    b = anderson_coefficients(mesh, fs)
    xr = sum(bj * x[0] for bj, x in zip(b, xs))
    xm = sum(bj * x[1] for bj, x in zip(b, xs))
    fr = sum(bj * f[0] for bj, f in zip(b, fs))
    fm = sum(bj * f[1] for bj, f in zip(b, fs))
    return xr + alpha * kerker(mesh, fr, k0), xm + alpha * fm, b


# ---------------------------------------------------------------- two-grid transfer
def interpolate_block(coarse: Mesh, fine: Mesh, Yc):
    """eqn:FEWfnsCMesh: the degree-(p-1) spinor fields of the scaled block
    Yc = M_D,c^{1/2} Uc evaluated at the degree-p nodes of the same cells,
    returned scaled by M_D,f^{1/2}.  Every fine node takes its value from the
    cells that hold it (all give the same value: the coarse field is continuous)."""
    assert coarse.n_cells == fine.n_cells and fine.p == coarse.p + 1
    Uc = Yc / np.repeat(np.sqrt(coarse.lumped_mass()), 2)[:, None]
    T, _ = lagrange_tables(coarse.xi, fine.xi)            # T[i, a] = l_i^{p-1}(xi_a^p)
    Lc, Lf = coarse.loc, fine.loc
    T3 = T[Lc[:, 0]][:, Lf[:, 0]] * T[Lc[:, 1]][:, Lf[:, 1]] * T[Lc[:, 2]][:, Lf[:, 2]]   # [nc^3][nf^3]
    Uf = np.zeros((2 * fine.n_nodes, Yc.shape[1]), dtype=Yc.dtype)
    for e in range(fine.n_cell_total):
        gc, gf = coarse.cell_nodes(e), fine.cell_nodes(e)
        for a in range(2):
            Uf[2 * gf + a] = T3.T @ Uc[2 * gc + a]
    return Uf * np.repeat(np.sqrt(fine.lumped_mass()), 2)[:, None]


# ---------------------------------------------------------------- the SCF loop
class Grid:
    """One discretisation of the system: mesh, operator builder, block."""

    def __init__(self, system, atoms):
        self.s = system
        self.mesh = ham.mesh_for(system)
        self.atoms = atoms
        self.MD = self.mesh.lumped_mass()

    def operator(self, V, B, ik=0):
        k = self.s.kpts[ik]
        Hloc = ham.assemble_local(self.mesh, V, B, k)
        projs = ham.spinor_projectors(self.mesh, self.atoms, k, self.s.box)
        return ham.Operator(Hloc, projs, self.MD)


KSEED = 7919      # start block of k-point ik: the seeded block of seed + KSEED ik


def k_weights(system, kweights=None):
    """The zone-average weights of the system's k-points (equal by default; given
    weights must be >= 0 and sum to one)."""
    nk = len(system.kpts)
    if kweights is None:
        return np.full(nk, 1.0 / nk)
    w = np.asarray(kweights, dtype=np.float64).reshape(-1)
    if w.shape[0] != nk or (w < 0).any() or abs(w.sum() - 1.0) > 1e-12:
        raise ValueError("need one weight >= 0 per k-point, summing to one")
    return w


def occupations(thetas, w, n_electrons, kT):
    """f_nk (list per k), mu: one Fermi level for all (n, k) with weights w_k."""
    eps = np.concatenate([np.asarray(t, dtype=np.float64) for t in thetas])
    wts = np.concatenate([np.full(len(t), wk) for t, wk in zip(thetas, w)])
    f, mu, _ = oden.fermi_dirac(eps, n_electrons, kT, weights=wts)
    out, i0 = [], 0
    for t in thetas:
        out.append(f[i0:i0 + len(t)])
        i0 += len(t)
    return out, mu


def scf(fine_system, vext, bext, rho0, m0, n_electrons, kT, *, coarse_system=None, n_vec=None, degree=None,
        passes_first=4, passes=1, depth=4, alpha=0.5, k0=0.0, tol=1e-8, tol_coarse=1e-3, max_iter=40,
        max_coarse=20, seed=0, lanczos_steps=40, X0=None, kweights=None):
    """Run the SCF loop.  vext [E][nq^3], bext [E][nq^3][3] at the (shared)
    quadrature points; rho0, m0 the initial input densities; every k-point of the
    system is sampled with the weights kweights (equal by default); X0 an optional
    start block (one array, or one per k-point).  Returns a dict with the history
    [(degree p of the grid, residual norm, mu, sum_k w_k sum_n f_nk theta_nk,
    lowest theta over k, upper bound b of the filter at the first k-point, the
    bounds of all k-points)], the final input and output densities, and theta, X,
    occ of the first k-point (theta_k, X_k, occ_k: all k-points)."""
    import synth
    grids = ([Grid(coarse_system, coarse_system.atoms)] if coarse_system is not None else []) + \
        [Grid(fine_system, fine_system.atoms)]
    nk = len(fine_system.kpts)
    if coarse_system is not None:
        assert np.array_equal(np.asarray(coarse_system.kpts), np.asarray(fine_system.kpts))
    w = k_weights(fine_system, kweights)
    n_vec = fine_system.n_vec if n_vec is None else n_vec
    degree = fine_system.degree if degree is None else degree
    rho_in, m_in = rho0.copy(), m0.copy()
    hist, xs, fs = [], [], []
    X = None
    theta = [None] * nk
    it = 0
    for gi, g in enumerate(grids):
        last = gi == len(grids) - 1
        if X is None:
            if X0 is None:
                X = [synth.random_block(seed + KSEED * ik, g.s.n_dof, n_vec) for ik in range(nk)]
            else:
                X = [np.array(x, copy=True) for x in (X0 if isinstance(X0, (list, tuple)) else [X0])]
                assert len(X) == nk
        else:
            X = [interpolate_block(grids[gi - 1].mesh, g.mesh, x) for x in X]
        xs, fs = [], []
        first = True
        n_here = 0
        while True:
            it += 1
            n_here += 1
            V, B = potentials(g.mesh, rho_in, m_in, vext, bext)
            bs = []
            for ik in range(nk):
                H = g.operator(V, B, ik)
                _, b = och.lanczos_bounds(H, synth.lanczos_start(g.s, g.s.n_dof), lanczos_steps)
                bs.append(b)
                if first:
                    X[ik] = och.chol_gs(X[ik])
                    theta[ik], X[ik], _ = och.rayleigh_ritz(H, X[ik])
                for _ in range(passes_first if (first and gi == 0) else passes):
                    X[ik] = och.cheb_filter(H, X[ik], degree, float(theta[ik][-1]), b, float(theta[ik][0]))
                    X[ik] = och.chol_gs(X[ik])
                    theta[ik], X[ik], r = och.rayleigh_ritz(H, X[ik])
            first = False
            f, mu = occupations(theta, w, n_electrons, kT)
            rho_out, m_out = 0.0, 0.0
            for ik in range(nk):
                r_k, m_k = oden.density_magnetisation(g.mesh, g.MD, X[ik], w[ik] * f[ik])
                rho_out, m_out = rho_out + r_k, m_out + m_k
            q = n_electrons / integrate(g.mesh, rho_out)
            rho_out, m_out = q * rho_out, q * m_out
            fr, fm = rho_out - rho_in, m_out - m_in
            nres = float(np.sqrt(inner(g.mesh, fr, fm, fr, fm)))
            eband = float(sum(w[ik] * np.dot(f[ik], theta[ik]) for ik in range(nk)))
            th0 = float(min(t[0] for t in theta))
            hist.append((g.s.p, nres, mu, eband, th0, bs[0], tuple(bs)))
            conv = nres < (tol if last else tol_coarse)
            if last and (conv or it >= max_iter):
                return {"history": hist, "rho_in": rho_in, "m_in": m_in, "rho_out": rho_out, "m_out": m_out,
                        "theta": theta[0], "X": X[0], "occ": f[0], "theta_k": np.array(theta), "X_k": X,
                        "occ_k": np.array(f), "converged": conv}
            xs.append((rho_in, m_in))
            fs.append((fr, fm))
            xs, fs = xs[-depth:], fs[-depth:]
            rho_in, m_in, _ = anderson_next(g.mesh, xs, fs, alpha, k0)
            if not last and (conv or n_here >= max_coarse or it >= max_iter):
                break
        # the grid changes: the mixed input densities carry over, the history does not
    raise AssertionError("unreachable")
