"""Electron and magnetisation densities from Rayleigh-Ritz output with
Fermi-Dirac occupations, FP64.  Test infrastructure only.

eqn:rho and eqn:mag: rho(r) = sum_n f_n psi_n^H psi_n, m(r) = sum_n f_n psi_n^H sigma psi_n
(for periodic systems the sum over n includes the Brillouin-zone average, i.e. the
k-point weights); the occupations are Fermi-Dirac numbers at the smearing
temperature (Sec. V: 500 K), with the Fermi level fixed by the electron count, and
the entropy term E_ent = kT sum w [f ln f + (1 - f) ln(1 - f)] of Sec. II.B.
With psi = exp(ik.r) u the densities depend on the periodic parts u only.  The
vectors here are the scaled blocks X = M_D^{1/2} U, so u_n(q) is the field
sum_i N_i(r_q) (M_D^{-1/2} x_n)_i at the quadrature point.
"""
from __future__ import annotations

import math

import numpy as np

from .adjoint import at_quadrature
from .hamiltonian import PAULI

KELVIN_TO_HA = 3.166811563e-6      # Boltzmann constant in Ha / K


def fermi_function(eps, mu, kT):
    """1 / (1 + exp((eps - mu) / kT)), elementwise, in a form that never overflows."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / kT
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def fermi_dirac(eps, n_electrons, kT, weights=None):
    """(occupations, mu, E_ent): mu by bisection on the monotone electron count
    sum_i w_i f(eps_i; mu) = n_electrons."""
    eps = np.asarray(eps, dtype=np.float64)
    w = np.ones_like(eps) if weights is None else np.asarray(weights, dtype=np.float64)
    if not (0.0 < n_electrons < w.sum()):
        raise ValueError("need 0 < n_electrons < sum of weights")
    lo, hi = eps.min() - 50.0 * kT, eps.max() + 50.0 * kT
    for _ in range(400):
        mu = 0.5 * (lo + hi)
        if (w * fermi_function(eps, mu, kT)).sum() < n_electrons:
            lo = mu
        else:
            hi = mu
        if hi - lo <= 1e-15 * max(1.0, abs(mu)):
            break
    mu = 0.5 * (lo + hi)
    f = fermi_function(eps, mu, kT)
    ent = 0.0
    for fi, wi in zip(f, w):
        if 0.0 < fi < 1.0:
            ent += wi * (fi * math.log(fi) + (1.0 - fi) * math.log(1.0 - fi))
    return f, mu, kT * ent


def density_magnetisation(mesh, M_D, X, occ):
    """rho[e, q] = sum_n occ_n |u_n(q)|^2, m[e, q, d] = sum_n occ_n u_n(q)^H sigma_d u_n(q)."""
    xq = at_quadrature(mesh, M_D, X)                     # [e, q, alpha, n]
    f = np.asarray(occ, dtype=np.float64)
    rho = np.real(np.einsum("eqan,eqan,n->eq", xq.conj(), xq, f))
    m = np.zeros(rho.shape + (3,))
    for d in range(3):
        m[:, :, d] = np.real(np.einsum("eqan,ab,eqbn,n->eq", xq.conj(), PAULI[d], xq, f))
    return rho, m


def density_at_cells(mesh, M_D, rows_fn, cells, occ):
    """density_magnetisation restricted to the listed cells, the block's rows read
    through rows_fn(row_indices) -> [len(rows), n] so that a large block need not
    exist on the host.  Returns rho [len(cells), nq^3], m [len(cells), nq^3, 3]."""
    f = np.asarray(occ, dtype=np.float64)
    nq3 = mesh.nq ** 3
    rho = np.zeros((len(cells), nq3))
    m = np.zeros((len(cells), nq3, 3))
    for i, e in enumerate(cells):
        g = mesh.cell_nodes(e)
        rows = np.stack([2 * g, 2 * g + 1], axis=1).ravel()
        Z = np.asarray(rows_fn(rows)).reshape(len(g), 2, -1) / np.sqrt(M_D[g])[:, None, None]
        u = np.einsum("iq,ian->qan", mesh.Nt, Z)                 # [q, alpha, n]
        rho[i] = np.real(np.einsum("qan,qan,n->q", u.conj(), u, f))
        for d in range(3):
            m[i, :, d] = np.real(np.einsum("qan,ab,qbn,n->q", u.conj(), PAULI[d], u, f))
    return rho, m
