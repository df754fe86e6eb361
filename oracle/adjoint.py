"""Adjoint of the operator application and of the Chebyshev filter, FP64,
plain form (every forward state kept).  Test infrastructure only.

Gradients follow PyTorch's convention for a real loss L of complex Y:
G = 2 dL/d conj(Y), so that dL = Re <G, dY> with <a, b> = sum conj(a) b.

The operator depends linearly on the fields at the quadrature points
(eqn:FEHlocEl): dH_hat/dV(e,q) = M^{-1/2} R_e^T (w_q J N(q) N(q)^T (x) 1) R_e M^{-1/2}
and dH_hat/dB_d(e,q) the same with sigma_d, so for any two blocks Lam, Y

    Re <Lam, dH_hat/dV(e,q) Y> = w_q J Re sum_n lam_n(q)^H y_n(q),
    Re <Lam, dH_hat/dB_d(e,q) Y> = w_q J Re sum_n lam_n(q)^H sigma_d y_n(q),

with z(q) = sum_i N_i(r_q) (M^{-1/2} Z)_{I(e,i)} (the unscaled field at r_q).
For L = sum_n Re <x_n, H_hat x_n> these are w_q J rho(e,q) and w_q J m_d(e,q)
with rho, m of eqn:rho / eqn:mag (unit occupations), the closed form that
pins the adjoint (it is also the Hellmann-Feynman form of the appendix on
the generalised functional).
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import PAULI


def at_quadrature(mesh, M_D, Z):
    """z[e, q, alpha, n] = sum_i N_i(r_q) (M^{-1/2} Z)[2 I(e,i) + alpha, n]."""
    Zs = Z / np.repeat(np.sqrt(M_D), 2)[:, None]
    out = np.zeros((mesh.n_cell_total, mesh.nq ** 3, 2, Z.shape[1]), dtype=np.complex128)
    for e in range(mesh.n_cell_total):
        g = mesh.cell_nodes(e)
        for a in range(2):
            out[e, :, a, :] = mesh.Nt.T @ Zs[2 * g + a, :]
    return out


def cross_density(mesh, M_D, Lam, Y):
    """(dV, dB): w_q J Re sum_n lam^H [1 | sigma_d] y at every (e, q)."""
    lq = at_quadrature(mesh, M_D, Lam)
    yq = at_quadrature(mesh, M_D, Y)
    wJ = mesh.wq * mesh.J
    dV = wJ[None, :] * np.real(np.einsum("eqan,eqan->eq", lq.conj(), yq))
    dB = np.zeros(dV.shape + (3,))
    for d in range(3):
        dB[:, :, d] = wJ[None, :] * np.real(np.einsum("eqan,ab,eqbn->eq", lq.conj(), PAULI[d], yq))
    return dV, dB


def density_magnetisation(mesh, M_D, X):
    """rho(e,q) = sum_n |x_n(q)|^2 and m_d(e,q) = sum_n x_n(q)^H sigma_d x_n(q)."""
    xq = at_quadrature(mesh, M_D, X)
    rho = np.real(np.einsum("eqan,eqan->eq", xq.conj(), xq))
    m = np.zeros(rho.shape + (3,))
    for d in range(3):
        m[:, :, d] = np.real(np.einsum("eqan,ab,eqbn->eq", xq.conj(), PAULI[d], xq))
    return rho, m


def filter_coefficients(m, a, b, a0):
    """(alpha_k, beta_k) of the scaled recurrence Y_k = alpha_k (H - c) Y_{k-1} + beta_k Y_{k-2},
    k = 1..m (beta_1 = 0), and the shift c."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    s1 = e / (a0 - c)
    al = [s1 / e]
    be = [0.0]
    s = s1
    for _ in range(2, m + 1):
        sn = 1.0 / (2.0 / s1 - s)
        al.append(2.0 * sn / e)
        be.append(-s * sn)
        s = sn
    return np.array(al), np.array(be), c


def filter_backward(H, mesh, M_D, X, G, m, a, b, a0):
    """Xbar, dV, dB for Y = filter(X) given G = 2 dL/d conj(Y).
    Reverse recurrence Lam_m = G, Lam_{k-1} = alpha_k (H - c) Lam_k + beta_{k+1} Lam_{k+1};
    dL/dtheta = sum_k alpha_k Re <Lam_k, dH/dtheta Y_{k-1}>."""
    al, be, c = filter_coefficients(m, a, b, a0)
    Ys = [X]
    Y_prev, Y = None, X
    for k in range(1, m + 1):
        Yn = al[k - 1] * (H @ Y - c * Y)
        if k > 1:
            Yn = Yn + be[k - 1] * Y_prev
        Y_prev, Y = Y, Yn
        Ys.append(Y)
    dV = np.zeros((mesh.n_cell_total, mesh.nq ** 3))
    dB = np.zeros(dV.shape + (3,))
    lam_next = np.zeros_like(G)            # Lam_{k+1}
    lam = G                                # Lam_k
    for k in range(m, 0, -1):
        v, bb = cross_density(mesh, M_D, lam, Ys[k - 1])
        dV += al[k - 1] * v
        dB += al[k - 1] * bb
        beta_next = be[k] if k < m else 0.0
        lam_prev = al[k - 1] * (H @ lam - c * lam) + beta_next * lam_next
        lam_next, lam = lam, lam_prev
    return lam, dV, dB
