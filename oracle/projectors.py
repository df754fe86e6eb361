"""Synthetic spin-orbit nonlocal projectors (paper Sec. II.B eqn:nlOP; eqn:CMat;
eqn:FEHnloc; the cell form with Delta_{2chi+alpha, 2chi'+beta} = D^{chi chi'}_{alpha beta}).

The ONCV data the paper uses are not available.  Stand-in: for each atom and
each l <= lmax, the 2l+1 real solid harmonics times a normalised Gaussian,
    p_lm(r) = c_l r^l Y_lm(r_hat) exp(-r^2 / (2 sigma^2)),  zero for r >= r_c,
with c_l^2 = 2 / (Gamma(l + 3/2) sigma^(2l+3)) so that int |p_lm|^2 = 1, and
    Delta = D0_l 1 + D_so L.S   (S = sigma_Pauli / 2)   within each l shell.
Test infrastructure only.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

Poly = Dict[Tuple[int, int, int], complex]


def real_harmonic_polys(l: int) -> List[Poly]:
    """r^l Y_lm as homogeneous polynomials, orthonormal real harmonics.
    Order: l=1 (x, y, z); l=2 (xy, yz, 3z^2-r^2, xz, x^2-y^2)."""
    if l == 0:
        return [{(0, 0, 0): 0.5 / math.sqrt(math.pi)}]
    if l == 1:
        c = math.sqrt(3.0 / (4.0 * math.pi))
        return [{(1, 0, 0): c}, {(0, 1, 0): c}, {(0, 0, 1): c}]
    if l == 2:
        c = 0.5 * math.sqrt(15.0 / math.pi)
        cz = 0.25 * math.sqrt(5.0 / math.pi)
        cx = 0.25 * math.sqrt(15.0 / math.pi)
        return [{(1, 1, 0): c}, {(0, 1, 1): c},
                {(0, 0, 2): 2 * cz, (2, 0, 0): -cz, (0, 2, 0): -cz},
                {(1, 0, 1): c}, {(2, 0, 0): cx, (0, 2, 0): -cx}]
    raise ValueError("l <= 2 supported")


def _deriv(poly: Poly, d: int) -> Poly:
    out: Poly = {}
    for mono, c in poly.items():
        if mono[d] == 0:
            continue
        m = list(mono)
        k = m[d]
        m[d] -= 1
        out[tuple(m)] = out.get(tuple(m), 0.0) + c * k
    return out


def _mul_var(poly: Poly, d: int) -> Poly:
    out: Poly = {}
    for mono, c in poly.items():
        m = list(mono)
        m[d] += 1
        out[tuple(m)] = out.get(tuple(m), 0.0) + c
    return out


def _add(a: Poly, b: Poly, sb=1.0) -> Poly:
    out = dict(a)
    for k, v in b.items():
        out[k] = out.get(k, 0.0) + sb * v
    return out


def angular_momentum(l: int) -> np.ndarray:
    """[3][2l+1][2l+1] matrices of L_c = -i (r x grad)_c in the real-harmonic
    basis: L_c phi_m' = sum_m (L_c)[m, m'] phi_m, found by applying the
    differential operator to each basis polynomial and solving for the
    coefficients in the basis."""
    basis = real_harmonic_polys(l)
    monos = sorted({k for p in basis for k in p})
    Bm = np.array([[p.get(k, 0.0) for p in basis] for k in monos], dtype=np.complex128)
    Ls = np.zeros((3, len(basis), len(basis)), dtype=np.complex128)
    # (r x grad)_x = y d_z - z d_y, _y = z d_x - x d_z, _z = x d_y - y d_x
    pairs = [(1, 2), (2, 0), (0, 1)]
    for c, (a, b) in enumerate(pairs):
        for j, phi in enumerate(basis):
            t = _add(_mul_var(_deriv(phi, b), a), _mul_var(_deriv(phi, a), b), -1.0)
            vec = np.array([-1j * t.get(k, 0.0) for k in monos], dtype=np.complex128)
            coef, *_ = np.linalg.lstsq(Bm, vec, rcond=None)
            Ls[c, :, j] = coef
    return Ls


PAULI = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128)


def delta_matrix(atom) -> np.ndarray:
    """Delta [2 n_pj][2 n_pj], index 2 chi + alpha: D0_l delta + D_so L.S per shell."""
    blocks = []
    for l in range(atom.lmax + 1):
        n = 2 * l + 1
        D = atom.d0[l] * np.eye(2 * n, dtype=np.complex128)
        if l > 0 and atom.dso != 0.0:
            Lm = angular_momentum(l)
            for c in range(3):
                D = D + atom.dso * np.kron(Lm[c], PAULI[c] / 2.0)
        blocks.append(D)
    n_tot = sum(b.shape[0] for b in blocks)
    out = np.zeros((n_tot, n_tot), dtype=np.complex128)
    o = 0
    for b in blocks:
        out[o:o + b.shape[0], o:o + b.shape[0]] = b
        o += b.shape[0]
    return out


def n_orbitals(atom) -> int:
    return sum(2 * l + 1 for l in range(atom.lmax + 1))


def _eval_poly(poly: Poly, d: np.ndarray) -> np.ndarray:
    out = np.zeros(d.shape[0])
    for (a, b, c), coef in poly.items():
        out += coef * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c
    return out


def projector_values(atom, d: np.ndarray) -> np.ndarray:
    """p_chi(d) for displacements d [P][3] -> [P][n_pj] (real)."""
    r2 = np.einsum("ij,ij->i", d, d)
    inside = r2 < atom.rcut * atom.rcut
    out = np.zeros((d.shape[0], n_orbitals(atom)))
    col = 0
    for l in range(atom.lmax + 1):
        cl = math.sqrt(2.0 / (math.gamma(l + 1.5) * atom.sigma ** (2 * l + 3)))
        g = np.where(inside, cl * np.exp(-r2 / (2.0 * atom.sigma ** 2)), 0.0)
        for poly in real_harmonic_polys(l):
            out[:, col] = g * _eval_poly(poly, d)
            col += 1
    return out


def bloch_projector(atom, pts: np.ndarray, k, box) -> np.ndarray:
    """beta_chi(r) = sum_L exp(-i k.(r - L)) p_chi(r - R_a - L) at pts [P][3]
    (eqn:HnlocPeriodic; eqn:CMat with the atom position included)."""
    L = np.asarray(box, dtype=np.float64)
    R = np.asarray(atom.pos, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    # points and atoms lie in [0, L): an image n contributes only if |n| L < L + r_c
    nimg = [int(math.ceil(atom.rcut / L[d])) for d in range(3)]
    out = np.zeros((pts.shape[0], n_orbitals(atom)), dtype=np.complex128)
    for ix in range(-nimg[0], nimg[0] + 1):
        for iy in range(-nimg[1], nimg[1] + 1):
            for iz in range(-nimg[2], nimg[2] + 1):
                sh = np.array([ix, iy, iz]) * L
                d = pts - R - sh
                r2 = np.einsum("ij,ij->i", d, d)
                m = r2 < atom.rcut * atom.rcut
                if not np.any(m):
                    continue
                vals = projector_values(atom, d[m])
                phase = np.exp(-1j * ((pts[m] - sh) @ k))
                out[m] += phase[:, None] * vals
    return out
