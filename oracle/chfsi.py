"""Chebyshev-filtered subspace iteration, plain FP64 (paper Sec. III.B.2, eqn:chebfilt
and the Rayleigh-Ritz projection that follows it).

Readings taken where the paper is silent:
* the filter uses the scaled three-term recurrence of Zhou, Saad, Tiago and
  Chelikowsky (2006, cited by the paper), which equals T_m(H_s) X divided by the
  scalar T_m((a0 - c)/e), so spans and Ritz values equal the plain form's;
* the upper bound b comes from k Lanczos steps as theta_max + ||f_k||
  (Zhou and Li 2011); lambda_T (= a) is the largest Ritz value of the previous
  pass and a0 the smallest;
* the generalised projected problem is solved by first making the block
  orthonormal (Cholesky-Gram-Schmidt: S = X^H X = L L^H, X <- X L^{-H}) and then
  a standard Hermitian eigenproblem, which gives the same Ritz pairs.
Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def lanczos_bounds(H, v0, steps: int):
    """k-step Lanczos on Hermitian H from v0.  Returns (theta_min, theta_max + ||f_k||)."""
    v = v0 / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for j in range(steps):
        w = H @ v
        alpha = float(np.real(np.vdot(v, w)))
        w = w - alpha * v - beta * v_prev
        beta_new = float(np.linalg.norm(w))
        alphas.append(alpha)
        if j < steps - 1:
            betas.append(beta_new)
        v_prev, v, beta = v, w / beta_new, beta_new
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    theta = np.linalg.eigvalsh(T)
    return float(theta[0]), float(theta[-1] + beta)


def lanczos_coefficients(H, v0, steps: int):
    """The (alpha_j, beta_j) sequence of the same Lanczos run (for parity tests)."""
    v = v0 / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for _ in range(steps):
        w = H @ v
        alpha = float(np.real(np.vdot(v, w)))
        w = w - alpha * v - beta * v_prev
        beta = float(np.linalg.norm(w))
        alphas.append(alpha)
        betas.append(beta)
        v_prev, v = v, w / beta
    return np.array(alphas), np.array(betas)


def cheb_filter(H, X, m: int, a: float, b: float, a0: float):
    """Degree-m scaled Chebyshev filter damping [a, b] and amplifying below a.
    e = (b-a)/2, c = (b+a)/2, sigma_1 = e/(a0-c);
    Y_1 = (sigma_1/e)(H - c) X;  sigma_{k+1} = 1/(2/sigma_1 - sigma_k);
    Y_{k+1} = (2 sigma_{k+1}/e)(H - c) Y_k - sigma_k sigma_{k+1} Y_{k-1}."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma = e / (a0 - c)
    sigma1 = sigma
    Y_prev = X
    Y = (H @ X - c * X) * (sigma1 / e)
    for _ in range(2, m + 1):
        sigma_new = 1.0 / (2.0 / sigma1 - sigma)
        Y_new = (H @ Y - c * Y) * (2.0 * sigma_new / e) - (sigma * sigma_new) * Y_prev
        Y_prev, Y, sigma = Y, Y_new, sigma_new
    return Y


def chol_gs(X):
    """Cholesky-Gram-Schmidt: S = X^H X = L L^H (L lower, positive diagonal),
    returns X L^{-H}, whose columns are orthonormal and span the same space."""
    S = X.conj().T @ X
    L = np.linalg.cholesky(S)
    return sla.solve_triangular(L, X.conj().T, lower=True).conj().T


def rayleigh_ritz(H, X):
    """Ritz pairs of H on the orthonormal block X: H_p = X^H H X (lower triangle
    used), H_p = Q diag(theta) Q^H ascending; returns theta, X Q and the
    residual norms ||H x_i - theta_i x_i||."""
    HX = H @ X
    Hp = X.conj().T @ HX
    theta, Q = np.linalg.eigh(Hp, UPLO="L")
    Xn = X @ Q
    HXn = HX @ Q
    r = np.linalg.norm(HXn - Xn * theta[None, :], axis=0)
    return theta, Xn, r


def run(H, X0, degree: int, passes: int, block: int, b: float, history=None):
    """Prologue (CholGS + RR on X0), then `passes` x [filter each block of
    `block` columns with (a, b, a0) = (max theta, b, min theta) of the previous
    RR; CholGS; RR].  Returns (theta, X, resid)."""
    X = chol_gs(X0)
    theta, X, r = rayleigh_ritz(H, X)
    if history is not None:
        history.append((theta.copy(), r.copy(), None))
    for _ in range(passes):
        a, a0 = float(theta[-1]), float(theta[0])
        X = X.copy()
        for s in range(0, X.shape[1], block):
            X[:, s:s + block] = cheb_filter(H, X[:, s:s + block], degree, a, b, a0)
        X = chol_gs(X)
        theta, X, r = rayleigh_ritz(H, X)
        if history is not None:
            history.append((theta.copy(), r.copy(), (a, b, a0)))
    return theta, X, r


def sin_largest_angle(U, V):
    """sin of the largest principal angle between span(U) and span(V)
    (both with orthonormal columns, same count)."""
    P = U - V @ (V.conj().T @ U)
    return float(np.linalg.norm(P, 2))
