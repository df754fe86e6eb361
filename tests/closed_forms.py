"""Closed-form reference pieces used by the tests (test infrastructure):
the 1-D periodic spectral-element operator in GLL collocation, whose Kronecker
sum is the 3-D operator of a constant potential and field."""
import numpy as np

from oracle import fe


def periodic_1d(ncell, L, p, k):
    """M^{-1/2} (1/2 K - i k C + k^2/2 M) M^{-1/2} on a periodic 1-D mesh of
    ncell cells of degree p with GLL collocation (M diagonal)."""
    xi, w = fe.gauss_lobatto(p)
    _, D = fe.lagrange_tables(xi, xi)       # D[i, q] = l_i'(xi_q)
    h = L / ncell
    n = ncell * p
    K = np.zeros((n, n)); C = np.zeros((n, n)); M = np.zeros(n)
    for c in range(ncell):
        g = (c * p + np.arange(p + 1)) % n
        Kc = (2 / h) * (D * w) @ D.T
        Cc = np.diag(w) @ D.T
        for a in range(p + 1):
            M[g[a]] += w[a] * h / 2
            for b in range(p + 1):
                K[g[a], g[b]] += Kc[a, b]
                C[g[a], g[b]] += Cc[a, b]
    A = 0.5 * K - 1j * k * C + 0.5 * k * k * np.diag(M)
    s = 1 / np.sqrt(M)
    return s[:, None] * A * s[None, :]
