"""Oracle pins for the eigensolver steps (paper Sec. III.B.2: eqn:chebfilt,
the spectral bounds and the Rayleigh-Ritz projection)."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import synth
from oracle import chfsi, hamiltonian as ham


@pytest.fixture(scope="module")
def small():
    s = synth.make_system("small", n_cells=(2, 2, 2), box=(5.0, 5.0, 5.0), p=3,
                          n_atoms=2, lmax=1, rcut_sigmas=5.0, n_vec=24, degree=8)
    _, H, _, _, _ = ham.build(s, synth.veff, synth.bxc)
    A = H.toarray()
    w, U = np.linalg.eigh(A)
    return s, H, A, w, U


def _T(m, x):
    return npcheb.chebval(x, [0] * m + [1])


def test_filter_on_exact_eigenvectors(small):
    """Filtering an eigenvector v (eigenvalue lam) returns
    T_m((lam - c)/e) / T_m((a0 - c)/e) v."""
    s, H, A, w, U = small
    a, b, a0 = w[20], w[-1] + 0.5, w[0]
    e, c = (b - a) / 2, (b + a) / 2
    idx = [0, 3, 10, 19, 25, 60, len(w) - 1]
    Y = chfsi.cheb_filter(H, U[:, idx], 11, a, b, a0)
    for j, i in enumerate(idx):
        f = _T(11, (w[i] - c) / e) / _T(11, (a0 - c) / e)
        assert np.abs(Y[:, j] - f * U[:, i]).max() < 1e-10 * max(1.0, abs(f))
    # inside [a, b] the filter damps by at least 1/|T_m((a0-c)/e)|
    assert all(abs(_T(11, (w[i] - c) / e)) <= 1 + 1e-12 for i in idx if w[i] >= a)


def test_lanczos_bound(small):
    s, H, A, w, U = small
    v0 = synth.lanczos_start(s, A.shape[0])
    lo, hi = chfsi.lanczos_bounds(H, v0, 40)
    assert hi >= w[-1]
    assert hi <= w[-1] + 0.5 * (w[-1] - w[0])     # an upper bound, not a wild one
    assert lo >= w[0] - 1e-12


def test_cholgs(small):
    s, H, A, w, U = small
    rng = np.random.default_rng(0)
    X = rng.normal(size=(A.shape[0], 12)) + 1j * rng.normal(size=(A.shape[0], 12))
    Q = chfsi.chol_gs(X)
    assert np.abs(Q.conj().T @ Q - np.eye(12)).max() < 1e-13
    # same span; upper-triangular relation X = Q R with positive real diagonal
    R = Q.conj().T @ X
    assert np.abs(np.tril(R, -1)).max() < 1e-12
    assert np.all(np.diag(R).real > 0) and np.abs(np.diag(R).imag).max() < 1e-12
    assert np.abs(Q @ R - X).max() < 1e-12
    # an already orthonormal block is returned unchanged
    assert np.abs(chfsi.chol_gs(Q) - Q).max() < 1e-13


def test_rayleigh_ritz(small):
    s, H, A, w, U = small
    idx = [2, 5, 7, 30]
    rng = np.random.default_rng(1)
    G = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))[0]
    th, X, r = chfsi.rayleigh_ritz(H, U[:, idx] @ G)          # invariant subspace
    assert np.allclose(th, w[idx], atol=1e-12)
    assert r.max() < 1e-11
    # Courant-Fischer on a random subspace: theta_i >= lambda_i, and |theta_i - lambda_j| <= r_i
    Xr = chfsi.chol_gs(rng.normal(size=(A.shape[0], 10)) + 1j * rng.normal(size=(A.shape[0], 10)))
    th, X, r = chfsi.rayleigh_ritz(H, Xr)
    assert np.all(th >= w[:10] - 1e-12)
    for i in range(10):
        assert np.min(np.abs(w - th[i])) <= r[i] + 1e-12


def test_chfsi_converges_to_dense_eigenpairs(small):
    s, H, A, w, U = small
    X0 = synth.start_block(s, A.shape[0])
    _, b = chfsi.lanczos_bounds(H, synth.lanczos_start(s, A.shape[0]), 40)
    th, X, r = chfsi.run(H, X0, 8, 60, s.block, b)
    nconv = 16
    assert np.abs(th[:nconv] - w[:nconv]).max() < 1e-10
    assert chfsi.sin_largest_angle(X[:, :nconv], U[:, :nconv]) < 1e-8


def test_tiny_config_converges_to_dense():
    """The tiny workload (3^3 cells, p=4, N=32) run to convergence matches the
    dense eigendecomposition of the 3456 x 3456 H_hat to 1e-10 Ha."""
    s = synth.config("tiny")
    _, H, _, _, _ = ham.build(s, synth.veff, synth.bxc)
    w = np.linalg.eigvalsh(H.toarray())
    X0 = synth.start_block(s, s.n_dof)
    _, b = chfsi.lanczos_bounds(H, synth.lanczos_start(s, s.n_dof), 40)
    th, X, r = chfsi.run(H, X0, s.degree, 40, s.block, b)
    assert np.abs(th[:24] - w[:24]).max() < 1e-10
