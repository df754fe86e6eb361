"""Oracle pins for the adjoint: central finite differences of the oracle's own
operator and filter, and the density/magnetisation closed form (eqn:rho,
eqn:mag; the stationarity relations of the appendix on the generalised
functional give dE/dV = rho and dE/dB = m)."""
import numpy as np
import pytest

import synth
from oracle import adjoint as adj, chfsi as och, hamiltonian as ham


@pytest.fixture(scope="module")
def sysop():
    s = synth.make_system("adj", n_cells=(2, 2, 3), box=(4.0, 4.0, 5.0), p=2, n_atoms=1, lmax=1,
                          rcut_sigmas=5.0, kpts=[(0.1, -0.2, 0.05)], n_vec=3)
    mesh, H, MD, V, B = ham.build(s, synth.veff, synth.bxc)
    return s, mesh, H, MD, V, B


def _H(s, V, B):
    return ham.build(s, synth.veff, synth.bxc, V=V, B=B)[1]


def test_density_closed_form_by_finite_differences(sysop):
    s, mesh, H, MD, V, B = sysop
    rng = np.random.default_rng(0)
    X = rng.normal(size=(s.n_dof, 3)) + 1j * rng.normal(size=(s.n_dof, 3))
    rho, m = adj.density_magnetisation(mesh, MD, X)
    wJ = mesh.wq * mesh.J
    dV, dB = adj.cross_density(mesh, MD, X, X)
    assert np.allclose(dV, wJ * rho) and np.allclose(dB, wJ[None, :, None] * m)
    # |m| <= rho pointwise for any spinor set
    assert np.all(np.linalg.norm(m, axis=-1) <= rho * (1 + 1e-12))

    def L(Vp, Bp):
        Hp = _H(s, Vp, Bp)
        return float(np.real(np.sum(X.conj() * (Hp @ X))))
    h = 1e-6
    dVd = rng.normal(size=V.shape)
    fd = (L(V + h * dVd, B) - L(V - h * dVd, B)) / (2 * h)
    an = float(np.sum(wJ * rho * dVd))
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an))
    dBd = rng.normal(size=B.shape)
    fd = (L(V, B + h * dBd) - L(V, B - h * dBd)) / (2 * h)
    an = float(np.sum(wJ[None, :, None] * m * dBd))
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an))


def test_filter_backward_by_finite_differences(sysop):
    s, mesh, H, MD, V, B = sysop
    rng = np.random.default_rng(1)
    X = rng.normal(size=(s.n_dof, 3)) + 1j * rng.normal(size=(s.n_dof, 3))
    lam = np.linalg.eigvalsh(H.toarray())
    m, a, b, a0 = 5, float(lam[20]), float(lam[-1] + 1), float(lam[0])

    def L(Xp, Vp, Bp):
        Y = och.cheb_filter(_H(s, Vp, Bp), Xp, m, a, b, a0)
        return float(np.sum(np.abs(Y) ** 2))
    Y = och.cheb_filter(H, X, m, a, b, a0)
    Xbar, dV, dB = adj.filter_backward(H, mesh, MD, X, 2 * Y, m, a, b, a0)
    h = 1e-6
    D = rng.normal(size=X.shape) + 1j * rng.normal(size=X.shape)
    fd = (L(X + h * D, V, B) - L(X - h * D, V, B)) / (2 * h)
    an = float(np.real(np.vdot(Xbar, D)))
    assert abs(fd - an) < 1e-6 * abs(an)
    dVd = rng.normal(size=V.shape)
    fd = (L(X, V + h * dVd, B) - L(X, V - h * dVd, B)) / (2 * h)
    an = float(np.sum(dV * dVd))
    assert abs(fd - an) < 1e-6 * abs(an)
    dBd = rng.normal(size=B.shape)
    fd = (L(X, V, B + h * dBd) - L(X, V, B - h * dBd)) / (2 * h)
    an = float(np.sum(dB * dBd))
    assert abs(fd - an) < 1e-6 * abs(an)
    # Xbar = p(H)^2 X for this loss (p(H) is Hermitian)
    assert np.abs(Xbar - 2 * och.cheb_filter(H, Y, m, a, b, a0)).max() < 1e-10 * np.abs(Xbar).max()
