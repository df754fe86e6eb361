"""Oracle pins for the densities and the Fermi-Dirac occupations (eqn:rho,
eqn:mag; Fermi-Dirac smearing of Sec. V with the entropy term of Sec. II.B)."""
import math

import numpy as np

import synth
from oracle import density as od, hamiltonian as ham


def test_fermi_function_symmetry_and_range():
    kT = 1e-3
    x = np.array([-1e4, -3.0, -1e-3, 0.0, 1e-3, 3.0, 1e4])
    f = od.fermi_function(x, 0.0, kT)
    assert np.all(np.isfinite(f)) and np.all((f >= 0) & (f <= 1))
    assert f[3] == 0.5
    assert np.allclose(f + f[::-1], 1.0, atol=1e-15)     # f(mu + x) + f(mu - x) = 1
    assert np.all(np.diff(f) <= 0)                        # decreasing in eps


def test_fermi_dirac_two_level_closed_form():
    # two levels symmetric about 0 with one electron: mu = 0 by symmetry and
    # f = 1 / (1 + exp(-/+ 1/kT))
    kT = 0.3
    f, mu, _ = od.fermi_dirac([-1.0, 1.0], 1.0, kT)
    assert abs(mu) < 1e-13
    assert abs(f[0] - 1.0 / (1.0 + math.exp(-1.0 / kT))) < 1e-14
    assert abs(f.sum() - 1.0) < 1e-14


def test_fermi_dirac_count_weights_and_grand_potential():
    rng = np.random.default_rng(3)
    eps = np.sort(rng.uniform(-1.0, 1.0, size=40))
    w = rng.uniform(0.1, 1.0, size=40)
    kT = 500 * od.KELVIN_TO_HA
    n_e = 0.37 * w.sum()
    f, mu, ent = od.fermi_dirac(eps, n_e, kT, w)
    assert abs((w * f).sum() - n_e) < 1e-12 * n_e
    assert ent <= 0.0
    # grand potential: sum w f eps + E_ent - mu N = -kT sum w ln(1 + exp(-(eps - mu)/kT))
    x = (eps - mu) / kT
    omega = -kT * np.sum(w * (np.maximum(-x, 0) + np.log1p(np.exp(-np.abs(x)))))
    lhs = (w * f * eps).sum() + ent - mu * n_e
    assert abs(lhs - omega) < 1e-12 * max(1.0, abs(omega))


def test_fermi_dirac_cold_limit_is_a_step():
    eps = np.array([0.0, 0.1, 0.2, 0.3, 0.4])
    f, mu, ent = od.fermi_dirac(eps, 3.0, 1e-5)
    assert np.allclose(f, [1, 1, 1, 0, 0], atol=1e-12)
    assert 0.2 < mu < 0.3 and abs(ent) < 1e-12


def _gll_system():
    return synth.make_system("dens", n_cells=(2, 2, 3), box=(4.0, 4.0, 5.0), p=3, quad="gll", n_atoms=1,
                             lmax=1, rcut_sigmas=5.0, n_vec=6)


def test_density_integral_equals_occupation_sum_in_gll_mode():
    # with GLL collocation the quadrature weights at the nodes are the lumped mass,
    # so the integral of rho is sum_n f_n x_n^H x_n exactly
    s = _gll_system()
    mesh = ham.mesh_for(s)
    MD = mesh.lumped_mass()
    X = np.linalg.qr(synth.start_block(s, s.n_dof))[0]
    f = np.array([1.0, 1.0, 0.7, 0.3, 0.05, 0.0])
    rho, m = od.density_magnetisation(mesh, MD, X, f)
    integral = float(np.sum(mesh.wq[None, :] * mesh.J * rho))
    assert abs(integral - f.sum()) < 1e-12
    assert np.all(np.linalg.norm(m, axis=-1) <= rho * (1 + 1e-12) + 1e-300)


def test_density_of_a_uniform_spinor():
    # u(r) = c chi everywhere: rho = |c|^2, m = |c|^2 (chi^H sigma chi), a unit Bloch vector
    s = _gll_system()
    mesh = ham.mesh_for(s)
    MD = mesh.lumped_mass()
    chi = np.array([np.cos(0.4), np.exp(0.9j) * np.sin(0.4)])
    c = 0.3
    X = np.zeros((s.n_dof, 1), dtype=np.complex128)
    X[0::2, 0] = c * chi[0] * np.sqrt(MD)
    X[1::2, 0] = c * chi[1] * np.sqrt(MD)
    rho, m = od.density_magnetisation(mesh, MD, X, [2.0])
    bloch = np.array([np.sin(0.8) * np.cos(0.9), np.sin(0.8) * np.sin(0.9), np.cos(0.8)])
    assert np.allclose(rho, 2.0 * c * c, atol=1e-14)
    assert np.allclose(m, 2.0 * c * c * bloch[None, None, :], atol=1e-14)


def test_density_at_cells_agrees_with_the_whole_mesh_form():
    s = synth.make_system("dens2", n_cells=(2, 3, 2), box=(4.0, 5.0, 4.0), p=3, n_atoms=1, lmax=1,
                          rcut_sigmas=5.0, n_vec=4)
    mesh = ham.mesh_for(s)
    MD = mesh.lumped_mass()
    X = synth.random_block(2, s.n_dof, 4)
    f = [1.0, 0.5, 0.25, 0.0]
    rho, m = od.density_magnetisation(mesh, MD, X, f)
    cells = [0, 5, 11]
    rc, mc = od.density_at_cells(mesh, MD, lambda r: X[r], cells, f)
    assert np.allclose(rc, rho[cells], rtol=0, atol=1e-13 * rho.max())
    assert np.allclose(mc, m[cells], rtol=0, atol=1e-13 * rho.max())
