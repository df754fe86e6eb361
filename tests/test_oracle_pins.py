"""Pins of the oracle's kinetic normalisation, Jacobian, k-term sign and
projector Bloch phase against closed forms of the continuum problem
(eqn:FEHloc with its k-terms, eqn:HnlocPeriodic, eqn:CMat):

* free electrons (V = 0, B = 0) at a general k: the FE levels converge to
  (1/2)|k + G|^2 (each twice, spin) under p-refinement;
* the interpolant of the plane wave exp(i G.r) has the Rayleigh quotient
  U^H H U / U^H M_D U -> (1/2)|k + G|^2, which fixes the sign of the -i k.grad
  term (the level set alone is symmetric under k -> -k);
* for Gaussian projectors the FE projection of a plane wave converges to the
  Fourier transform  sum_I conj(P[I, chi]) exp(i G.r_I) -> exp(i (k+G).R) p~_chi(k+G),
  p~(q) = int exp(i q.t) p(t) dt (closed form for Gaussian s and p functions),
  which fixes the sign of the Bloch phase exp(-i k.(r - L)) relative to the
  k-term.

Each pin is also run against a copy of the oracle with one planted mistake
(the 1/2, the 2/h Jacobian, the k-term sign, the phase sign) to show that the
pin catches it."""
import math

import numpy as np
import pytest

import synth
from oracle import fe, hamiltonian as ham, projectors

K_GEN = np.array([0.3, -0.2, 0.1])


def _free_local(mesh, k):
    nq3 = mesh.nq ** 3
    V = np.zeros((mesh.n_cell_total, nq3))
    B = np.zeros((mesh.n_cell_total, nq3, 3))
    return ham.assemble_local(mesh, V, B, k)


def _analytic_levels(box, k, n):
    r = range(-4, 5)
    g = [0.5 * np.sum((k + 2 * np.pi * np.array([a / box[0], b / box[1], c / box[2]])) ** 2)
         for a in r for b in r for c in r]
    g = np.sort(np.repeat(g, 2))
    return g[:n], g[n] - g[n - 1]


def level_errors(quad, p, k=K_GEN, box=(4.0, 4.5, 5.0), n=40):
    """max |eps_i - (1/2)|k+G|^2_i| over the n lowest levels of the free-electron operator."""
    m = fe.Mesh((2, 2, 2), box, p, quad, p + 1)
    H = ham.Operator(_free_local(m, k), [], m.lumped_mass())
    w = np.linalg.eigvalsh(H.loc.toarray())[:n]
    ex, gap = _analytic_levels(box, k, n)
    assert gap > 0.05          # the n-th and (n+1)-th analytic levels are separated
    return float(np.abs(w - ex).max())


G_LIST = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (1, 1, 0), (1, -1, 1), (2, 0, -1)]


def plane_wave_quotients(quad, p, k=np.array([0.3, -0.2, 0.25]), box=(5.0, 6.0, 7.0)):
    """[(R_G, (1/2)|k+G|^2, (1/2)|G-k|^2)] for the interpolated plane waves of G_LIST."""
    m = fe.Mesh((3, 3, 3), box, p, quad, p + 1)
    Hl = _free_local(m, k)
    MD = m.lumped_mass()
    r = m.node_coords()
    out = []
    for n in G_LIST:
        G = 2 * np.pi * np.asarray(n) / np.asarray(box)
        u = np.exp(1j * (r @ G))
        U = np.kron(u, np.array([1.0, 0.0]))
        R = np.vdot(U, Hl @ U).real / np.vdot(u, MD * u).real
        out.append((R, 0.5 * np.sum((k + G) ** 2), 0.5 * np.sum((G - k) ** 2)))
    return np.array(out)


def gaussian_ft(atom, q):
    """p~_chi(q) = int exp(i q.t) p_chi(t) dt for the l <= 1 Gaussian projectors
    (s: c_0 Y_00 (2 pi s^2)^{3/2} exp(-s^2 q^2/2); p_d: the q_d-derivative form
    i s^2 q_d times the same Gaussian with c_1 sqrt(3/(4 pi)))."""
    s = atom.sigma
    g = (2 * np.pi * s * s) ** 1.5 * np.exp(-0.5 * s * s * (q @ q))
    c0 = math.sqrt(2.0 / (math.gamma(1.5) * s ** 3)) * 0.5 / math.sqrt(math.pi)
    out = [c0 * g]
    if atom.lmax >= 1:
        c1 = math.sqrt(2.0 / (math.gamma(2.5) * s ** 5)) * math.sqrt(3.0 / (4.0 * math.pi))
        out += [c1 * 1j * s * s * q[d] * g for d in range(3)]
    return np.array(out)


PW_ATOM = synth.Atom((1.3, 2.1, 0.7), 1, 0.9, 7.2, (1.0, 0.5), 0.05)


def projection_errors(quad, p, k=np.array([0.3, -0.2, 0.25]), box=(5.0, 6.0, 7.0), atom=PW_ATOM):
    """(max |P^H u_G - exp(i(k+G).R) p~(k+G)|, min over G of the same expected value's
    distance to the flipped-phase value exp(i(G-k).R) p~(G-k), max |expected|)."""
    m = fe.Mesh((3, 3, 3), box, p, quad, p + 1)
    P = ham.projector_matrix(m, atom, k, box)
    r = m.node_coords()
    R = np.asarray(atom.pos)
    err, sep, scale = 0.0, np.inf, 0.0
    for n in [(0, 0, 0)] + G_LIST[:6]:
        G = 2 * np.pi * np.asarray(n) / np.asarray(box)
        c = P.conj().T @ np.exp(1j * (r @ G))
        ex = np.exp(1j * ((k + G) @ R)) * gaussian_ft(atom, k + G)
        flip = np.exp(1j * ((G - k) @ R)) * gaussian_ft(atom, G - k)
        err = max(err, float(np.abs(c - ex).max()))
        sep = min(sep, float(np.abs(ex - flip).max()))
        scale = max(scale, float(np.abs(ex).max()))
    return err, sep, scale


# ---------------------------------------------------------------- the pins
@pytest.mark.parametrize("quad", ["gl", "gll"])
def test_free_electron_levels_converge_to_half_k_plus_G_squared(quad):
    errs = [level_errors(quad, p) for p in (3, 4, 5)]
    print(f"[free electron {quad}] max level error p=3,4,5: {errs}")
    assert errs[1] < errs[0] / 20 and errs[2] < errs[1] / 20
    assert errs[2] < 1e-4


@pytest.mark.parametrize("quad", ["gl", "gll"])
def test_plane_wave_rayleigh_quotient_fixes_k_term_sign(quad):
    errs = []
    for p in (4, 5, 6):
        o = plane_wave_quotients(quad, p)
        errs.append(float(np.abs(o[:, 0] - o[:, 1]).max()))
    sep = float(np.abs(o[:, 1] - o[:, 2]).min())
    print(f"[plane waves {quad}] max |R - |k+G|^2/2| p=4,5,6: {errs}; |k+G|^2/2 vs |G-k|^2/2 >= {sep:.3f}")
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10
    assert errs[2] < 2e-5 and sep > 1e4 * errs[2]


@pytest.mark.parametrize("quad", ["gl", "gll"])
def test_projector_plane_wave_projection_fixes_bloch_phase(quad):
    errs = []
    for p in (4, 5, 6):
        e, sep, scale = projection_errors(quad, p)
        errs.append(e)
    print(f"[projector phase {quad}] max error p=4,5,6: {errs}; flipped phase differs by >= {sep:.3f} "
          f"(scale {scale:.3f})")
    assert errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5
    assert errs[2] < 1e-4 * scale and sep > 1e3 * errs[2]


# ---------------------------------------------------------------- planted mistakes
def test_pins_catch_a_wrong_kinetic_factor(monkeypatch):
    orig = ham.cell_reference_matrices
    monkeypatch.setattr(ham, "cell_reference_matrices", lambda m, k: (lambda K, Mc, C: (2 * K, Mc, C))(*orig(m, k)))
    assert level_errors("gl", 5) > 0.1


def test_pins_catch_a_wrong_jacobian(monkeypatch):
    orig_init = fe.Mesh.__init__

    def init(self, *a, **kw):
        orig_init(self, *a, **kw)
        self.dNt[1] = 0.5 * self.dNt[1]      # the y Jacobian factor 2/h_y halved
    monkeypatch.setattr(fe.Mesh, "__init__", init)
    assert level_errors("gl", 5) > 0.1


def test_pins_catch_a_flipped_k_term(monkeypatch):
    orig = ham.cell_reference_matrices
    monkeypatch.setattr(ham, "cell_reference_matrices", lambda m, k: (lambda K, Mc, C: (K, Mc, -C))(*orig(m, k)))
    # the free-electron level set is symmetric under k -> -k and cannot see it ...
    assert level_errors("gl", 5) < 1e-4
    # ... the plane-wave quotients do
    o = plane_wave_quotients("gl", 5)
    assert np.abs(o[:, 0] - o[:, 1]).max() > 0.1


def test_pins_catch_a_flipped_bloch_phase(monkeypatch):
    orig = projectors.bloch_projector

    def flipped(atom, pts, k, box):
        return np.conj(orig(atom, pts, k, box))   # exp(+i k.(r - L)) p (p real)
    monkeypatch.setattr(projectors, "bloch_projector", flipped)
    e, sep, scale = projection_errors("gl", 5)
    assert e > 0.1 * scale
