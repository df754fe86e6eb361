"""Oracle pins for the assembled operator (paper eqn:FEHloc, eqn:FEHnloc,
eqn:CMat, eqn:OvlapMap, eqn:GHEP) and the synthetic SOC projectors
(eqn:nlOP; the cell form Delta_{2chi+a,2chi'+b} = D^{chi chi'}_{ab})."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import fe, hamiltonian as ham, projectors
from closed_forms import periodic_1d as _periodic_1d


def _const_fields(mesh, v0=0.0, bvec=(0.0, 0.0, 0.0)):
    nq3 = mesh.nq ** 3
    V = np.full((mesh.n_cell_total, nq3), v0)
    B = np.tile(np.asarray(bvec, dtype=float), (mesh.n_cell_total, nq3, 1))
    return V, B


def _op(mesh, V, B, k, atoms=(), box=None):
    Hloc = ham.assemble_local(mesh, V, B, k)
    projs = ham.spinor_projectors(mesh, list(atoms), k, mesh.box if box is None else box)
    return ham.Operator(Hloc, projs, mesh.lumped_mass())


# ---------------------------------------------------------------- structure
def test_hermitian_with_k_soc_and_field():
    s = synth.make_system("t", n_cells=(2, 3, 2), box=(5.0, 6.0, 5.5), p=3,
                          kpts=[(0.21, -0.13, 0.07)], n_atoms=2, lmax=2, rcut_sigmas=6.0)
    mesh, H, MD, V, B = ham.build(s, synth.veff, synth.bxc)
    A = H.toarray()
    assert np.abs(A - A.conj().T).max() <= 1e-13 * np.abs(A).max()


def test_kinetic_annihilates_constants_and_k_term_antisymmetric():
    m = fe.Mesh((2, 3, 2), (4.0, 5.0, 4.5), 3, "gl", 5)
    K, Mc, C = ham.cell_reference_matrices(m, np.array([0.3, -0.2, 0.5]))
    assert np.abs(K.sum(axis=1)).max() < 1e-13 * np.abs(K).max()
    assert np.abs(C.sum(axis=1)).max() < 1e-13 * np.abs(C).max()     # k.grad(1) = 0
    # global k-gradient matrix is antisymmetric on the periodic mesh (integration by parts)
    rows, cols, vals = [], [], []
    for e in range(m.n_cell_total):
        g = m.cell_nodes(e)
        rows.append(np.repeat(g, g.size)); cols.append(np.tile(g, g.size)); vals.append(C.ravel())
    Cg = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(m.n_nodes, m.n_nodes)).toarray()
    assert np.abs(Cg + Cg.T).max() < 1e-13 * np.abs(Cg).max()
    # consistent-mass row sums equal the lumped (GLL) mass
    rows, cols, vals = [], [], []
    for e in range(m.n_cell_total):
        g = m.cell_nodes(e)
        rows.append(np.repeat(g, g.size)); cols.append(np.tile(g, g.size)); vals.append(Mc.ravel())
    Mg = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(m.n_nodes, m.n_nodes))
    assert np.allclose(np.asarray(Mg.sum(axis=1)).ravel(), m.lumped_mass(), rtol=1e-13)


@pytest.mark.parametrize("quad", ["gl", "gll"])
def test_free_electron_constant_mode_exact(quad):
    """-(1/2)(grad + ik)^2 + v0 + B.sigma on a constant spinor aligned with +-B:
    eigenvalue |k|^2/2 + v0 +- |B| exactly, the lowest level for small k."""
    k = np.array([0.12, -0.05, 0.2])
    m = fe.Mesh((3, 2, 3), (4.0, 3.0, 4.5), 3, quad, 4)
    bvec = np.array([0.03, -0.04, 0.12])
    V, B = _const_fields(m, -0.7, bvec)
    H = _op(m, V, B, k)
    bmag = np.linalg.norm(bvec)
    sqM = np.sqrt(m.lumped_mass())
    for sgn in (+1, -1):
        # spinor eigenvector of b.sigma with eigenvalue sgn
        bs = sum(bvec[d] / bmag * projectors.PAULI[d] for d in range(3))
        w, U = np.linalg.eigh(bs)
        chi = U[:, np.argmin(np.abs(w - sgn))]
        x = np.kron(sqM, chi)
        y = H @ x[:, None]
        lam = 0.5 * k @ k - 0.7 + sgn * bmag
        assert np.abs(y[:, 0] - lam * x).max() < 1e-12 * np.abs(x).max() * 10
    ev = np.linalg.eigvalsh(H.toarray())
    assert abs(ev[0] - (0.5 * k @ k - 0.7 - bmag)) < 1e-11


def test_gll_mode_separable_spectrum_with_k_field_and_shift():
    """In GLL collocation the 3-D operator is a Kronecker sum of 1-D operators:
    its spectrum is every sum of three 1-D eigenvalues; a uniform B splits
    every level by exactly +-|B| and a constant V shifts every level."""
    nc, L, p = (3, 2, 4), (4.0, 3.0, 5.0), 3
    k = np.array([0.11, -0.23, 0.05])
    m = fe.Mesh(nc, L, p, "gll")
    v0, bvec = 0.4, np.array([0.0, 0.05, 0.02])
    V, B = _const_fields(m, v0, bvec)
    ev3 = np.linalg.eigvalsh(_op(m, V, B, k).toarray())
    e1 = [np.linalg.eigvalsh(_periodic_1d(nc[d], L[d], p, k[d])) for d in range(3)]
    sums = (e1[0][:, None, None] + e1[1][None, :, None] + e1[2][None, None, :]).ravel() + v0
    bmag = np.linalg.norm(bvec)
    expect = np.sort(np.concatenate([sums + bmag, sums - bmag]))
    assert np.abs(ev3 - expect).max() < 1e-11 * np.abs(expect).max()


# ---------------------------------------------------------------- projectors
def _sphere_int(a, b, c):
    if a % 2 or b % 2 or c % 2:
        return 0.0
    g = math.gamma
    return 2 * g((a + 1) / 2) * g((b + 1) / 2) * g((c + 1) / 2) / g((a + b + c + 3) / 2)


@pytest.mark.parametrize("l", [0, 1, 2])
def test_real_harmonics_orthonormal_on_sphere(l):
    basis = projectors.real_harmonic_polys(l)
    G = np.zeros((len(basis), len(basis)))
    for i, pa in enumerate(basis):
        for j, pb in enumerate(basis):
            G[i, j] = sum(ca * cb * _sphere_int(ma[0] + mb[0], ma[1] + mb[1], ma[2] + mb[2])
                          for ma, ca in pa.items() for mb, cb in pb.items())
    assert np.allclose(G, np.eye(len(basis)), atol=1e-14)


@pytest.mark.parametrize("l", [1, 2])
def test_angular_momentum_algebra(l):
    Lm = projectors.angular_momentum(l)
    for c in range(3):
        assert np.allclose(Lm[c], Lm[c].conj().T, atol=1e-14)
    L2 = sum(Lm[c] @ Lm[c] for c in range(3))
    assert np.allclose(L2, l * (l + 1) * np.eye(2 * l + 1), atol=1e-13)
    for a, b, c in [(0, 1, 2), (1, 2, 0), (2, 0, 1)]:
        assert np.allclose(Lm[a] @ Lm[b] - Lm[b] @ Lm[a], 1j * Lm[c], atol=1e-13)
    if l == 1:  # (L_c)_{ab} = -i eps_{cab} in the (x, y, z) basis
        eps = np.zeros((3, 3, 3))
        for (i, j, k), s in {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1,
                             (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}.items():
            eps[i, j, k] = s
        assert np.allclose(Lm, -1j * eps, atol=1e-14)


@pytest.mark.parametrize("l", [1, 2])
def test_angular_momentum_acts_on_projector_functions(l):
    """(L_z f)(r) = -i (x d_y - y d_x) f by central differences equals
    sum_m (L_z c)_m p_m for f = sum_m c_m p_m -- independent of the polynomial algebra."""
    atom = synth.Atom((0.0, 0.0, 0.0), l, 0.8, 10.0, (1.0,) * (l + 1), 0.0)
    rng = np.random.default_rng(3)
    r = rng.normal(scale=0.9, size=(40, 3))
    off = sum(2 * j + 1 for j in range(l))
    nl = 2 * l + 1
    cvec = rng.normal(size=nl) + 1j * rng.normal(size=nl)
    Lm = projectors.angular_momentum(l)
    h = 1e-5

    def f(pts):
        return projectors.projector_values(atom, pts)[:, off:off + nl] @ cvec

    for c, (a, b) in enumerate([(1, 2), (2, 0), (0, 1)]):
        eb = np.zeros(3); eb[b] = h
        ea = np.zeros(3); ea[a] = h
        dfb = (f(r + eb) - f(r - eb)) / (2 * h)
        dfa = (f(r + ea) - f(r - ea)) / (2 * h)
        lhs = -1j * (r[:, a] * dfb - r[:, b] * dfa)
        rhs = projectors.projector_values(atom, r)[:, off:off + nl] @ (Lm[c] @ cvec)
        assert np.abs(lhs - rhs).max() < 1e-7 * max(1.0, np.abs(rhs).max())


@pytest.mark.parametrize("l", [0, 1, 2])
def test_projector_normalisation(l):
    """int |p_lm|^2 d^3r = 1 on a fine uniform grid (spectrally accurate for Gaussians)."""
    atom = synth.Atom((0.0, 0.0, 0.0), l, 0.7, 50.0, (1.0,) * (l + 1), 0.0)
    g = np.arange(-6.0, 6.0, 0.07) + 0.035
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    vals = projectors.projector_values(atom, pts)
    off = sum(2 * j + 1 for j in range(l))
    G = vals[:, off:off + 2 * l + 1].T @ vals[:, off:off + 2 * l + 1] * 0.07 ** 3
    assert np.allclose(G, np.eye(2 * l + 1), atol=1e-9)


def test_ls_spectrum():
    for l, (up, dn) in [(1, (0.5, -1.0)), (2, (1.0, -1.5))]:
        atom = synth.Atom((0, 0, 0), l, 1.0, 5.0, tuple([0.0] * (l + 1)), 1.0)
        D = projectors.delta_matrix(atom)
        off = 2 * sum(2 * j + 1 for j in range(l))
        w = np.linalg.eigvalsh(D[off:, off:])
        assert np.allclose(w, np.sort([dn] * (2 * l) + [up] * (2 * l + 2)), atol=1e-13)


def test_isolated_atom_nonlocal_spectrum_4_plus_2():
    """l <= 1 atom at a mesh vertex of a cubic mesh: the nonzero spectrum of
    P Delta P^H is s_0 D0_0 (x2) and s_1 (D0_1 + D_so {+1/2 x4, -1 x2})
    with s_l = ||p_hat_chi||^2 -- the p-shell 4+2 split of the Gamma triplet."""
    m = fe.Mesh((3, 3, 3), (6.0, 6.0, 6.0), 3, "gl", 4)
    atom = synth.Atom((2.0, 4.0, 2.0), 1, 0.6, 2.9, (0.9, 0.4), 0.07)
    (Ps, D), = ham.spinor_projectors(m, [atom], np.zeros(3), m.box)
    s = sp.diags(np.repeat(1 / np.sqrt(m.lumped_mass()), 2))
    Pd = (s @ Ps).toarray()
    G = Pd.conj().T @ Pd
    s0, s1 = G[0, 0].real, G[2, 2].real
    assert np.allclose(G, np.diag(np.repeat([s0, s1, s1, s1], 2)), atol=1e-12 * s1)
    w = np.linalg.eigvalsh(Pd @ D @ Pd.conj().T)
    nz = np.sort(w[np.abs(w) > 1e-10 * s1])
    expect = np.sort([s0 * 0.9] * 2 + [s1 * (0.4 + 0.035)] * 4 + [s1 * (0.4 - 0.07)] * 2)
    assert nz.size == 8
    assert np.allclose(nz, expect, rtol=1e-12)


def test_kramers_degeneracy_and_k_symmetry():
    """Time reversal: at Gamma with B = 0 and SOC on, every level is doubly
    degenerate; with B = 0, eps(k) = eps(-k)."""
    s = synth.make_system("k", n_cells=(2, 2, 3), box=(4.0, 4.0, 5.0), p=3, b_mag=0.0,
                          n_atoms=2, lmax=1, rcut_sigmas=5.0, dso=0.2)
    _, H, _, _, _ = ham.build(s, synth.veff, synth.bxc)
    w = np.linalg.eigvalsh(H.toarray())
    assert np.abs(w[0::2] - w[1::2]).max() < 1e-11
    assert np.min(w[2::2] - w[1:-1:2]) > 1e-6      # pairs, not quartets by accident
    k = np.array([0.2, -0.1, 0.15])
    s2 = synth.make_system("k", n_cells=(2, 2, 3), box=(4.0, 4.0, 5.0), p=3, b_mag=0.0,
                           n_atoms=2, lmax=1, rcut_sigmas=5.0, dso=0.2, kpts=[k, -k])
    wp = np.linalg.eigvalsh(ham.build(s2, synth.veff, synth.bxc, ik=0)[1].toarray())
    wm = np.linalg.eigvalsh(ham.build(s2, synth.veff, synth.bxc, ik=1)[1].toarray())
    assert np.abs(wp - wm).max() < 1e-11
    assert np.abs(wp[0::2] - wp[1::2]).max() > 1e-6    # B=0, k != 0: no Kramers pairing at k


def test_row_sampled_apply_equals_assembled():
    """oracle.rows (for meshes too large to assemble) against the assembled operator."""
    from oracle import rows
    s = synth.make_system("r", n_cells=(3, 2, 3), box=(5.0, 4.0, 5.0), p=3, kpts=[(0.1, 0.05, -0.1)],
                          n_atoms=2, lmax=2, rcut_sigmas=5.0)
    _, H, MD, V, B = ham.build(s, synth.veff, synth.bxc)
    X = synth.random_block(3, s.n_dof, 5)
    ref = H @ X
    nodes = np.array([0, 7, 13, 101, s.n_nodes - 1])
    got = rows.apply_rows(s, nodes, lambda r: X[r], synth.veff, synth.bxc)
    exp = np.stack([ref[2 * nodes], ref[2 * nodes + 1]], axis=1)
    assert np.abs(got - exp).max() < 1e-13 * np.abs(exp).max()
