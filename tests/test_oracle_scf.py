"""Oracle pins for the SCF loop (Sec. III.B eqn:fixedpointmap, eqn:innerPdt,
Anderson mixing with Kerker; Sec. IV.A eqn:FEWfnsCMesh) and the stand-in map
(Hartree with a uniform background, LSDA exchange under the locally collinear
substitution of Sec. II.B)."""
import math

import numpy as np
import pytest

import synth
from oracle import fe, hamiltonian as ham, scf


def _mesh(nc=(3, 3, 3), box=(5.0, 6.0, 5.5), p=4, nq=None):
    return fe.Mesh(nc, box, p, "gl", nq or p + 1)


# ---------------------------------------------------------------- exchange
def test_exchange_closed_forms_and_derivatives():
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.01, 0.3, size=50)
    # unpolarised: V = -(3 rho / pi)^(1/3), B = 0
    V, B, e = scf.exchange(rho, np.zeros((50, 3)))
    assert np.allclose(V, -np.cbrt(3 * rho / np.pi), rtol=1e-14) and np.abs(B).max() == 0.0
    assert np.allclose(e, -0.75 * (3 / np.pi) ** (1 / 3) * rho ** (4 / 3), rtol=1e-14)
    # fully polarised along a coordinate axis (|m| = rho exactly): V = v_up/2, B = (v_up/2) m_hat
    d = np.eye(3)[rng.integers(0, 3, size=50)] * rng.choice([-1.0, 1.0], size=(50, 1))
    V, B, e = scf.exchange(rho, rho[:, None] * d)
    vup = -(6 / np.pi) ** (1 / 3) * np.cbrt(rho)
    assert np.allclose(V, 0.5 * vup, rtol=1e-13) and np.allclose(B, 0.5 * vup[:, None] * d, rtol=1e-12)
    # V = de/drho and B = de/dm by central differences at partial polarisation
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    m = 0.6 * rho[:, None] * d
    V, B, _ = scf.exchange(rho, m)
    h = 1e-6
    fd = (scf.exchange(rho + h, m)[2] - scf.exchange(rho - h, m)[2]) / (2 * h)
    assert np.abs(fd - V).max() < 1e-7
    for c in range(3):
        dm = np.zeros(3)
        dm[c] = h
        fd = (scf.exchange(rho, m + dm)[2] - scf.exchange(rho, m - dm)[2]) / (2 * h)
        assert np.abs(fd - B[:, c]).max() < 1e-7


# ---------------------------------------------------------------- field solves
def _cos_field(m, G, amp=1.0, base=0.0):
    pts = m.all_quad_points()
    return base + amp * np.cos(pts @ G), pts


def test_inner_product_of_constant_fields():
    m = _mesh()
    vol = float(np.prod(m.box))
    E, nq3 = m.n_cell_total, m.nq ** 3
    one = np.ones((E, nq3))
    z = np.zeros((E, nq3, 3))
    mz = np.zeros((E, nq3, 3))
    mz[..., 2] = 2.0
    assert abs(scf.inner(m, one, z, one, z) - 0.5 * vol) < 1e-12 * vol
    assert abs(scf.inner(m, 0 * one, mz, 0 * one, mz) - 2.0 * vol) < 1e-12 * vol


def test_hartree_of_a_cosine_converges_to_4pi_over_G2():
    G = 2 * np.pi * np.array([1 / 5.0, 0.0, 1 / 5.5])
    errs = []
    for p in (3, 4, 5):
        m = _mesh(box=(5.0, 6.0, 5.5), p=p)
        rho, pts = _cos_field(m, G, 0.02, 0.05)
        V = scf.hartree(m, rho)
        ex = 4 * np.pi * 0.02 / (G @ G) * np.cos(pts @ G)
        errs.append(np.abs(V - ex).max() / np.abs(ex).max())
    print(f"[hartree] rel errors p=3,4,5: {errs}")
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4 and errs[2] < 1e-3
    m = _mesh(p=3)
    assert np.abs(scf.hartree(m, np.full((m.n_cell_total, m.nq ** 3), 0.07))).max() < 1e-13


def test_kerker_annihilates_constants_and_damps_long_waves():
    k0 = 0.9
    G = 2 * np.pi * np.array([0.0, 1 / 6.0, 0.0])
    errs = []
    for p in (3, 4, 5):
        m = _mesh(p=p)
        rho, pts = _cos_field(m, G)
        K = scf.kerker(m, rho, k0)
        ex = (G @ G) / (G @ G + k0 * k0) * rho
        errs.append(np.abs(K - ex).max())
    print(f"[kerker] errors p=3,4,5: {errs}")
    assert errs[2] < errs[0] / 10 and errs[2] < 1e-4
    m = _mesh(p=3)
    c = np.full((m.n_cell_total, m.nq ** 3), 0.3)
    assert np.abs(scf.kerker(m, c, k0)).max() < 1e-12
    assert np.array_equal(scf.kerker(m, c, 0.0), c)


# ---------------------------------------------------------------- mixing
def _fields(m, rng, k=1):
    E, nq3 = m.n_cell_total, m.nq ** 3
    return [(rng.normal(size=(E, nq3)), rng.normal(size=(E, nq3, 3))) for _ in range(k)]


def test_anderson_depth_one_is_linear_mixing():
    m = _mesh(p=2)
    rng = np.random.default_rng(2)
    x, f = _fields(m, rng)[0], _fields(m, rng)[0]
    xr, xm, b = scf.anderson_next(m, [x], [f], 0.3, 0.0)
    assert np.allclose(b, [1.0])
    assert np.allclose(xr, x[0] + 0.3 * f[0], rtol=1e-15) and np.allclose(xm, x[1] + 0.3 * f[1], rtol=1e-15)


def test_anderson_finds_the_fixed_point_of_a_linear_map_in_d_plus_1_steps():
    """F(x) = x* + M (x - x*) with M acting on a 3-dimensional subspace that holds
    the initial error: with the history kept whole, the residual vanishes after at
    most 4 evaluations (the affine minimisation spans the error subspace)."""
    m = _mesh(p=2)
    rng = np.random.default_rng(3)
    U = _fields(m, rng, 3)
    xs_star = _fields(m, rng)[0]
    lam = [0.4, -0.7, 1.6]

    def add(a, b, s=1.0):
        return a[0] + s * b[0], a[1] + s * b[1]

    def scale(a, s):
        return s * a[0], s * a[1]

    def apply_M(e):
        out = (0 * e[0], 0 * e[1])
        for li, u in zip(lam, U):
            out = add(out, scale(u, li * scf.inner(m, u[0], u[1], e[0], e[1])))
        return out

    x = add(xs_star, add(scale(U[0], 0.3), add(scale(U[1], -0.2), scale(U[2], 0.5))))
    xs, fs, norms = [], [], []
    for it in range(5):
        e = add(x, xs_star, -1.0)
        f = add(add(xs_star, apply_M(e)), x, -1.0)              # F(x) - x
        norms.append(math.sqrt(scf.inner(m, f[0], f[1], f[0], f[1])))
        if it == 4:
            break
        xs.append(x)
        fs.append(f)
        xr, xm, b = scf.anderson_next(m, xs, fs, 0.5, 0.0)
        assert abs(b.sum() - 1.0) < 1e-13
        x = (xr, xm)
    print(f"[anderson linear] residual norms {norms}")
    assert norms[4] < 1e-10 * norms[0]
    assert norms[1] > 1e-3 * norms[0]          # not a one-step accident


# ---------------------------------------------------------------- two-grid transfer
def test_two_grid_interpolation_keeps_the_coarse_field():
    """The degree-(p-1) field moved to the degree-p nodes is the same piecewise
    polynomial: equal at every quadrature point (same rule on both meshes)."""
    nc, box, nq = (2, 3, 2), (4.0, 5.0, 4.5), 6
    mc = fe.Mesh(nc, box, 3, "gl", nq)
    mf = fe.Mesh(nc, box, 4, "gl", nq)
    rng = np.random.default_rng(4)
    Yc = rng.normal(size=(2 * mc.n_nodes, 3)) + 1j * rng.normal(size=(2 * mc.n_nodes, 3))
    Yf = scf.interpolate_block(mc, mf, Yc)
    Uc = Yc / np.repeat(np.sqrt(mc.lumped_mass()), 2)[:, None]
    Uf = Yf / np.repeat(np.sqrt(mf.lumped_mass()), 2)[:, None]
    for a in range(2):
        for n in range(3):
            qc = scf.interpolate(mc, Uc[a::2, n])
            qf = scf.interpolate(mf, Uf[a::2, n])
            assert np.abs(qc - qf).max() < 1e-13 * np.abs(qc).max()


# ---------------------------------------------------------------- the loop
def _free_system(bvec, p=3):
    s = synth.make_system("ueg", n_cells=(2, 2, 2), box=(4.0, 4.0, 4.0), p=p, n_atoms=0, n_vec=6, degree=8)
    mesh = ham.mesh_for(s)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    vext = np.zeros((E, nq3))
    bext = np.tile(np.asarray(bvec, dtype=float), (E, nq3, 1))
    return s, mesh, vext, bext


def test_scf_reaches_the_polarised_uniform_gas_fixed_point():
    """No atoms, V_ext = 0, uniform B_ext, one electron: the fixed point is the
    constant spinor antiparallel to B_ext, rho = 1/Omega, m = -B_hat/Omega
    (V_H = 0), with lowest level eps_0 = -(6/pi)^(1/3) Omega^(-1/3) - |B_ext|
    (fully polarised exchange: V_x = v_up/2, |B_x| = |v_up|/2 along B_hat)."""
    bvec = np.array([0.03, -0.04, 0.12])
    s, mesh, vext, bext = _free_system(bvec)
    vol = 64.0
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    pts = mesh.all_quad_points()
    rho0 = (1.0 + 0.3 * np.cos(2 * np.pi * pts[..., 0] / 4.0)) / vol
    m0 = np.zeros((E, nq3, 3))
    m0[..., 0] = 0.5 * rho0                    # start polarised along x
    out = scf.scf(s, vext, bext, rho0, m0, 1.0, 1e-3, n_vec=6, degree=8, passes_first=6, passes=2,
                  depth=4, alpha=0.6, k0=0.7, tol=1e-9, max_iter=60)
    norms = [h[1] for h in out["history"]]
    print(f"[scf ueg] {len(norms)} iterations, residual norms {norms[0]:.2e} ... {norms[-1]:.2e}")
    assert out["converged"]
    bhat = bvec / np.linalg.norm(bvec)
    assert np.abs(out["rho_out"] - 1.0 / vol).max() < 1e-8
    assert np.abs(out["m_out"] + bhat[None, None, :] / vol).max() < 1e-8
    eps0 = -(6 / np.pi) ** (1 / 3) * vol ** (-1 / 3) - np.linalg.norm(bvec)
    assert abs(out["theta"][0] - eps0) < 1e-7


def test_scf_two_grid_with_atoms_converges_to_a_fixed_point():
    """Two pseudo-atoms with SOC, synthetic V_ext and B_ext, 5 electrons: degree 2
    until the residual is below 1e-2, then degree 3; at the end the map returns
    its input to the tolerance, and the output charge is the electron count."""
    kw = dict(n_cells=(2, 2, 2), box=(5.0, 5.0, 5.0), n_atoms=2, lmax=1, rcut_sigmas=5.0, n_vec=10,
              degree=8, seed=6)
    fine = synth.make_system("scf", p=3, n_q=5, **kw)
    coarse = synth.make_system("scf", p=2, n_q=5, **kw)
    mesh = ham.mesh_for(fine)
    pts = mesh.all_quad_points().reshape(-1, 3)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    vext = synth.veff(fine, pts).reshape(E, nq3)
    bext = synth.bxc(fine, pts).reshape(E, nq3, 3)
    n_e = 5.0
    rho0 = np.full((E, nq3), n_e / 125.0)
    m0 = 0.2 * bext / 0.1 * rho0[..., None]
    out = scf.scf(fine, vext, bext, rho0, m0, n_e, 500 * 3.166811563e-6, coarse_system=coarse,
                  passes_first=5, passes=2, depth=5, alpha=0.5, k0=0.8, tol=1e-7, tol_coarse=1e-2,
                  max_iter=60)
    h = out["history"]
    print("[scf two-grid] " + " ".join(f"p{g}:{r:.1e}" for g, r, *_ in h))
    assert out["converged"]
    assert h[0][0] == 2 and h[-1][0] == 3
    assert any(g == 2 and r < 1e-2 for g, r, *_ in h)
    assert abs(scf.integrate(mesh, out["rho_out"]) - n_e) < 1e-8
    fr = out["rho_out"] - out["rho_in"]
    fm = out["m_out"] - out["m_in"]
    assert math.sqrt(scf.inner(mesh, fr, fm, fr, fm)) < 1e-7
    # |m| <= rho pointwise
    assert np.all(np.linalg.norm(out["m_out"], axis=-1) <= out["rho_out"] * (1 + 1e-12))


# ---------------------------------------------------------------- Brillouin-zone sampling
def _kpt_system(kpts, seed=3, b_mag=None):
    """Two SOC pseudo-atoms (l <= 1) in a 2^3-cell box, p = 2: small enough for a
    dense diagonalisation per k-point."""
    kw = dict(n_cells=(2, 2, 2), box=(4.5, 4.5, 4.5), p=2, n_q=4, n_atoms=2, lmax=1, rcut_sigmas=5.0,
              n_vec=8, degree=8, seed=seed, kpts=kpts)
    if b_mag is not None:
        kw["b_mag"] = b_mag
    s = synth.make_system("kscf", **kw)
    mesh = ham.mesh_for(s)
    pts = mesh.all_quad_points().reshape(-1, 3)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    return s, mesh, synth.veff(s, pts).reshape(E, nq3), synth.bxc(s, pts).reshape(E, nq3, 3)


def test_scf_duplicated_kpoint_equals_the_single_kpoint():
    """The same k-point listed twice with weights 1/2, 1/2 (and the same start
    block) is the single k-point: history and densities agree to rounding."""
    k = (0.0, 0.0, 0.35)
    s1, mesh, vext, bext = _kpt_system([k])
    s2, _, _, _ = _kpt_system([k, k])
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    n_e = 3.0
    rho0 = np.full((E, nq3), n_e / 4.5 ** 3)
    m0 = 0.1 * rho0[..., None] * np.array([0.0, 0.6, 0.8])
    X0 = synth.random_block(0, s1.n_dof, 8)
    kw = dict(passes_first=5, passes=2, depth=4, alpha=0.5, k0=0.6, tol=1e-8, max_iter=6)
    a = scf.scf(s1, vext, bext, rho0, m0, n_e, 1e-3, X0=X0, **kw)
    b = scf.scf(s2, vext, bext, rho0, m0, n_e, 1e-3, X0=[X0, X0], kweights=[0.5, 0.5], **kw)
    assert len(a["history"]) == len(b["history"])
    for ha, hb in zip(a["history"], b["history"]):
        for i in range(1, 6):
            assert abs(ha[i] - hb[i]) <= 1e-11 * max(1.0, abs(ha[i])), (i, ha[i], hb[i])
    for key in ("rho_out", "m_out", "rho_in", "m_in"):
        assert np.abs(a[key] - b[key]).max() <= 1e-12 * np.abs(a[key]).max()
    assert np.abs(b["occ_k"][0] - b["occ_k"][1]).max() == 0.0


def test_scf_time_reversed_pair_cancels_the_magnetisation():
    """No external field, no input magnetisation, spin-orbit atoms: the pair
    {k, -k} with equal weights gives m = 0 (Kramers partners u_{-k} = i sigma_y
    conj(u_k) carry opposite spin densities) and the charge density of k alone,
    while k alone leaves a spin-orbit magnetisation."""
    k = np.array([0.0, 0.3, 0.45])
    s1, mesh, vext, _ = _kpt_system([tuple(k)])
    s2, _, _, _ = _kpt_system([tuple(k), tuple(-k)])
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    bext = np.zeros((E, nq3, 3))
    n_e = 3.0
    rho0 = np.full((E, nq3), n_e / 4.5 ** 3)
    m0 = np.zeros((E, nq3, 3))
    kw = dict(passes_first=10, passes=2, depth=3, alpha=0.5, k0=0.6, tol=1e-12, max_iter=1)
    one = scf.scf(s1, vext, bext, rho0, m0, n_e, 1e-3, **kw)
    pair = scf.scf(s2, vext, bext, rho0, m0, n_e, 1e-3, **kw)
    rmax = np.abs(pair["rho_out"]).max()
    m_one = np.abs(one["m_out"]).max() / rmax
    m_pair = np.abs(pair["m_out"]).max() / rmax
    d_rho = np.abs(pair["rho_out"] - one["rho_out"]).max() / rmax
    print(f"[scf k,-k] |m|/rho: k alone {m_one:.1e}, pair {m_pair:.1e}; rho difference {d_rho:.1e}")
    assert m_one > 1e-4
    assert m_pair < 1e-9 and d_rho < 1e-9
    occd = pair["occ_k"][0] > 1e-12          # the top of the block is not converged
    assert np.abs(pair["theta_k"][0] - pair["theta_k"][1])[occd].max() < 1e-9


def test_scf_one_iteration_is_the_dense_zone_average():
    """One map evaluation with two k-points of unequal weight against its plain
    definition: dense eigenpairs of each H^k, one Fermi level for all (n, k) with
    sum_k w_k sum_n f_nk = N_e, rho = sum_k w_k sum_n f_nk |u_nk|^2 (and m), scaled
    to N_e under the cell quadrature."""
    from oracle import density as oden
    kpts = [(0.0, 0.0, 0.7), (0.25, 0.0, -0.35)]
    s, mesh, vext, bext = _kpt_system(kpts, seed=5)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    n_e, kT, w = 3.0, 2e-3, np.array([0.3, 0.7])
    rho0 = np.full((E, nq3), n_e / 4.5 ** 3)
    m0 = 0.05 * rho0[..., None] * np.array([0.6, 0.0, 0.8])
    out = scf.scf(s, vext, bext, rho0, m0, n_e, kT, passes_first=12, max_iter=1, tol=1e-14, kweights=w)
    V, B = scf.potentials(mesh, rho0, m0, vext, bext)
    g = scf.Grid(s, s.atoms)
    th, vec = [], []
    for ik in range(2):
        ev, U = np.linalg.eigh(g.operator(V, B, ik).toarray())
        th.append(ev[:8])
        vec.append(U[:, :8])
    eps = np.concatenate(th)
    f, mu, _ = oden.fermi_dirac(eps, n_e, kT, weights=np.repeat(w, 8))
    rho, m = 0.0, 0.0
    for ik in range(2):
        r_k, m_k = oden.density_magnetisation(mesh, g.MD, vec[ik], w[ik] * f[8 * ik:8 * ik + 8])
        rho, m = rho + r_k, m + m_k
    q = n_e / scf.integrate(mesh, rho)
    rho, m = q * rho, q * m
    occd = f.reshape(2, 8) > 1e-12               # the top of the block is not converged
    d_th = np.abs(out["theta_k"] - np.array(th))[occd].max()
    d_rho = np.abs(out["rho_out"] - rho).max() / np.abs(rho).max()
    d_m = np.abs(out["m_out"] - m).max() / np.abs(rho).max()
    print(f"[scf zone average] theta {d_th:.1e}, mu {abs(out['history'][0][2] - mu):.1e}, rho {d_rho:.1e}, m {d_m:.1e}")
    assert d_th < 1e-10 and abs(out["history"][0][2] - mu) < 1e-10
    assert d_rho < 1e-9 and d_m < 1e-9
    assert abs(float(np.dot(w, [np.dot(f[8 * i:8 * i + 8], th[i]) for i in range(2)])) - out["history"][0][3]) < 1e-10
