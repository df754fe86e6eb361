"""GPU parity of the SCF loop (Sec. III.B eqn:fixedpointmap, eqn:innerPdt,
Anderson mixing with Kerker; Sec. IV.A eqn:FEWfnsCMesh) against the oracle's
loop on the same seeded inputs.

Pieces: the eqn:innerPdt product, the Hartree potential (CG on the FE scalar
operator vs the oracle's sparse direct solve), the Kerker preconditioner, the
LSDA exchange, the two-grid block transfer.  Whole loop: the polarised uniform
gas (closed-form fixed point) and a two-grid run with atoms; the per-iteration
record (degree, residual norm, mu, band energy, lowest Ritz value) is compared
with the oracle's history, and the final densities with the oracle's.

Tolerances: field pieces 1e-11 relative (CG to 1e-13 relative residual on
operators of condition number below 1e3; the direct solve is exact to
roundoff); exchange 1e-14 relative; the block transfer 1e-13 relative.  The
loops run with the oracle's filter bounds (its Lanczos runs and the library's
agree only to about 1e-8 relative, and the unconverged part of each iterate
depends on the bound): every record to 1e-6 relative + 1e-11 absolute, the final
densities to 1e-9 relative, the Ritz values to 1e-9 Ha.  With the library's own
Lanczos bounds the loop must reach the same fixed point: densities to 1e-6
relative, occupied Ritz values to 1e-8 Ha, iteration counts within a few.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import fe, hamiltonian as ham, scf

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _op(nc, box, p, nq=None, atoms=(), form="cell", kpts=None):
    from paper_2410_02754_amd import Operator
    op = Operator(nc, box, p, "gl", nq or p + 1, kpts, form=form)
    op.set_atoms(list(atoms))
    return op


def _mesh(nc, box, p, nq=None):
    return fe.Mesh(nc, box, p, "gl", nq or p + 1)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("p,nq", [(3, None), (4, 6)])
def test_inner_hartree_kerker_match_oracle(p, nq):
    nc, box = (3, 2, 3), (5.0, 4.0, 5.5)
    m = _mesh(nc, box, p, nq)
    op = _op(nc, box, p, nq)
    pts = m.all_quad_points()
    rng = np.random.default_rng(11)
    # a smooth positive charge (a few Gaussians) and a random magnetisation
    rho = 0.02 + sum(a * np.exp(-np.sum((pts - c) ** 2, axis=-1) / 1.5)
                     for a, c in zip(rng.uniform(0.1, 0.5, 3), rng.uniform(0, 1, (3, 3)) * np.array(box)))
    mag = 0.3 * rho[..., None] * rng.normal(size=pts.shape)
    r2 = np.cos(pts[..., 0]) * rho
    m2 = rng.normal(size=pts.shape)
    got = op.field_inner(_dev(rho), _dev(mag), _dev(r2), _dev(m2))
    ref = scf.inner(m, rho, mag, r2, m2)
    assert abs(got - ref) <= 1e-13 * abs(ref)
    assert abs(op.field_inner(_dev(rho), None, _dev(r2), None) - scf.inner(m, rho, 0 * mag, r2, 0 * mag)) \
        <= 1e-13 * abs(ref)
    vh = torch.empty_like(_dev(rho))
    it = op.hartree(_dev(rho), vh)
    ref = scf.hartree(m, rho)
    err = np.abs(vh.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say(f"[fields p={p}] Hartree: {it} CG steps, rel err vs oracle {err:.2e}")
    assert it > 0 and err < 1e-11
    for k0 in (0.0, 0.8):
        out = torch.empty_like(vh)
        it = op.kerker(_dev(r2), out, k0)
        ref = scf.kerker(m, r2, k0)
        err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
        _say(f"[fields p={p}] Kerker k0={k0}: {it} CG steps, rel err {err:.2e}")
        assert err < 1e-11
    op.close()


def test_exchange_matches_oracle():
    nc, box, p = (2, 2, 2), (4.0, 4.0, 4.0), 3
    op = _op(nc, box, p)
    shp = (op.n_cells, op.nq3)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.0, 0.4, size=shp)
    mag = rng.normal(size=shp + (3,)) * rho[..., None] * 0.5
    mag[0, :5] = 0.0                                     # m = 0: B_x = 0
    mag[1, :5] = 2.0 * rho[1, :5, None] * np.array([1.0, 0.0, 0.0])   # |m| > rho: clamped spin-down
    vx, bx = torch.empty_like(_dev(rho)), torch.empty_like(_dev(mag))
    op.exchange(_dev(rho), _dev(mag), vx, bx)
    V, B, _ = scf.exchange(rho, mag)
    assert np.abs(vx.cpu().numpy() - V).max() <= 1e-14 * np.abs(V).max()
    assert np.abs(bx.cpu().numpy() - B).max() <= 1e-14 * np.abs(B).max()
    op.close()


def test_block_transfer_matches_oracle():
    from paper_2410_02754_amd import interpolate_block
    nc, box, nq = (2, 3, 2), (4.0, 5.0, 4.5), 6
    mc, mf = _mesh(nc, box, 3, nq), _mesh(nc, box, 4, nq)
    oc, of = _op(nc, box, 3, nq), _op(nc, box, 4, nq)
    rng = np.random.default_rng(4)
    Yc = rng.normal(size=(2 * mc.n_nodes, 5)) + 1j * rng.normal(size=(2 * mc.n_nodes, 5))
    ref = scf.interpolate_block(mc, mf, Yc)
    Yf = torch.empty((of.n_dof, 5), dtype=torch.complex128, device="cuda")
    interpolate_block(oc, of, torch.tensor(Yc, device="cuda"), Yf)
    err = np.abs(Yf.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say(f"[two-grid] block transfer rel err {err:.2e}")
    assert err < 1e-13
    oc.close()
    of.close()


def _compare_history(got, ref, rtol, atol, label):
    assert len(got) == len(ref), (len(got), len(ref))
    worst = 0.0
    for g, r in zip(got, ref):
        p, nres, mu, eb, th0 = r[:5]
        assert g["p"] == p
        d = abs(g["resid"] - nres)
        worst = max(worst, d / (atol + rtol * nres))
        assert d <= atol + rtol * nres, (d, nres)
        for key, val in (("mu", mu), ("band_energy", eb), ("theta0", th0)):
            assert abs(g[key] - val) <= atol + rtol * abs(val), (key, g[key], val)
    _say(f"[{label}] history within {worst:.2f} of the bar (rtol {rtol}, atol {atol})")


def _bounds(ref):
    """The oracle's filter bounds, iteration-major over the k-points."""
    return [b for h in ref for b in h[6]]


def test_scf_uniform_gas_matches_oracle_and_closed_form():
    from paper_2410_02754_amd import scf_run
    bvec = np.array([0.03, -0.04, 0.12])
    s = synth.make_system("ueg", n_cells=(2, 2, 2), box=(4.0, 4.0, 4.0), p=3, n_atoms=0, n_vec=6, degree=8)
    mesh = ham.mesh_for(s)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    vext = np.zeros((E, nq3))
    bext = np.tile(bvec, (E, nq3, 1))
    vol = 64.0
    pts = mesh.all_quad_points()
    rho0 = (1.0 + 0.3 * np.cos(2 * np.pi * pts[..., 0] / 4.0)) / vol
    m0 = np.zeros((E, nq3, 3))
    m0[..., 0] = 0.5 * rho0
    kw = dict(passes_first=6, passes=2, depth=4, alpha=0.6, k0=0.7, tol=1e-9, max_iter=60)
    out = scf.scf(s, vext, bext, rho0, m0, 1.0, 1e-3, n_vec=6, degree=8, **kw)
    op = _op(s.n_cells, s.box, s.p)
    rho, m = _dev(rho0), _dev(m0)
    ro, mo = torch.empty_like(rho), torch.empty_like(m)
    X = torch.empty((op.n_dof, 6), dtype=torch.complex128, device="cuda")
    # the oracle's filter bounds: the two loops see the same operators
    hist, th, occ, conv = scf_run(op, _dev(vext), _dev(bext), rho, m, ro, mo, X, 1.0, 1e-3, 8, seed=0,
                                  lanczos_seed=s.seed + 1, bounds=_bounds(out["history"]), **kw)
    _say(f"[scf ueg] gpu {len(hist)} iterations, residual {hist[-1]['resid']:.2e}; oracle {len(out['history'])}")
    for g, r in zip(hist, out["history"]):
        _say(f"   p{g['p']} gpu {g['resid']:.6e} oracle {r[1]:.6e} d={abs(g['resid'] - r[1]):.1e}")
    assert conv and out["converged"]
    _compare_history(hist, out["history"], 1e-6, 1e-11, "scf ueg")
    # with its own Lanczos bounds the loop reaches the same fixed point
    rho2, m2 = _dev(rho0), _dev(m0)
    ro2, mo2 = torch.empty_like(rho2), torch.empty_like(m2)
    h2, th2, _, conv2 = scf_run(op, _dev(vext), _dev(bext), rho2, m2, ro2, mo2, X, 1.0, 1e-3, 8, seed=0,
                                lanczos_seed=s.seed + 1, **kw)
    _say(f"[scf ueg] own bounds: {len(h2)} iterations, residual {h2[-1]['resid']:.2e}")
    assert conv2 and abs(len(h2) - len(hist)) <= 2
    assert np.abs(ro2.cpu().numpy() - out["rho_out"]).max() <= 1e-8 * np.abs(out["rho_out"]).max()
    bhat = bvec / np.linalg.norm(bvec)
    assert np.abs(ro.cpu().numpy() - 1.0 / vol).max() < 1e-8
    assert np.abs(mo.cpu().numpy() + bhat[None, None, :] / vol).max() < 1e-8
    eps0 = -(6 / np.pi) ** (1 / 3) * vol ** (-1 / 3) - np.linalg.norm(bvec)
    assert abs(th[0] - eps0) < 1e-7
    op.close()


@pytest.mark.parametrize("form,nq", [("cell", 5), ("matrix_free", 4)])
def test_scf_two_grid_with_atoms_matches_oracle(form, nq):
    """The two grids share the quadrature points; with the matrix-free operator on
    the fine grid (n_q = p + 1 = 4) the coarse grid keeps its cell matrices."""
    from paper_2410_02754_amd import scf_run
    kw_sys = dict(n_cells=(2, 2, 2), box=(5.0, 5.0, 5.0), n_atoms=2, lmax=1, rcut_sigmas=5.0, n_vec=10,
                  degree=8, seed=6)
    fine = synth.make_system("scf", p=3, n_q=nq, **kw_sys)
    coarse = synth.make_system("scf", p=2, n_q=nq, **kw_sys)
    mesh = ham.mesh_for(fine)
    pts = mesh.all_quad_points().reshape(-1, 3)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    vext = synth.veff(fine, pts).reshape(E, nq3)
    bext = synth.bxc(fine, pts).reshape(E, nq3, 3)
    n_e, kT = 5.0, 500 * 3.166811563e-6
    rho0 = np.full((E, nq3), n_e / 125.0)
    m0 = 0.2 * bext / 0.1 * rho0[..., None]
    kw = dict(passes_first=5, passes=2, depth=5, alpha=0.5, k0=0.8, tol=1e-7, tol_coarse=1e-2, max_iter=60)
    out = scf.scf(fine, vext, bext, rho0, m0, n_e, kT, coarse_system=coarse, **kw)
    of = _op(fine.n_cells, fine.box, 3, nq, fine.atoms, form)
    oc = _op(coarse.n_cells, coarse.box, 2, nq, coarse.atoms, "cell")
    rho, m = _dev(rho0), _dev(m0)
    ro, mo = torch.empty_like(rho), torch.empty_like(m)
    X = torch.empty((of.n_dof, 10), dtype=torch.complex128, device="cuda")
    hist, th, occ, conv = scf_run(of, _dev(vext), _dev(bext), rho, m, ro, mo, X, n_e, kT, 8, coarse=oc, seed=0,
                                  lanczos_seed=fine.seed + 1, bounds=_bounds(out["history"]), **kw)
    _say(f"[scf two-grid] gpu {len(hist)} iterations; oracle {len(out['history'])}")
    for g, r in zip(hist, out["history"]):
        _say(f"   p{g['p']} gpu {g['resid']:.6e} oracle {r[1]:.6e} d={abs(g['resid'] - r[1]):.1e} "
             f"mu d={abs(g['mu'] - r[2]):.1e} (Hartree CG {g['hartree_iters']})")
    assert conv and out["converged"]
    _compare_history(hist, out["history"], 1e-6, 1e-11, "scf two-grid")
    for got, ref in ((ro, out["rho_out"]), (mo, out["m_out"]), (rho, out["rho_in"]), (m, out["m_in"])):
        assert np.abs(got.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()
    assert np.abs(th - out["theta"]).max() <= 1e-9
    # with its own Lanczos bounds: the same fixed point (to the stopping tolerance)
    rho2, m2 = _dev(rho0), _dev(m0)
    ro2, mo2 = torch.empty_like(rho2), torch.empty_like(m2)
    h2, th2, _, conv2 = scf_run(of, _dev(vext), _dev(bext), rho2, m2, ro2, mo2, X, n_e, kT, 8, coarse=oc, seed=0,
                                lanczos_seed=fine.seed + 1, **kw)
    d_rho = np.abs(ro2.cpu().numpy() - out["rho_out"]).max() / np.abs(out["rho_out"]).max()
    _say(f"[scf two-grid] own bounds: {len(h2)} iterations, residual {h2[-1]['resid']:.2e}, rho rel diff {d_rho:.1e}")
    assert conv2 and abs(len(h2) - len(hist)) <= 4
    # the occupied Ritz values are converged; the top of the block (unoccupied, two
    # passes per iteration) is not, and depends on the filter bounds
    occd = out["occ"] > 0.5
    d_th = np.abs(th2 - out["theta"])[occd].max()
    _say(f"[scf two-grid] own bounds: occupied Ritz values within {d_th:.1e} Ha")
    assert d_rho <= 1e-6 and d_th <= 1e-8
    of.close()
    oc.close()


def test_scf_kpoint_sampling_two_grid_matches_oracle():
    """Brillouin-zone sampling: two k-points of weights 0.3 and 0.7, each with its
    own block, bound and passes, one Fermi level, densities summed with the
    weights; two-grid start (every k-point's block moved to degree p).  Record by
    record with the oracle's filter bounds, then the final densities, the
    occupied Ritz values of both k-points and their occupations."""
    from paper_2410_02754_amd import scf_run
    kpts = [(0.0, 0.0, 0.7), (0.25, 0.0, -0.35)]
    w = [0.3, 0.7]
    kw_sys = dict(n_cells=(2, 2, 2), box=(4.5, 4.5, 4.5), n_atoms=2, lmax=1, rcut_sigmas=5.0, n_vec=8,
                  degree=8, seed=5, kpts=kpts)
    fine = synth.make_system("kscf", p=3, n_q=5, **kw_sys)
    coarse = synth.make_system("kscf", p=2, n_q=5, **kw_sys)
    mesh = ham.mesh_for(fine)
    pts = mesh.all_quad_points().reshape(-1, 3)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    vext = synth.veff(fine, pts).reshape(E, nq3)
    bext = synth.bxc(fine, pts).reshape(E, nq3, 3)
    # 3.4 electrons: the Fermi level sits in a partly filled level (with a whole number
    # of filled levels it would lie anywhere in a gap, fixed only by rounding)
    n_e, kT = 3.4, 2e-3
    rho0 = np.full((E, nq3), n_e / 4.5 ** 3)
    m0 = 0.05 * rho0[..., None] * np.array([0.6, 0.0, 0.8])
    kw = dict(passes_first=5, passes=2, depth=4, alpha=0.5, k0=0.6, tol=1e-7, tol_coarse=1e-2, max_iter=60)
    out = scf.scf(fine, vext, bext, rho0, m0, n_e, kT, coarse_system=coarse, kweights=w, **kw)
    of = _op(fine.n_cells, fine.box, 3, 5, fine.atoms, kpts=kpts)
    oc = _op(coarse.n_cells, coarse.box, 2, 5, coarse.atoms, kpts=kpts)
    rho, m = _dev(rho0), _dev(m0)
    ro, mo = torch.empty_like(rho), torch.empty_like(m)
    X = torch.empty((2, of.n_dof, 8), dtype=torch.complex128, device="cuda")
    hist, th, occ, conv = scf_run(of, _dev(vext), _dev(bext), rho, m, ro, mo, X, n_e, kT, 8, coarse=oc, seed=0,
                                  lanczos_seed=fine.seed + 1, bounds=_bounds(out["history"]), kweights=w, **kw)
    _say(f"[scf k-points] gpu {len(hist)} iterations; oracle {len(out['history'])}")
    for g, r in zip(hist, out["history"]):
        _say(f"   p{g['p']} gpu {g['resid']:.6e} oracle {r[1]:.6e} d={abs(g['resid'] - r[1]):.1e} "
             f"mu d={abs(g['mu'] - r[2]):.1e}")
    assert conv and out["converged"]
    _compare_history(hist, out["history"], 1e-6, 1e-11, "scf k-points")
    for got, ref in ((ro, out["rho_out"]), (mo, out["m_out"]), (rho, out["rho_in"]), (m, out["m_in"])):
        assert np.abs(got.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()
    occd = out["occ_k"] > 1e-12
    assert th.shape == (2, 8) and np.abs(th - out["theta_k"])[occd].max() <= 1e-9
    assert np.abs(occ - out["occ_k"]).max() <= 1e-8
    # the weights enter: both k-points hold electrons, in the ratio of the zone average
    assert abs(float(np.dot(w, occ.sum(axis=1))) - n_e) < 1e-10
    of.close()
    oc.close()


def test_scf_mixed_precision_reaches_the_fp64_fixed_point():
    """Mixed precision in the SCF loop runs the residual form of the filter (FP32
    products on H x residual only, Sec. III.B.2): the loop converges as far as the
    FP64 one (to 1e-9 here, where FP32 products on the whole block stall near
    3e-8) and lands on the oracle's fixed point."""
    from paper_2410_02754_amd import scf_run
    kw_sys = dict(n_cells=(2, 2, 2), box=(5.0, 5.0, 5.0), n_atoms=2, lmax=1, rcut_sigmas=5.0, n_vec=10,
                  degree=8, seed=6)
    fine = synth.make_system("scf", p=3, n_q=5, **kw_sys)
    coarse = synth.make_system("scf", p=2, n_q=5, **kw_sys)
    mesh = ham.mesh_for(fine)
    pts = mesh.all_quad_points().reshape(-1, 3)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    vext = synth.veff(fine, pts).reshape(E, nq3)
    bext = synth.bxc(fine, pts).reshape(E, nq3, 3)
    n_e, kT = 5.0, 500 * 3.166811563e-6
    rho0 = np.full((E, nq3), n_e / 125.0)
    m0 = 0.2 * bext / 0.1 * rho0[..., None]
    kw = dict(passes_first=5, passes=2, depth=5, alpha=0.5, k0=0.8, tol=1e-9, tol_coarse=1e-2, max_iter=50)
    out = scf.scf(fine, vext, bext, rho0, m0, n_e, kT, coarse_system=coarse, **kw)
    of = _op(fine.n_cells, fine.box, 3, 5, fine.atoms)
    oc = _op(coarse.n_cells, coarse.box, 2, 5, coarse.atoms)
    res = {}
    for prec in ("fp64", "mixed"):
        rho, m = _dev(rho0), _dev(m0)
        ro, mo = torch.empty_like(rho), torch.empty_like(m)
        X = torch.empty((of.n_dof, 10), dtype=torch.complex128, device="cuda")
        hist, th, occ, conv = scf_run(of, _dev(vext), _dev(bext), rho, m, ro, mo, X, n_e, kT, 8, coarse=oc, seed=0,
                                      lanczos_seed=fine.seed + 1, prec=prec, **kw)
        _say(f"[scf {prec}] {len(hist)} iterations, residual {hist[-1]['resid']:.2e}, converged {conv}")
        assert conv
        res[prec] = (len(hist), ro.cpu().numpy(), mo.cpu().numpy(), th, occ)
    n64, r64, m64, t64, o64 = res["fp64"]
    nmx, rmx, mmx, tmx, omx = res["mixed"]
    d_rho = np.abs(rmx - r64).max() / np.abs(r64).max()
    d_ref = np.abs(rmx - out["rho_out"]).max() / np.abs(out["rho_out"]).max()
    occd = o64 > 0.5
    d_th = np.abs(tmx - t64)[occd].max()
    _say(f"[scf mixed] rho vs FP64 {d_rho:.1e}, vs oracle {d_ref:.1e}; occupied theta {d_th:.1e} Ha")
    assert abs(nmx - n64) <= 2
    assert d_rho <= 1e-9 and d_ref <= 1e-8 and d_th <= 1e-9
    assert np.abs(mmx - m64).max() <= 1e-9 * np.abs(r64).max()
    of.close()
    oc.close()


def test_scf_restart_from_given_blocks_matches_oracle():
    """start_given: the loop continues from the caller's block and densities (here the
    state left by four iterations), as the oracle does from the same X0, rho0, m0."""
    from paper_2410_02754_amd import scf_run
    fine = synth.make_system("scf", p=3, n_q=5, n_cells=(2, 2, 2), box=(5.0, 5.0, 5.0), n_atoms=2, lmax=1,
                             rcut_sigmas=5.0, n_vec=10, degree=8, seed=6)
    mesh = ham.mesh_for(fine)
    pts = mesh.all_quad_points().reshape(-1, 3)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    vext = synth.veff(fine, pts).reshape(E, nq3)
    bext = synth.bxc(fine, pts).reshape(E, nq3, 3)
    n_e, kT = 5.0, 500 * 3.166811563e-6
    rho0 = np.full((E, nq3), n_e / 125.0)
    m0 = 0.2 * bext / 0.1 * rho0[..., None]
    of = _op(fine.n_cells, fine.box, 3, 5, fine.atoms)
    rho, m = _dev(rho0), _dev(m0)
    ro, mo = torch.empty_like(rho), torch.empty_like(m)
    X = torch.empty((of.n_dof, 10), dtype=torch.complex128, device="cuda")
    kw = dict(passes_first=3, passes=2, depth=4, alpha=0.5, k0=0.8, tol=1e-30)
    scf_run(of, _dev(vext), _dev(bext), rho, m, ro, mo, X, n_e, kT, 8, seed=0, lanczos_seed=fine.seed + 1,
            max_iter=4, **kw)
    X0, r0, mm0 = X.cpu().numpy(), rho.cpu().numpy(), m.cpu().numpy()
    out = scf.scf(fine, vext, bext, r0, mm0, n_e, kT, X0=X0, max_iter=5, **kw)
    hist, th, occ, conv = scf_run(of, _dev(vext), _dev(bext), rho, m, ro, mo, X, n_e, kT, 8,
                                  lanczos_seed=fine.seed + 1, max_iter=5, start_given=True,
                                  bounds=_bounds(out["history"]), **kw)
    for g, r in zip(hist, out["history"]):
        _say(f"   restart gpu {g['resid']:.6e} oracle {r[1]:.6e} d={abs(g['resid'] - r[1]):.1e}")
    _compare_history(hist, out["history"], 1e-6, 1e-11, "scf restart")
    assert np.abs(ro.cpu().numpy() - out["rho_out"]).max() <= 1e-9 * np.abs(out["rho_out"]).max()
    of.close()


def test_scf_kpoints_mixed_precision_reaches_the_fp64_fixed_point():
    """Brillouin-zone sampling with the mixed-precision (residual-form) filter: the same
    fixed point as the FP64 loop over the same two weighted k-points, and the oracle's."""
    from paper_2410_02754_amd import scf_run
    kpts = [(0.0, 0.0, 0.7), (0.25, 0.0, -0.35)]
    w = [0.3, 0.7]
    s = synth.make_system("kscf", p=3, n_q=5, n_cells=(2, 2, 2), box=(4.5, 4.5, 4.5), n_atoms=2, lmax=1,
                          rcut_sigmas=5.0, n_vec=8, degree=8, seed=5, kpts=kpts)
    mesh = ham.mesh_for(s)
    pts = mesh.all_quad_points().reshape(-1, 3)
    E, nq3 = mesh.n_cell_total, mesh.nq ** 3
    vext = synth.veff(s, pts).reshape(E, nq3)
    bext = synth.bxc(s, pts).reshape(E, nq3, 3)
    n_e, kT = 3.4, 2e-3
    rho0 = np.full((E, nq3), n_e / 4.5 ** 3)
    m0 = 0.05 * rho0[..., None] * np.array([0.6, 0.0, 0.8])
    kw = dict(passes_first=5, passes=2, depth=4, alpha=0.5, k0=0.6, tol=1e-9, max_iter=60)
    out = scf.scf(s, vext, bext, rho0, m0, n_e, kT, kweights=w, **kw)
    op = _op(s.n_cells, s.box, 3, 5, s.atoms, kpts=kpts)
    res = {}
    for prec in ("fp64", "mixed"):
        rho, m = _dev(rho0), _dev(m0)
        ro, mo = torch.empty_like(rho), torch.empty_like(m)
        X = torch.empty((2, op.n_dof, 8), dtype=torch.complex128, device="cuda")
        hist, th, occ, conv = scf_run(op, _dev(vext), _dev(bext), rho, m, ro, mo, X, n_e, kT, 8, seed=0,
                                      lanczos_seed=s.seed + 1, kweights=w, prec=prec, **kw)
        _say(f"[scf k-points {prec}] {len(hist)} iterations, residual {hist[-1]['resid']:.2e}")
        assert conv
        res[prec] = (ro.cpu().numpy(), mo.cpu().numpy(), th, occ)
    r64, m64, t64, o64 = res["fp64"]
    rmx, mmx, tmx, omx = res["mixed"]
    occd = o64 > 1e-12
    d_rho = np.abs(rmx - r64).max() / np.abs(r64).max()
    d_ref = np.abs(rmx - out["rho_out"]).max() / np.abs(out["rho_out"]).max()
    d_th = np.abs(tmx - t64)[occd].max()
    _say(f"[scf k-points mixed] rho vs FP64 {d_rho:.1e}, vs oracle {d_ref:.1e}; occupied theta {d_th:.1e} Ha")
    assert d_rho <= 1e-9 and d_ref <= 1e-8 and d_th <= 1e-9
    assert np.abs(mmx - m64).max() <= 1e-9 * np.abs(r64).max()
    op.close()
