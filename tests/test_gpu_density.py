"""GPU densities (eqn:rho, eqn:mag) through the C ABI, against the oracle's
plain definition on small systems (several column groups, ragged column tails,
p = 3 .. 8 with up to 10^3 quadrature points per cell, and the sum-factorised
kernel at every order p = 1 .. 8 with n_q = p + 1), against properties
that hold at any size (GLL charge integral, |m| <= rho, additivity over
blocks, run-to-run identity), and on sampled cells of the large workload
(20^3 cells, p = 6, 512 columns, Fermi-Dirac occupations at 500 K)."""
import numpy as np
import pytest

import synth
from oracle import density as od, hamiltonian as ham

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KT500 = 500 * od.KELVIN_TO_HA


def _op(s):
    from paper_2410_02754_amd import Operator
    return Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts)


def _fields(op):
    rho = torch.zeros((op.n_cells, op.nq3), dtype=torch.float64, device="cuda")
    mag = torch.zeros((op.n_cells, op.nq3, 3), dtype=torch.float64, device="cuda")
    return rho, mag


def _occ(seed, n):
    from paper_2410_02754_amd import fermi_dirac
    eps = np.sort(np.random.default_rng(seed).uniform(-0.3, 0.1, size=n))
    f, _, _ = fermi_dirac(eps, 0.6 * n, KT500)
    return f


CASES = [
    ("p3k", dict(n_cells=(2, 3, 2), box=(4.0, 5.0, 4.0), p=3, kpts=[(0.1, -0.15, 0.05)]), 5),
    ("p4", dict(n_cells=(2, 2, 3), box=(4.0, 4.0, 6.0), p=4), 37),
    ("p6", dict(n_cells=(2, 2, 2), box=(2.4, 2.4, 2.4), p=6, n_q=8), 70),
    ("p8q10", dict(n_cells=(2, 2, 2), box=(3.2, 3.2, 3.2), p=8, n_q=10), 9),
]


@pytest.mark.parametrize("name,kw,n_vec", CASES, ids=[c[0] for c in CASES])
def test_density_matches_oracle(name, kw, n_vec):
    s = synth.make_system(name, n_atoms=1, lmax=1, rcut_sigmas=5.0, n_vec=n_vec, **kw)
    mesh = ham.mesh_for(s)
    MD = mesh.lumped_mass()
    X0 = synth.random_block(7, s.n_dof, n_vec)
    f = _occ(1, n_vec)
    rho_o, m_o = od.density_magnetisation(mesh, MD, X0, f)
    op = _op(s)
    rho, mag = _fields(op)
    op.density(torch.tensor(X0, device="cuda"), f, rho, mag)
    r, m = rho.cpu().numpy(), mag.cpu().numpy()
    scale = np.abs(rho_o).max()
    er, em = np.abs(r - rho_o).max() / scale, np.abs(m - m_o).max() / scale
    print(f"[density {name}] n_vec {n_vec}: rel err rho {er:.2e} m {em:.2e}", flush=True)
    assert er < 1e-13 and em < 1e-13
    op.close()


SF_CASES = [(p, (2, 2, 2)) for p in range(1, 9)] + [(1, (16, 16, 16)), (2, (16, 16, 16))]


@pytest.mark.parametrize("p,nc", SF_CASES, ids=[f"p{c[0]}_{c[1][0]}x{c[1][1]}x{c[1][2]}" for c in SF_CASES])
def test_density_quadrature_point_kernel_every_order(p, nc):
    """n_q = p + 1 (the sum-factorised kernel, one padded LDS layout per order):
    every order p = 1..8 against the oracle's definition, 13 or 21 columns in
    chunks of 4 (ragged last chunk); on the 16^3-cell meshes each column group
    walks several chunks (the prefetch path)."""
    nv = 21 if nc[0] == 16 else 13
    s = synth.make_system("dsf", n_cells=nc, box=tuple(1.5 * c for c in nc), p=p, n_atoms=1, lmax=1,
                          rcut_sigmas=5.0, n_vec=nv)
    assert s.n_q == p + 1
    mesh = ham.mesh_for(s)
    MD = mesh.lumped_mass()
    X0 = synth.random_block(7, s.n_dof, nv)
    f = np.linspace(1.0, 0.1, nv)
    rho_o, m_o = od.density_magnetisation(mesh, MD, X0, f)
    op = _op(s)
    rho, mag = _fields(op)
    op.density(torch.tensor(X0, device="cuda"), f, rho, mag)
    r, m = rho.cpu().numpy(), mag.cpu().numpy()
    scale = np.abs(rho_o).max()
    er, em = np.abs(r - rho_o).max() / scale, np.abs(m - m_o).max() / scale
    print(f"[density sf p{p} {nc}] rel err rho {er:.2e} m {em:.2e}", flush=True)
    assert er < 1e-13 and em < 1e-13
    op.close()


def test_density_is_additive_and_reproducible():
    """Two half blocks added in turn give the whole block's density (to rounding);
    the same call twice gives identical bits; zero occupations add nothing."""
    s = synth.make_system("add", n_cells=(2, 2, 2), box=(4.0, 4.0, 4.0), p=4, n_atoms=1, lmax=1,
                          rcut_sigmas=5.0, n_vec=24)
    op = _op(s)
    X = torch.tensor(synth.random_block(3, s.n_dof, 24), device="cuda")
    f = _occ(2, 24)
    r1, m1 = _fields(op)
    op.density(X, f, r1, m1)
    r2, m2 = _fields(op)
    op.density(X, f, r2, m2)
    assert torch.equal(r1, r2) and torch.equal(m1, m2)
    r3, m3 = _fields(op)
    op.density(X[:, :11].contiguous(), f[:11], r3, m3)
    op.density(X[:, 11:].contiguous(), f[11:], r3, m3)
    assert float((r3 - r1).abs().max()) < 1e-14 * float(r1.abs().max())
    assert float((m3 - m1).abs().max()) < 1e-14 * float(r1.abs().max())
    r4, m4 = _fields(op)
    op.density(X, np.zeros(24), r4, m4)
    assert float(r4.abs().max()) == 0.0 and float(m4.abs().max()) == 0.0
    with pytest.raises(ValueError):
        op.density(X, f[:5], r4, m4)
    op.close()


def test_gll_charge_integral_and_bloch_bound():
    """GLL collocation: the integral of rho is sum_n f_n x_n^H x_n exactly, and
    |m| <= rho pointwise for any occupation-weighted sum of spinor densities."""
    s = synth.make_system("gllq", n_cells=(3, 2, 2), box=(6.0, 4.0, 4.0), p=5, quad="gll", n_atoms=1, lmax=1,
                          rcut_sigmas=5.0, n_vec=33)
    op = _op(s)
    X0 = synth.random_block(5, s.n_dof, 33)
    f = _occ(3, 33)
    rho, mag = _fields(op)
    op.density(torch.tensor(X0, device="cuda"), f, rho, mag)
    mesh = ham.mesh_for(s)
    integral = float(np.sum(mesh.wq[None, :] * mesh.J * rho.cpu().numpy()))
    expect = float(np.sum(f * np.sum(np.abs(X0) ** 2, axis=0)))
    print(f"[density gll] integral {integral:.15e} vs {expect:.15e}", flush=True)
    assert abs(integral - expect) < 1e-12 * expect
    mn = torch.linalg.norm(mag, dim=-1)
    assert bool((mn <= rho * (1 + 1e-12) + 1e-300).all())
    op.close()


def test_density_large_workload_sampled_cells():
    """20^3 cells, p = 6, 512 columns with Fermi-Dirac occupations at 500 K, the
    shape of the densities after a pass of the large workload; cells across the
    box checked one by one against the oracle."""
    from oracle.fe import Mesh
    from paper_2410_02754_amd import fermi_dirac
    s = synth.config("scale")
    op = _op(s)
    n_vec = s.n_vec
    X = torch.empty((s.n_dof, n_vec), dtype=torch.complex128, device="cuda")
    op.fill_random(X, s.seed, n_total_cols=n_vec)
    eps = np.sort(np.random.default_rng(4).uniform(-0.5, 0.2, size=n_vec))
    f, _, _ = fermi_dirac(eps, 0.9 * n_vec, KT500)
    rho, mag = _fields(op)
    op.density(X, f, rho, mag)
    cells = np.array([0, 1, 19, 20, 399, 400, 4210, 7999])
    got_r = rho[torch.tensor(cells, device="cuda")].cpu().numpy()
    got_m = mag[torch.tensor(cells, device="cuda")].cpu().numpy()
    del X
    op.close()
    mesh = Mesh(s.n_cells, s.box, s.p, s.quad, s.n_q)
    MD = mesh.lumped_mass()
    ref_r, ref_m = od.density_at_cells(mesh, MD, lambda r: synth.random_rows(s.seed, r, n_vec, n_vec), cells, f)
    scale = np.abs(ref_r).max()
    er, em = np.abs(got_r - ref_r).max() / scale, np.abs(got_m - ref_m).max() / scale
    print(f"[density scale] {len(cells)} cells: rel err rho {er:.2e} m {em:.2e}", flush=True)
    assert er < 1e-13 and em < 1e-13


def test_density_of_a_block_in_a_wider_array_and_argument_checks():
    """Columns 5..29 of a 40-column array (ld = 40) give the density of that
    sub-block; bad shapes and sizes are refused before any launch."""
    import ctypes as C
    from paper_2410_02754_amd import ChfsiError
    s = synth.make_system("wide", n_cells=(2, 2, 2), box=(4.0, 4.0, 4.0), p=4, n_atoms=1, lmax=1,
                          rcut_sigmas=5.0, n_vec=40)
    op = _op(s)
    Xw = torch.tensor(synth.random_block(9, s.n_dof, 40), device="cuda")
    f = _occ(5, 25)
    r1, m1 = _fields(op)
    op.density(Xw[:, 5:30], f, r1, m1)
    r2, m2 = _fields(op)
    op.density(Xw[:, 5:30].contiguous(), f, r2, m2)
    assert torch.equal(r1, r2) and torch.equal(m1, m2)
    with pytest.raises(ValueError):
        op.density(Xw[:, :25], f, r1[:1], m1)
    pd = C.POINTER(C.c_double)
    fo = np.ascontiguousarray(f)
    rc = op.lib.chfsi_density(op.ctx, C.c_void_p(Xw.data_ptr()), 40, 0, fo.ctypes.data_as(pd),
                              C.c_void_p(r1.data_ptr()), C.c_void_p(m1.data_ptr()))
    assert rc == -1
    rc = op.lib.chfsi_density(op.ctx, C.c_void_p(Xw.data_ptr()), 40, 25, None, C.c_void_p(r1.data_ptr()),
                              C.c_void_p(m1.data_ptr()))
    assert rc == -1
    bad = fo.copy()
    bad[3] = np.nan
    with pytest.raises(ChfsiError):
        op.density(Xw[:, :25], bad, r1, m1)
    op.close()
