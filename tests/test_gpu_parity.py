"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs (apply, filter, CholGS, Rayleigh-Ritz, Lanczos, full passes).

Tolerances: FP64 products agree to 1e-12 relative to max|y| (summation order
differs: colour-ordered cell products vs CSR rows); Ritz values to 1e-10 Ha;
spans of gap-separated clusters to sin(angle) <= 1e-9; mixed precision
(FP32 cell/projector products) to 2e-6 relative per apply.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import chfsi as och, hamiltonian as ham

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _op(s):
    from paper_2410_02754_amd import Operator
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts)
    pts = op.quad_points().reshape(-1, 3)
    V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
    B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
    op.set_local(V, B)
    op.set_atoms(s.atoms)
    return op


def _oracle(s, ik=0):
    _, H, _, _, _ = ham.build(s, synth.veff, synth.bxc, ik=ik)
    return H


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


SYSTEMS = {
    "tiny": lambda: synth.config("tiny"),
    "k_l2_aniso": lambda: synth.make_system(
        "k_l2_aniso", n_cells=(2, 3, 4), box=(4.0, 5.0, 6.5), p=3, kpts=[(0.21, -0.13, 0.3)],
        n_atoms=2, lmax=2, rcut_sigmas=6.0, n_vec=20, degree=7),
    "gll_p5": lambda: synth.make_system(
        "gll_p5", n_cells=(2, 2, 3), box=(4.0, 4.0, 6.0), p=5, quad="gll", n_atoms=1, lmax=1,
        rcut_sigmas=5.0, n_vec=16),
    "gl_p2_nq4": lambda: synth.make_system(
        "gl_p2_nq4", n_cells=(3, 2, 2), box=(4.0, 3.0, 3.0), p=2, n_q=4, n_atoms=3, lmax=2,
        rcut_sigmas=4.0, kpts=[(0.0, 0.4, 0.0)], n_vec=8),
    # complex projector values with 4 projectors per atom: the packed contraction rows
    "k_l1": lambda: synth.make_system(
        "k_l1", n_cells=(2, 3, 2), box=(4.0, 5.5, 4.5), p=3, kpts=[(0.17, 0.29, -0.11)],
        n_atoms=3, lmax=1, rcut_sigmas=5.0, n_vec=16),
}


def test_quadrature_points_match_oracle():
    s = SYSTEMS["k_l2_aniso"]()
    from paper_2410_02754_amd import Operator
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts)
    mesh = ham.mesh_for(s)
    assert np.abs(op.quad_points() - mesh.all_quad_points()).max() < 1e-14
    assert op.n_dof == s.n_dof
    op.close()


@pytest.mark.parametrize("name", list(SYSTEMS))
@pytest.mark.parametrize("n_vec", [1, 37, 130])
def test_apply_H_fp64(name, n_vec):
    s = SYSTEMS[name]()
    _say(f"[apply_H fp64] {name} n_vec={n_vec}")
    H = _oracle(s)
    op = _op(s)
    X0 = synth.random_block(7, s.n_dof, n_vec)
    X = torch.tensor(X0, device="cuda")
    Y = torch.full_like(X, complex(np.nan, np.nan))    # output must be fully overwritten
    op.apply_H(X, Y)
    ref = H @ X0
    err = np.abs(Y.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say(f"   rel err {err:.3e}")
    assert err < 1e-12
    op.close()


def test_apply_H_block_of_wider_array_and_determinism():
    s = SYSTEMS["tiny"]()
    H = _oracle(s)
    op = _op(s)
    Xw = torch.tensor(synth.random_block(3, s.n_dof, 96), device="cuda")
    Yw = torch.zeros_like(Xw)
    blk = slice(32, 80)
    op.apply_H(Xw[:, blk], Yw[:, blk])
    ref = H @ Xw[:, blk].cpu().numpy()
    assert np.abs(Yw[:, blk].cpu().numpy() - ref).max() < 1e-12 * np.abs(ref).max()
    assert torch.count_nonzero(Yw[:, :32]) == 0 and torch.count_nonzero(Yw[:, 80:]) == 0
    Y2 = torch.zeros_like(Xw)
    op.apply_H(Xw[:, blk], Y2[:, blk])
    assert torch.equal(Yw, Y2)                       # bitwise reproducible (no atomics)
    op.close()


@pytest.mark.parametrize("name", ["tiny", "k_l2_aniso", "k_l1"])
def test_apply_H_mixed(name):
    s = SYSTEMS[name]()
    H = _oracle(s)
    op = _op(s)
    X0 = synth.random_block(11, s.n_dof, 64)
    X = torch.tensor(X0, device="cuda")
    Y = torch.empty_like(X)
    op.apply_H(X, Y, prec="mixed")
    ref = H @ X0
    err = np.abs(Y.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say(f"[apply_H mixed] {name} rel err {err:.3e}")
    assert 1e-9 < err < 2e-6
    op.close()


def _bounds(H, X0):
    th, _, _ = och.rayleigh_ritz(H, och.chol_gs(X0))
    lam = np.linalg.eigvalsh(H.toarray())
    return float(th[-1]), float(lam[-1] + 0.7), float(th[0])


@pytest.mark.parametrize("name,degree", [("tiny", 10), ("k_l2_aniso", 7), ("gl_p2_nq4", 1)])
def test_cheb_filter_fp64(name, degree):
    s = SYSTEMS[name]()
    H = _oracle(s)
    op = _op(s)
    X0 = synth.start_block(s, s.n_dof)
    a, b, a0 = _bounds(H, X0)
    X = torch.tensor(X0, device="cuda")
    W = torch.empty_like(X)
    op.cheb_filter(X, W, degree, a, b, a0)
    ref = och.cheb_filter(H, X0, degree, a, b, a0)
    err = np.abs(X.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say(f"[filter] {name} m={degree} rel err {err:.3e}")
    assert err < 1e-11
    op.close()


def test_cholgs_and_rr_parity():
    s = SYSTEMS["tiny"]()
    H = _oracle(s)
    op = _op(s)
    X0 = synth.start_block(s, s.n_dof)
    X = torch.tensor(X0, device="cuda")
    op.chol_gs(X)
    Xg = X.cpu().numpy()
    Xo = och.chol_gs(X0)
    assert np.abs(Xg.conj().T @ Xg - np.eye(s.n_vec)).max() < 1e-13
    assert np.abs(Xg - Xo).max() < 1e-12          # Cholesky with positive diagonal is unique
    W = torch.empty_like(X)
    th, r = op.rayleigh_ritz(X, W)
    tho, Xro, ro = och.rayleigh_ritz(H, Xo)
    assert np.abs(th - tho).max() < 1e-11
    assert np.abs(r - ro).max() < 1e-10
    assert och.sin_largest_angle(X.cpu().numpy(), Xro) < 1e-10
    op.close()


def test_lanczos_bounds():
    s = SYSTEMS["tiny"]()
    H = _oracle(s)
    op = _op(s)
    v0 = synth.lanczos_start(s, s.n_dof)
    lo, hi = op.lanczos_bounds(torch.tensor(v0, device="cuda"), 40)
    lo_o, hi_o = och.lanczos_bounds(H, v0, 40)
    lam = np.linalg.eigvalsh(H.toarray())
    _say(f"[lanczos] gpu ({lo}, {hi}) oracle ({lo_o}, {hi_o}) lam_max {lam[-1]}")
    assert hi >= lam[-1]
    assert abs(hi - hi_o) < 1e-8 * abs(hi_o)
    assert abs(lo - lo_o) < 1e-8 * max(1.0, abs(lo_o))
    op.close()


def test_full_passes_tiny():
    """Three ChFSI passes on the tiny workload (3^3 cells, p=4, N=32, m=10)
    with the same Lanczos bound on both sides: Ritz values to 1e-10 Ha."""
    s = SYSTEMS["tiny"]()
    H = _oracle(s)
    op = _op(s)
    X0 = synth.start_block(s, s.n_dof)
    _, b = och.lanczos_bounds(H, synth.lanczos_start(s, s.n_dof), 40)
    hist = []
    tho, Xo, ro = och.run(H, X0, s.degree, s.passes, s.block, b, hist)
    X = torch.tensor(X0, device="cuda")
    W = torch.empty_like(X)
    op.chol_gs(X)
    th, r = op.rayleigh_ritz(X, W)
    for p in range(s.passes):
        op.cheb_filter(X, W, s.degree, float(th[-1]), b, float(th[0]))
        op.chol_gs(X)
        th, r = op.rayleigh_ritz(X, W)
        d = np.abs(th - hist[p + 1][0]).max()
        _say(f"[passes] pass {p + 1}: max |dtheta| = {d:.3e}")
    assert np.abs(th - tho).max() < 1e-10
    assert np.abs(r - ro).max() < 1e-8
    Xg = X.cpu().numpy()
    # spans of gap-separated clusters
    gaps = np.where(np.diff(tho) > 1e-6)[0]
    edges = [0] + list(gaps + 1) + [len(tho)]
    for i0, i1 in zip(edges[:-1], edges[1:]):
        assert och.sin_largest_angle(Xg[:, i0:i1], Xo[:, i0:i1]) < 1e-8
    op.close()


def test_full_passes_p6_degree24():
    """Two ChFSI passes at the large workload's element order, mesh size and
    filter degree (p=6, h=1.2 bohr, m=24) on a 2x2x3-cell periodic piece (even and
    odd colourings) with an l<=2 atom whose support wraps the box, N=64 in two
    blocks of 32 with shared bounds: Ritz values to 1e-10 Ha, spans of
    gap-separated clusters."""
    s = synth.make_system("p6m24", n_cells=(2, 2, 3), box=(2.4, 2.4, 3.6), p=6, n_gauss=3, n_atoms=1,
                          lmax=2, rcut_sigmas=6.0, n_vec=64, block=32, degree=24, passes=2, seed=4)
    H = _oracle(s)
    op = _op(s)
    X0 = synth.start_block(s, s.n_dof)
    _, b = och.lanczos_bounds(H, synth.lanczos_start(s, s.n_dof), 40)
    hist = []
    tho, Xo, ro = och.run(H, X0, s.degree, s.passes, s.block, b, hist)
    X = torch.tensor(X0, device="cuda")
    W = torch.empty_like(X)
    op.chol_gs(X)
    th, r = op.rayleigh_ritz(X, W)
    for p in range(s.passes):
        a, a0 = float(th[-1]), float(th[0])
        for c0 in range(0, s.n_vec, s.block):
            op.cheb_filter(X[:, c0:c0 + s.block], W[:, :s.block], s.degree, a, b, a0)
        op.chol_gs(X)
        th, r = op.rayleigh_ritz(X, W)
        _say(f"[passes p6] pass {p + 1}: max |dtheta| = {np.abs(th - hist[p + 1][0]).max():.3e}")
    assert np.abs(th - tho).max() < 1e-10
    assert np.abs(r - ro).max() < 1e-8
    Xg = X.cpu().numpy()
    gaps = np.where(np.diff(tho) > 1e-6)[0]
    edges = [0] + list(gaps + 1) + [len(tho)]
    for i0, i1 in zip(edges[:-1], edges[1:]):
        assert och.sin_largest_angle(Xg[:, i0:i1], Xo[:, i0:i1]) < 1e-8
    op.close()


def test_fill_random_bit_exact():
    s = SYSTEMS["tiny"]()
    from paper_2410_02754_amd import Operator
    op = Operator(s.n_cells, s.box, s.p)
    X = torch.empty((100, 24), dtype=torch.complex128, device="cuda")
    op.fill_random(X, 12345, row0=37, col0=5, n_total_cols=64)
    ref = synth.random_block(12345, 100, 24, row0=37, col0=5, n_total_cols=64)
    assert np.array_equal(X.cpu().numpy(), ref)
    op.close()


def test_error_paths():
    from paper_2410_02754_amd import ChfsiError
    s = SYSTEMS["gl_p2_nq4"]()
    op = _op(s)
    X = torch.tensor(synth.random_block(1, s.n_dof, 4), device="cuda")
    X[:, 2] = X[:, 1]                                # rank deficient
    with pytest.raises(ChfsiError) as ei:
        op.chol_gs(X)
    assert ei.value.code == -4 and ei.value.bad_col == 2
    W = torch.empty_like(X)
    with pytest.raises(ChfsiError) as ei:
        op.cheb_filter(X, W, 5, 1.0, 0.5, -1.0)       # a > b
    assert ei.value.code == -1
    V = torch.full((op.n_cells, op.nq3), float("nan"), dtype=torch.float64, device="cuda")
    Bf = torch.zeros((op.n_cells, op.nq3, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ChfsiError) as ei:
        op.set_local(V, Bf)
    assert ei.value.code == -6
    bad = np.eye(2 * 4, dtype=np.complex128)
    bad[0, 1] = 1j
    a = synth.Atom((1.0, 1.0, 1.0), 1, 0.6, 3.0, (1.0, 0.5), 0.0)
    with pytest.raises(ChfsiError) as ei:
        op.set_atoms([a], delta_overrides=[bad])
    assert ei.value.code == -5
    op.close()


def test_empty_blocks_are_rejected():
    """A block of zero columns is an argument error (CHFSI_EINVAL) at every call that
    takes one, and leaves the other operands untouched."""
    from paper_2410_02754_amd import ChfsiError
    s = SYSTEMS["gl_p2_nq4"]()
    op = _op(s)
    E = torch.empty((s.n_dof, 0), dtype=torch.complex128, device="cuda")
    W = torch.ones((s.n_dof, 4), dtype=torch.complex128, device="cuda")
    rho = torch.zeros((op.n_cells, op.nq3), dtype=torch.float64, device="cuda")
    mag = torch.zeros((op.n_cells, op.nq3, 3), dtype=torch.float64, device="cuda")
    calls = {
        "apply_H": lambda: op.apply_H(E, E),
        "cheb_filter": lambda: op.cheb_filter(E, W, 3, 1.0, 2.0, 0.0),
        "chol_gs": lambda: op.chol_gs(E),
        "rayleigh_ritz": lambda: op.rayleigh_ritz(E, W),
        "density": lambda: op.density(E, np.zeros(0), rho, mag),
    }
    for name, call in calls.items():
        with pytest.raises(ChfsiError) as ei:
            call()
        assert ei.value.code == -1, name
    torch.cuda.synchronize()
    assert bool((W == 1).all()) and float(rho.abs().max()) == 0.0 and float(mag.abs().max()) == 0.0
    op.close()


def test_cheb_filter_residual_form():
    """The residual form Y = X p(Theta) + Z equals the plain filter (FP64), and
    with FP32 products its error shrinks with the residuals (the correction Z
    is what passes through the FP32 products), unlike FP32 applies."""
    s = SYSTEMS["tiny"]()
    H = _oracle(s)
    op = _op(s)
    X0 = synth.start_block(s, s.n_dof)
    a, b, a0 = _bounds(H, X0)
    X = torch.tensor(X0, device="cuda")
    W = torch.empty_like(X)
    Wz = torch.empty((s.n_dof, 2 * s.n_vec), dtype=torch.complex128, device="cuda")
    op.chol_gs(X)
    th, r = op.rayleigh_ritz(X, W)
    ratios = []
    for npass in range(1, 7):
        op.cheb_filter(X, W, 10, float(th[-1]), b, float(th[0]))
        op.chol_gs(X)
        th, r = op.rayleigh_ritz(X, W)
        if npass not in (1, 6):
            continue
        R = W.clone()
        op.ritz_residual(X, R, th)
        Xr = X.cpu().numpy()
        assert np.abs(R.cpu().numpy() - (H @ Xr - Xr * th[None, :])).max() < 1e-12 * np.abs(H @ Xr).max()
        ref = och.cheb_filter(H, Xr, s.degree, th[-1], b, th[0])
        out = {}
        for prec in ("fp64", "mixed"):
            Y = X.clone()
            op.cheb_filter_resid(Y, R, th, Wz, s.degree, th[-1], b, th[0], prec=prec)
            out[prec] = np.abs(Y.cpu().numpy() - ref).max() / np.abs(ref).max()
            Yp = X.clone()
            op.cheb_filter(Yp, torch.empty_like(Yp), s.degree, th[-1], b, th[0], prec=prec)
            out[prec + "_plain"] = np.abs(Yp.cpu().numpy() - ref).max() / np.abs(ref).max()
        _say(f"[filter resid] after {npass} passes (max resid {r.max():.1e}): rel err fp64 {out['fp64']:.2e} "
             f"(plain {out['fp64_plain']:.2e}); mixed {out['mixed']:.2e} (plain mixed {out['mixed_plain']:.2e})")
        assert out["fp64"] < 1e-11
        assert out["mixed"] < out["mixed_plain"]
        ratios.append(out["mixed"] / out["mixed_plain"])
    assert ratios[-1] < 0.5 * ratios[0]          # the advantage grows with convergence
    op.close()


def test_cholgs_badly_scaled_columns_and_overlap():
    """CholGS on a block whose column norms span 12 orders of magnitude (the
    diagonal pre-scaling keeps the factor well conditioned): X^H X = I to 1e-13
    through chfsi_overlap, and the span equals the oracle's CholGS span.  The
    overlap itself is the plain definition X^H Y."""
    s = SYSTEMS["tiny"]()
    op = _op(s)
    X0 = synth.start_block(s, s.n_dof)
    scale = 10.0 ** np.linspace(-6, 6, s.n_vec)
    Xs = X0 * scale[None, :]
    Y0 = synth.random_block(9, s.n_dof, s.n_vec)
    S = op.overlap(torch.tensor(Xs, device="cuda"), torch.tensor(Y0, device="cuda"))
    ref = Xs.conj().T @ Y0
    assert np.abs(S - ref).max() <= 1e-13 * np.abs(ref).max()
    X = torch.tensor(Xs, device="cuda")
    op.chol_gs(X)
    G = op.overlap(X, X)
    orth = np.abs(G - np.eye(s.n_vec)).max()
    Xo = och.chol_gs(Xs)
    span = och.sin_largest_angle(X.cpu().numpy(), Xo)
    _say(f"[cholgs scaled] ||X^H X - I||_max {orth:.2e}, sin(angle) to the oracle span {span:.2e}")
    assert orth < 1e-13 and span < 1e-10
    op.close()


def test_workspace_bytes_bound_the_library_allocations():
    """chfsi_workspace_bytes covers what a fresh context allocates for a filter,
    CholGS and Rayleigh-Ritz (device memory measured before and after; the
    allocator's page rounding is allowed for)."""
    s = SYSTEMS["k_l2_aniso"]()
    op = _op(s)
    X = torch.tensor(synth.start_block(s, s.n_dof), device="cuda")
    W = torch.empty_like(X)
    torch.cuda.synchronize()
    ws = {k: op.workspace_bytes(s.n_vec, k) for k in ("apply", "filter", "chol_gs", "rayleigh_ritz", "density")}
    _say(f"[workspace] {ws}")
    assert all(v > 0 for v in ws.values())
    assert ws["filter"] == ws["apply"] and ws["rayleigh_ritz"] >= ws["filter"]
    free0 = torch.cuda.mem_get_info()[0]
    op.cheb_filter(X, W, 4, 5.0, 40.0, -2.0)
    op.chol_gs(X)
    op.rayleigh_ritz(X, W)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    bound = ws["filter"] + ws["chol_gs"] + ws["rayleigh_ritz"] + (8 << 20)
    _say(f"[workspace] measured {used} B, bound {bound} B")
    assert used <= bound
    op.close()
