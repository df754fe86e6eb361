"""GPU checks at the full size of the large workload (20^3 cells, p = 6,
3.456 M spinor dofs, 128-column blocks as in the benchmark) against closed
forms that need no oracle.

In GLL collocation with a constant potential v0 and a uniform field B the
scaled operator is the Kronecker sum of three 1-D periodic operators plus
v0 + B.sigma, so x (x) y (x) z (x) chi is an exact eigenvector with eigenvalue
lam_x + lam_y + lam_z + v0 +- |B| when chi is the +-B_hat.sigma eigenspinor.
"""
import numpy as np
import pytest

from closed_forms import periodic_1d

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NC, L, P = 20, 24.0, 6


def _product_block(k, bvec, v0, n_vec, seed=0):
    """Columns: product eigenvectors (device) and their eigenvalues (host)."""
    rng = np.random.default_rng(seed)
    ev, U = [], []
    for d in range(3):
        w, V = np.linalg.eigh(periodic_1d(NC, L, P, k[d]))
        ev.append(w)
        U.append(V)
    bmag = np.linalg.norm(bvec)
    bs = sum(bvec[d] / bmag * np.array(m) for d, m in enumerate(
        [[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]]))
    wb, chi = np.linalg.eigh(bs)
    n1 = NC * P
    # lowest modes first, then random ones across the spectrum
    picks = [(i, j, l, s) for i in range(3) for j in range(3) for l in range(3) for s in range(2)][:min(n_vec, 54)]
    while len(picks) < n_vec:
        picks.append(tuple(rng.integers(0, n1, size=3)) + (int(rng.integers(0, 2)),))
    lam = np.array([ev[0][i] + ev[1][j] + ev[2][l] + v0 + wb[s] * bmag for i, j, l, s in picks])
    dev = "cuda"
    Ux = torch.tensor(U[0], device=dev)
    Uy = torch.tensor(U[1], device=dev)
    Uz = torch.tensor(U[2], device=dev)
    X = torch.empty((2 * n1 ** 3, n_vec), dtype=torch.complex128, device=dev)
    Xv = X.view(n1, n1, n1, 2, n_vec)            # [iz][iy][ix][spin][col]
    for c, (i, j, l, s) in enumerate(picks):
        prod = Uz[:, l][:, None, None] * Uy[:, j][None, :, None] * Ux[:, i][None, None, :]
        ch = torch.tensor(chi[:, s], device=dev)
        Xv[:, :, :, 0, c] = prod * ch[0]
        Xv[:, :, :, 1, c] = prod * ch[1]
    return X, lam


@pytest.mark.parametrize("form", ["cell", "matrix_free"])
@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.05, -0.03, 0.02)])
def test_gll_kronecker_eigenvectors_full_scale(k, form):
    from paper_2410_02754_amd import Operator
    n_vec, v0, bvec = 128, -0.3, np.array([0.02, -0.05, 0.08])
    op = Operator((NC, NC, NC), (L, L, L), P, "gll", None, [k], form=form)
    V = torch.full((op.n_cells, op.nq3), v0, dtype=torch.float64, device="cuda")
    B = torch.tensor(np.tile(bvec, (op.n_cells, op.nq3, 1)), device="cuda")
    op.set_local(V, B)
    del V, B
    X, lam = _product_block(np.array(k), bvec, v0, n_vec)
    Y = torch.empty_like(X)
    lam_d = torch.tensor(lam, device="cuda")
    scale = float(np.abs(lam).max()) * float(X.abs().max())
    op.apply_H(X, Y)
    err = float((Y - X * lam_d[None, :]).abs().max()) / scale
    print(f"[scale gll k={k} {form}] fp64 max |H x - lam x| / (|lam| |x|) = {err:.3e}", flush=True)
    assert err < 1e-12
    if form == "matrix_free":
        op.close()
        return
    op.apply_H(X, Y, prec="mixed")
    errm = float((Y - X * lam_d[None, :]).abs().max()) / scale
    print(f"[scale gll k={k}] mixed rel residual = {errm:.3e}", flush=True)
    assert errm < 2e-6
    op.close()


def _sample_nodes(s, rng, n_near=48, n_far=16):
    """Nodes within r_c/2 of the first atom and of the last atom (opposite
    corners of the box, so different cells and colours)."""
    from oracle.fe import Mesh
    mesh = Mesh(s.n_cells, s.box, s.p, s.quad, s.n_q)
    cand = rng.choice(s.n_nodes, min(400000, s.n_nodes), replace=False)
    Nx, Ny, _ = mesh.N
    idx = np.stack([cand % Nx, (cand // Nx) % Ny, cand // (Nx * Ny)], axis=1)
    xyz = np.stack([(idx[:, d] // s.p) * mesh.h[d] + (mesh.xi[idx[:, d] % s.p] + 1) * mesh.h[d] / 2
                    for d in range(3)], axis=1)
    L = np.asarray(s.box)
    dist = []
    for a in s.atoms:
        d = xyz - np.asarray(a.pos)
        d = d - L * np.round(d / L)
        dist.append(np.linalg.norm(d, axis=1))
    dist = np.stack(dist)
    near = cand[dist[0] < s.atoms[0].rcut / 2][:n_near]
    far = cand[dist[-1] < s.atoms[-1].rcut / 2][:n_far]
    return np.sort(np.concatenate([near, far]))


def test_scale_workload_sampled_rows():
    """The large workload (20^3 cells, p=6, 64 SOC atoms, N = 128 as timed by the
    benchmark): rows of H_hat X from the oracle, cell by cell, at sampled nodes."""
    import synth
    from oracle import rows
    from paper_2410_02754_amd import Operator
    s = synth.config("scale")
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts)
    pts = op.quad_points().reshape(-1, 3)
    V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
    B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
    op.set_local(V, B)
    op.set_atoms(s.atoms)
    del V, B, pts
    n_vec = 128
    X = torch.empty((s.n_dof, n_vec), dtype=torch.complex128, device="cuda")
    op.fill_random(X, s.seed, n_total_cols=n_vec)
    Y = torch.empty_like(X)
    op.apply_H(X, Y)
    Ym = torch.empty_like(X)
    op.apply_H(X, Ym, prec="mixed")
    nodes = _sample_nodes(s, np.random.default_rng(11))
    rr = torch.tensor(np.stack([2 * nodes, 2 * nodes + 1], axis=1).ravel(), device="cuda")
    got = Y[rr].cpu().numpy().reshape(len(nodes), 2, n_vec)
    gotm = Ym[rr].cpu().numpy().reshape(len(nodes), 2, n_vec)
    del X, Y, Ym
    op.close()
    ref = rows.apply_rows(s, nodes, lambda r: synth.random_rows(s.seed, r, n_vec, n_vec), synth.veff, synth.bxc)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    errm = np.abs(gotm - ref).max() / np.abs(ref).max()
    print(f"[scale rows] {len(nodes)} nodes: fp64 rel err {err:.3e}, mixed {errm:.3e}", flush=True)
    assert err < 1e-12
    assert errm < 2e-6


def test_scale_workload_sampled_rows_matrix_free():
    """The large workload with the matrix-free local operator: rows of H_hat X
    from the oracle at sampled nodes, and the whole product against the
    cell-matrix path."""
    import synth
    from oracle import rows
    from paper_2410_02754_amd import Operator
    s = synth.config("scale")
    n_vec = 128
    X = torch.empty((s.n_dof, n_vec), dtype=torch.complex128, device="cuda")
    Ys = {}
    for form in ("matrix_free", "cell"):
        op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts, form=form)
        pts = op.quad_points().reshape(-1, 3)
        V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
        B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
        op.set_local(V, B)
        op.set_atoms(s.atoms)
        del V, B, pts
        op.fill_random(X, s.seed, n_total_cols=n_vec)
        Ys[form] = torch.empty_like(X)
        op.apply_H(X, Ys[form])
        op.close()
    scale = float(Ys["cell"].abs().max())
    d = float((Ys["matrix_free"] - Ys["cell"]).abs().max()) / scale
    nodes = _sample_nodes(s, np.random.default_rng(12))
    rr = torch.tensor(np.stack([2 * nodes, 2 * nodes + 1], axis=1).ravel(), device="cuda")
    got = Ys["matrix_free"][rr].cpu().numpy().reshape(len(nodes), 2, n_vec)
    del X, Ys
    ref = rows.apply_rows(s, nodes, lambda r: synth.random_rows(s.seed, r, n_vec, n_vec), synth.veff, synth.bxc)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"[scale rows matrix-free] {len(nodes)} nodes: rel err {err:.3e}; whole product vs cell path {d:.3e}",
          flush=True)
    assert err < 1e-12
    assert d < 1e-12
