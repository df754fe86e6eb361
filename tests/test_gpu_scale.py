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


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.05, -0.03, 0.02)])
def test_gll_kronecker_eigenvectors_full_scale(k):
    from paper_2410_02754_amd import Operator
    n_vec, v0, bvec = 128, -0.3, np.array([0.02, -0.05, 0.08])
    op = Operator((NC, NC, NC), (L, L, L), P, "gll", None, [k])
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
    print(f"[scale gll k={k}] fp64 max |H x - lam x| / (|lam| |x|) = {err:.3e}", flush=True)
    assert err < 1e-12
    op.apply_H(X, Y, prec="mixed")
    errm = float((Y - X * lam_d[None, :]).abs().max()) / scale
    print(f"[scale gll k={k}] mixed rel residual = {errm:.3e}", flush=True)
    assert errm < 2e-6
    op.close()
