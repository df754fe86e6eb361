"""FP64 ChFSI parity on the reduced instance of the large workload (6^3 cells,
p=6, h=1.2 bohr, the large workload's generator densities, N=128, degree 24,
4 passes) against the oracle's stored history (tests/golden/reduced_fp64_4pass.txt,
written by tests/golden/make_golden.py): both sides filter with the same bounds,
the Ritz values must agree to 1e-10 Ha after every pass, and the block's span
through the basis-independent probes Z = X X^H R at the stored rows."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "reduced_fp64_4pass.txt")


def _load():
    g = {"bounds": {}, "theta": {}, "z": []}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            t = line.split()
            if t[0] == "b":
                g["b"] = float(t[1])
            elif t[0] == "bounds":
                g["bounds"][int(t[1])] = tuple(float(v) for v in t[2:5])
            elif t[0] == "theta":
                g["theta"][int(t[1])] = np.array([float(v) for v in t[2:]])
            elif t[0] == "resid":
                g["resid"] = np.array([float(v) for v in t[1:]])
            elif t[0] == "probe_seed":
                g["probe_seed"], g["probe_cols"] = int(t[1]), int(t[3])
            elif t[0] == "z":
                v = np.array([float(x) for x in t[2:]])
                g["z"].append((int(t[1]), v[0::2] + 1j * v[1::2]))
    return g


@pytest.mark.parametrize("form", ["cell", "matrix_free"])
def test_reduced_instance_four_passes_match_oracle(form):
    from paper_2410_02754_amd import Operator
    g = _load()
    s = synth.config("reduced")
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts, form=form)
    pts = op.quad_points().reshape(-1, 3)
    V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
    B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
    op.set_local(V, B)
    op.set_atoms(s.atoms)
    v0 = torch.tensor(synth.lanczos_start(s, s.n_dof), device="cuda")
    _, b = op.lanczos_bounds(v0, 40)
    print(f"[reduced {form}] Lanczos bound {b:.12f} vs oracle {g['b']:.12f}", flush=True)
    assert abs(b - g["b"]) < 1e-9 * abs(g["b"])
    X = torch.tensor(synth.start_block(s, s.n_dof), device="cuda")
    W = torch.empty_like(X)
    op.chol_gs(X)
    th, r = op.rayleigh_ritz(X, W)
    assert np.abs(th - g["theta"][0]).max() < 1e-10
    for p in range(1, s.passes + 1):
        a, bb, a0 = g["bounds"][p]
        op.cheb_filter(X, W, s.degree, a, bb, a0)
        op.chol_gs(X)
        th, r = op.rayleigh_ritz(X, W)
        d = np.abs(th - g["theta"][p]).max()
        print(f"[reduced {form}] pass {p}: max |dtheta| vs oracle {d:.2e} Ha", flush=True)
        assert d < 1e-10
    assert np.abs(r - g["resid"]).max() < 1e-8
    R = synth.random_block(g["probe_seed"], s.n_dof, g["probe_cols"])
    Xh = X.cpu().numpy()
    Z = Xh @ (Xh.conj().T @ R)
    rows = np.array([row for row, _ in g["z"]])
    Zo = np.stack([v for _, v in g["z"]])
    err = np.abs(Z[rows] - Zo).max() / np.abs(Zo).max()
    print(f"[reduced {form}] span probes rel err {err:.2e}", flush=True)
    assert err < 1e-8
    op.close()
