"""GPU checks at the full size of the batched workload: the 2x2x2 Monkhorst-Pack
grid on 12^3 cells, p=5 (432 000 spinor dofs per k-point, N = 384) plus the
6^3-cell Gamma system of the uneven set, in the launch form the benchmark
times (persistent colour-phase launches replayed from a hipGraph).

* rows of H_hat X at a k != 0 point against the oracle's rows, cell by cell,
  at sampled nodes near two atoms (FP64 and FP32 products);
* the batched filter equals, bit for bit, each task's own chfsi_cheb_filter.
"""
import numpy as np
import pytest

import synth
from test_gpu_scale import _sample_nodes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _op(s, stream):
    from paper_2410_02754_amd import Operator
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts, stream=stream.cuda_stream)
    pts = op.quad_points().reshape(-1, 3)
    V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
    B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
    op.set_local(V, B)
    op.set_atoms(s.atoms)
    return op


def test_kgrid_full_size_rows_and_batch():
    from oracle import rows
    from paper_2410_02754_amd import Batch
    kg = synth.config("kgrid")
    u1 = synth.config("uneven1")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        op = _op(kg, stream)
        # --- row-sampled parity at a k != 0 point, N = 384 as in the workload
        ik = 5
        print(f"[kgrid] k[{ik}] = {kg.kpts[ik]}", flush=True)
        X = torch.empty((kg.n_dof, kg.n_vec), dtype=torch.complex128, device="cuda")
        op.fill_random(X, kg.seed, n_total_cols=kg.n_vec)
        Y = torch.empty_like(X)
        op.apply_H(X, Y, ik=ik)
        Ym = torch.empty_like(X)
        op.apply_H(X, Ym, ik=ik, prec="mixed")
        nodes = _sample_nodes(kg, np.random.default_rng(3), n_near=24, n_far=8)
        rr = torch.tensor(np.stack([2 * nodes, 2 * nodes + 1], axis=1).ravel(), device="cuda")
        # the oracle evaluates the last 32 of the 384 columns (columns are independent)
        c0, nc = kg.n_vec - 32, 32
        got = Y[rr].cpu().numpy().reshape(len(nodes), 2, kg.n_vec)[:, :, c0:]
        gotm = Ym[rr].cpu().numpy().reshape(len(nodes), 2, kg.n_vec)[:, :, c0:]
        del Y, Ym
        ref = rows.apply_rows(kg, nodes, lambda r: synth.random_rows(kg.seed, r, nc, kg.n_vec, col0=c0),
                              synth.veff, synth.bxc, ik=ik)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        errm = np.abs(gotm - ref).max() / np.abs(ref).max()
        print(f"[kgrid rows] {len(nodes)} nodes: fp64 rel err {err:.3e}, mixed {errm:.3e}", flush=True)
        assert err < 1e-12
        assert errm < 2e-6
        # --- batched filter (8 k-points + the 6^3 Gamma system) vs per-task filters
        op1 = _op(u1, stream)
        tasks = []
        for k in range(len(kg.kpts)):
            Xk = torch.empty((kg.n_dof, kg.n_vec), dtype=torch.complex128, device="cuda")
            op.fill_random(Xk, kg.seed + 100 * k, n_total_cols=kg.n_vec)
            tasks.append((op, k, Xk, torch.empty_like(Xk)))
        X1 = torch.empty((u1.n_dof, u1.n_vec), dtype=torch.complex128, device="cuda")
        op1.fill_random(X1, u1.seed, n_total_cols=u1.n_vec)
        tasks.append((op1, 0, X1, torch.empty_like(X1)))
        del X
        bounds = []
        for o, k, Xt, Wt in tasks:
            v0 = torch.empty((Xt.shape[0], 1), dtype=torch.complex128, device="cuda")
            o.fill_random(v0, 7)
            lo, hi = o.lanczos_bounds(v0[:, 0], 30, ik=k)
            bounds.append((lo + 0.2 * (hi - lo), hi, lo - 0.3))
        a, b, a0 = (np.array(v) for v in zip(*bounds))
        X0 = [t[2].clone() for t in tasks]
        batch = Batch(tasks, kg.degree, prec="fp64")
        cols, _ = batch.tiles()
        print(f"[kgrid batch] tile widths {cols}", flush=True)
        batch.filter(a, b, a0)
        torch.cuda.synchronize()
        for i, (o, k, Xt, Wt) in enumerate(tasks):
            Yt = X0[i].clone()
            o.cheb_filter(Yt, Wt, kg.degree, a[i], b[i], a0[i], ik=k)
            torch.cuda.synchronize()
            assert torch.isfinite(Yt).all()
            assert torch.equal(Yt, Xt), f"task {i} differs"
            del Yt
        print("[kgrid batch] batched filter bitwise equal to per-task filters", flush=True)
        batch.close()
        op1.close()
        op.close()
