"""Batched filter: 8 k-points of a 2x2x2 Monkhorst-Pack grid on one mesh plus
independent Gamma systems of uneven size and width, in persistent colour-phase
launches captured in a hipGraph, against per-task chfsi_cheb_filter (bitwise)
and against the oracle."""
import numpy as np
import pytest

import synth
from oracle import chfsi as och, hamiltonian as ham

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _op(s, stream, form="cell"):
    from paper_2410_02754_amd import Operator
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts, stream=stream.cuda_stream, form=form)
    pts = op.quad_points().reshape(-1, 3)
    V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
    B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
    op.set_local(V, B)
    op.set_atoms(s.atoms)
    return op


def _systems(bmag=0.1):
    L = 4.8
    kg = synth.make_system("kg", n_cells=(4, 4, 4), box=(L, L, L), p=3, kpts=synth.monkhorst_pack(2, (L, L, L)),
                           n_atoms=2, lmax=1, rcut_sigmas=5.0, n_vec=40, b_mag=bmag, seed=1)
    others = [synth.make_system("u1", n_cells=(2, 2, 2), box=(2.4, 2.4, 2.4), p=3, n_atoms=1, lmax=1,
                                rcut_sigmas=4.0, n_vec=16, seed=2),
              synth.make_system("u2", n_cells=(3, 2, 2), box=(3.6, 2.4, 2.4), p=3, n_atoms=1, lmax=2,
                                rcut_sigmas=4.0, n_vec=70, seed=3)]
    return kg, others


@pytest.mark.parametrize("prec,mf", [("fp64", False), ("mixed", False), ("fp64", True), ("mixed", True)])
def test_batch_equals_per_task_bitwise(prec, mf):
    """mf: the second uneven system uses the matrix-free form (its own launches
    inside the batched, graph-captured filter)."""
    from paper_2410_02754_amd import Batch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        kg, others = _systems()
        ops = [_op(kg, stream)] + [_op(s, stream, "matrix_free" if (mf and j == 1) else "cell")
                                   for j, s in enumerate(others)]
        tasks, blocks = [], []
        for ik in range(8):
            X = torch.tensor(synth.random_block(10 + ik, kg.n_dof, kg.n_vec), device="cuda")
            tasks.append((ops[0], ik, X, torch.empty_like(X)))
        for j, s in enumerate(others):
            X = torch.tensor(synth.random_block(20 + j, s.n_dof, s.n_vec), device="cuda")
            tasks.append((ops[1 + j], 0, X, torch.empty_like(X)))
        X0 = [t[2].clone() for t in tasks]
        degree = 9
        bounds = []
        for op, ik, X, W in tasks:
            v0 = torch.tensor(synth.lanczos_start(kg, X.shape[0]), device="cuda")
            lo, hi = op.lanczos_bounds(v0, 20, ik=ik)
            bounds.append((lo + 0.25 * (hi - lo), hi, lo - 0.5))
        a, b, a0 = (np.array(v) for v in zip(*bounds))
        batch = Batch(tasks, degree, prec=prec)
        cols, tune = batch.tiles()
        print(f"[batch {prec}] tile widths {cols}", flush=True)
        batch.filter(a, b, a0)
        torch.cuda.synchronize()
        got = [t[2].clone() for t in tasks]
        # per task, the single-operator filter
        for i, (op, ik, X, W) in enumerate(tasks):
            Y = X0[i].clone()
            op.cheb_filter(Y, torch.empty_like(Y), degree, a[i], b[i], a0[i], ik=ik, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(Y, got[i]), f"task {i} differs"
        # graph replay with the same bounds, then with new bounds
        for i, t in enumerate(tasks):
            t[2].copy_(X0[i])
        batch.filter(a, b, a0)
        torch.cuda.synchronize()
        for i, t in enumerate(tasks):
            assert torch.equal(t[2], got[i])
            t[2].copy_(X0[i])
        batch.filter(a * 0.9 + 0.1 * a0, b, a0)
        torch.cuda.synchronize()
        for i, (op, ik, X, W) in enumerate(tasks):
            Y = X0[i].clone()
            op.cheb_filter(Y, torch.empty_like(Y), degree, a[i] * 0.9 + 0.1 * a0[i], b[i], a0[i], ik=ik, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(Y, X)
        batch.close()
        for op in ops:
            op.close()


def test_batch_kpoint_parity_and_time_reversal():
    """One k-point task against the oracle's filter; and with B = 0 the Ritz
    values after a batched filter + CholGS + RR satisfy eps(k) = eps(-k)
    for the +-k pairs of the grid (time reversal)."""
    from paper_2410_02754_amd import Batch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        kg, _ = _systems(bmag=0.0)
        op = _op(kg, stream)
        tasks = []
        X0 = synth.random_block(5, kg.n_dof, kg.n_vec)
        # time reversal Theta = i sigma_y K: (u_up, u_dn) -> (conj(u_dn), -conj(u_up));
        # the -k task starts from Theta X0 so the two filtered subspaces are Theta-related
        TX0 = np.empty_like(X0)
        TX0[0::2] = np.conj(X0[1::2])
        TX0[1::2] = -np.conj(X0[0::2])
        k = kg.kpts
        for ik in range(8):
            j = int(np.argmin(np.linalg.norm(k + k[ik], axis=1)))
            X = torch.tensor(X0 if ik < j else TX0, device="cuda")
            tasks.append((op, ik, X, torch.empty_like(X)))
        H3 = ham.build(kg, synth.veff, synth.bxc, ik=3)[1]
        lam = np.linalg.eigvalsh(H3.toarray())
        a, b, a0 = float(lam[60]), float(lam[-1] + 1.0), float(lam[0] - 0.2)
        batch = Batch(tasks, 8)
        batch.filter(a, b, a0)
        torch.cuda.synchronize()
        j3 = int(np.argmin(np.linalg.norm(kg.kpts + kg.kpts[3], axis=1)))
        ref = och.cheb_filter(H3, X0 if 3 < j3 else TX0, 8, a, b, a0)
        err = np.abs(tasks[3][2].cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"[batch k parity] rel err {err:.2e}", flush=True)
        assert err < 1e-11
        th = []
        for op_, ik, X, W in tasks:
            op_.chol_gs(X)
            t, _ = op_.rayleigh_ritz(X, W, ik=ik)
            th.append(t)
        for i in range(8):
            j = int(np.argmin(np.linalg.norm(k + k[i], axis=1)))
            d = np.abs(th[i][:20] - th[j][:20]).max()
            assert d < 1e-9, (i, j, d)
        batch.close()
        op.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_graph_replays_across_chfsi_passes(prec):
    """The ChFSI pass loop with one batch: filter, CholGS + Rayleigh-Ritz on every
    task (which grows each context's own scratch buffers), filter again with the
    same bounds and then with new ones.  Every batched filter is bitwise equal to
    the per-task chfsi_cheb_filter of the same block, and the graph is captured
    once and replayed for the later passes."""
    from paper_2410_02754_amd import Batch
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        kg, others = _systems()
        ops = [_op(kg, stream)] + [_op(s, stream) for s in others]
        tasks = []
        for ik in (0, 5):
            X = torch.tensor(synth.random_block(30 + ik, kg.n_dof, kg.n_vec), device="cuda")
            tasks.append((ops[0], ik, X, torch.empty_like(X)))
        for j, s in enumerate(others):
            X = torch.tensor(synth.random_block(40 + j, s.n_dof, s.n_vec), device="cuda")
            tasks.append((ops[1 + j], 0, X, torch.empty_like(X)))
        degree = 7
        a, b, a0 = [], [], []
        for op, ik, X, W in tasks:
            v0 = torch.tensor(synth.lanczos_start(kg, X.shape[0]), device="cuda")
            lo, hi = op.lanczos_bounds(v0, 20, ik=ik)
            a.append(lo + 0.3 * (hi - lo)), b.append(hi), a0.append(lo - 0.5)
        a, b, a0 = np.array(a), np.array(b), np.array(a0)
        batch = Batch(tasks, degree, prec=prec)
        for p, (aa, bb, cc) in enumerate([(a, b, a0), (a, b, a0), (0.8 * a + 0.2 * a0, 1.1 * b, a0 - 0.3)]):
            before = [t[2].clone() for t in tasks]
            batch.filter(aa, bb, cc)
            torch.cuda.synchronize()
            for i, (op, ik, X, W) in enumerate(tasks):
                Y = before[i].clone()
                op.cheb_filter(Y, torch.empty_like(Y), degree, aa[i], bb[i], cc[i], ik=ik, prec=prec)
                torch.cuda.synchronize()
                assert torch.equal(Y, X), f"pass {p}: task {i} differs from its own filter"
            # CholGS + RR on every task, as in the pass loop; widens the gram scratch
            for op, ik, X, W in tasks:
                op.chol_gs(X)
                op.rayleigh_ritz(X, W, ik=ik)
            torch.cuda.synchronize()
        info = batch.graph_info()
        print(f"[batch replay {prec}] {info}", flush=True)
        assert info["captures"] == 1 and info["replays"] == 2
        # rebuilding a context's operator invalidates the batch
        pts = ops[1].quad_points().reshape(-1, 3)
        s1 = others[0]
        V = torch.tensor(synth.veff(s1, pts).reshape(ops[1].n_cells, ops[1].nq3), device="cuda")
        B = torch.tensor(synth.bxc(s1, pts).reshape(ops[1].n_cells, ops[1].nq3, 3), device="cuda")
        ops[1].set_local(V, B)
        with pytest.raises(Exception, match="CHFSI_ESTATE"):
            batch.filter(a, b, a0)
        batch.close()
        for op in ops:
            op.close()
