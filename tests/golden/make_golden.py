"""Writes the stored expected values under tests/golden/ from the oracle.

Calls only oracle/ (and the seeded inputs of synth/).  Run from the repository
root:  python tests/golden/make_golden.py [dense|reduced|all]

dense   : the lowest eigenvalues of H_hat (dense Hermitian eigensolver on the
          assembled operator) of two small systems, the reference for ChFSI runs
          taken to convergence (Sec. III.B.2: the pass loop repeated until the
          residuals are small):
            tiny      3^3 cells, p = 4, L = 8 bohr, 2 atoms l <= 1  (3456 dofs)
            p6piece   2x2x3 cells, p = 6, h = 1.2 bohr, 1 atom l <= 2 (5184 dofs)
reduced : the FP64 ChFSI history of the reduced instance of the large workload
          (6^3 cells, p = 6, h = 1.2 bohr, N = 128, m = 24, 4 passes): Lanczos
          bound, per-pass bounds (a, b, a0) and Ritz values, final residual
          norms, and span probes Z = X X^H R at sampled rows (R: 4 seeded
          SplitMix64 columns), which do not depend on the basis chosen inside
          the block.  The assembled operator has about 1e8 nonzeros; its
          products with a block are split over column groups in worker
          processes (each computes H @ X[:, cols] with the oracle's operator).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import chfsi as och, hamiltonian as ham  # noqa: E402


def dense_systems():
    return {
        "tiny": synth.config("tiny"),
        "p6piece": synth.make_system("p6piece", n_cells=(2, 2, 3), box=(2.4, 2.4, 3.6), p=6, n_gauss=3,
                                     n_atoms=1, lmax=2, rcut_sigmas=6.0, n_vec=48, block=48, degree=24,
                                     passes=2, seed=4),
    }


def write_dense(n_keep=64):
    for name, s in dense_systems().items():
        t = time.time()
        _, H, _, _, _ = ham.build(s, synth.veff, synth.bxc)
        w = np.linalg.eigvalsh(H.toarray())
        path = os.path.join(HERE, f"{name}_dense_eigs.txt")
        with open(path, "w") as fh:
            fh.write(f"# lowest {n_keep} eigenvalues (Ha) of H_hat for the '{name}' system, dense Hermitian "
                     f"eigensolver on the oracle's assembled operator ({H.shape[0]} dofs); "
                     f"written by tests/golden/make_golden.py\n")
            for v in w[:n_keep]:
                fh.write(f"{v:.17e}\n")
        print(f"{name}: {H.shape[0]} dofs, {time.time() - t:.1f} s -> {path}", flush=True)


_H = None


def _apply_cols(cols):
    return _H @ _X[:, cols]


class PoolOperator:
    """H @ X with the column groups of X computed in forked workers (the oracle's
    operator is inherited by the workers; nothing else is changed)."""

    def __init__(self, H, workers):
        self.H, self.workers = H, workers
        self.shape, self.dtype = H.shape, H.dtype

    def __matmul__(self, X):
        global _H, _X
        import multiprocessing as mp
        X = np.asarray(X)
        if X.ndim == 1 or X.shape[1] < 2 * self.workers:
            return self.H @ X
        _H, _X = self.H, X
        groups = np.array_split(np.arange(X.shape[1]), self.workers)
        with mp.get_context("fork").Pool(self.workers) as pool:
            parts = pool.map(_apply_cols, groups)
        return np.concatenate(parts, axis=1)


def write_reduced(workers=8, n_probe=4, n_rows=256):
    s = synth.config("reduced")
    t = time.time()
    _, H, _, _, _ = ham.build(s, synth.veff, synth.bxc)
    print(f"reduced: {H.shape[0]} dofs, local nnz {H.loc.nnz}, assembled in {time.time() - t:.1f} s", flush=True)
    Hp = PoolOperator(H, workers)
    X0 = synth.start_block(s, s.n_dof)
    t = time.time()
    _, b = och.lanczos_bounds(H, synth.lanczos_start(s, s.n_dof), 40)
    print(f"Lanczos b = {b:.12f} ({time.time() - t:.1f} s)", flush=True)
    hist = []
    t = time.time()
    theta, X, r = och.run(Hp, X0, s.degree, s.passes, s.block, b, hist)
    print(f"{s.passes} passes in {time.time() - t:.1f} s", flush=True)
    rng = np.random.Generator(np.random.PCG64(7))
    rows = np.sort(rng.choice(s.n_dof, size=n_rows, replace=False))
    R = synth.random_block(99, s.n_dof, n_probe)
    Z = X @ (X.conj().T @ R)
    path = os.path.join(HERE, "reduced_fp64_4pass.txt")
    with open(path, "w") as fh:
        fh.write("# FP64 ChFSI on the reduced instance of the large workload (6^3 cells, p=6, h=1.2 bohr, "
                 "N=128 in one block, degree 24, 4 passes, start block seed 0, Lanczos seed 1, 40 steps); "
                 "written by tests/golden/make_golden.py from the oracle\n")
        fh.write(f"b {b:.17e}\n")
        for p, (th, rr, bounds) in enumerate(hist):
            if bounds is not None:
                fh.write(f"bounds {p} {bounds[0]:.17e} {bounds[1]:.17e} {bounds[2]:.17e}\n")
            fh.write(f"theta {p} " + " ".join(f"{v:.17e}" for v in th) + "\n")
        fh.write("resid " + " ".join(f"{v:.17e}" for v in r) + "\n")
        fh.write("probe_seed 99 probe_cols %d\n" % n_probe)
        for i, row in enumerate(rows):
            fh.write(f"z {row} " + " ".join(f"{v.real:.17e} {v.imag:.17e}" for v in Z[row]) + "\n")
    print(f"-> {path}", flush=True)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("dense", "all"):
        write_dense()
    if what in ("reduced", "all"):
        write_reduced()
