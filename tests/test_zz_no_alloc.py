"""The allocation-free filter entry point (chfsi_cheb_filter_noalloc) against
chfsi_cheb_filter: equal outputs, bit for bit, on two calls in a row (the
second with a smaller input), in FP64 and mixed precision, including a block
wide enough that the contraction partials do not fit the fixed scratch at once
(the columns then run in groups); a width whose coefficient arrays alone exceed
the fixed scratch is rejected before any launch."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIXED = 64 << 20          # CHFSI_NOALLOC_SCRATCH_BYTES


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _op(s):
    from paper_2410_02754_amd import Operator
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts)
    pts = op.quad_points().reshape(-1, 3)
    V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
    B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
    op.set_local(V, B)
    op.set_atoms(s.atoms)
    return op


def _many_atoms():
    # 60 l <= 2 atoms whose cut-off sphere (5.6 bohr) covers the 4-bohr box
    # from every point: each atom's support is the whole mesh, 27 chunks
    # (13 full windows of 1024 nodes in two 512-entry chunks + one half window)
    return synth.make_system("many_atoms", n_cells=(4, 4, 4), box=(4.0, 4.0, 4.0), p=6, n_atoms=60,
                             lmax=2, rcut_sigmas=8.0, n_vec=320, degree=4)


def _bounds(op, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    v0 = torch.randn(op.n_dof, dtype=torch.complex128, device="cuda", generator=g)
    lo, hi = op.lanczos_bounds(v0, 30)
    return lo + 0.3 * (hi - lo), hi, lo - 0.1


def _block(op, n, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn(op.n_dof, n, dtype=torch.complex128, device="cuda", generator=g)


def _compare(op, X0, degree, a, b, a0, prec):
    X1, X2 = X0.clone(), X0.clone()
    W1, W2 = torch.empty_like(X0), torch.empty_like(X0)
    op.cheb_filter(X1, W1, degree, a, b, a0, prec=prec)
    op.cheb_filter_noalloc(X2, W2, degree, a, b, a0, prec=prec)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(X1)).all()
    d = (X1 - X2).abs().max().item()
    _say(f"  {prec} n_vec={X0.shape[1]}: max |noalloc - filter| = {d:.3e}")
    assert torch.equal(X1, X2)


def test_noalloc_filter_equals_filter_two_calls():
    s = _many_atoms()
    mr, n_chunks, n_atoms = 18, 60 * 27, 60
    per_col = n_chunks * mr * 16
    head = 2 * n_atoms * mr * 16
    # the first call's width does not fit the fixed scratch in one contraction
    assert (per_col + head) * 320 > FIXED
    _say("many_atoms: 4^3 cells p=6, 60 atoms l<=2, n_vec 320 then 24")
    op = _op(s)
    a, b, a0 = _bounds(op, 1)
    _compare(op, _block(op, 320, 2), 4, a, b, a0, "fp64")      # grouped contraction
    _compare(op, _block(op, 24, 3), 4, a, b, a0, "mixed")      # second call, smaller input
    op.close()
    t = synth.config("tiny")
    _say("tiny: 3^3 cells p=4, 2 atoms, n_vec 16")
    op = _op(t)
    a, b, a0 = _bounds(op, 4)
    _compare(op, _block(op, 16, 5), t.degree, a, b, a0, "fp64")
    _compare(op, _block(op, 9, 6), t.degree, a, b, a0, "mixed")
    op.close()


def test_noalloc_filter_rejects_too_wide_block():
    from paper_2410_02754_amd._lib import ChfsiError
    s = _many_atoms()
    op = _op(s)
    n = 2000     # 2 * 60 * 18 * 2000 * 16 bytes of coefficients alone exceed the fixed scratch
    assert 2 * 60 * 18 * n * 16 > FIXED
    X = _block(op, n, 7)
    W = torch.empty_like(X)
    X0 = X.clone()
    a, b, a0 = _bounds(op, 1)
    with pytest.raises(ChfsiError) as e:
        op.cheb_filter_noalloc(X, W, 4, a, b, a0)
    assert e.value.code == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(X, X0)            # nothing ran
    # the same context still filters through the fixed scratch afterwards
    _compare(op, _block(op, 8, 8), 3, a, b, a0, "fp64")
    op.close()
