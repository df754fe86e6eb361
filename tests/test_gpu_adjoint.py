"""GPU adjoint: chfsi_apply_H_backward / chfsi_cheb_filter_backward through the
C ABI and torch.autograd, against the oracle's plain adjoint, the
density/magnetisation closed form (eqn:rho, eqn:mag) and central finite
differences of the GPU forward path."""
import numpy as np
import pytest

import synth
from oracle import adjoint as oadj, chfsi as och, hamiltonian as ham

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _setup(s, form="cell"):
    from paper_2410_02754_amd import Operator
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts, form=form)
    pts = op.quad_points().reshape(-1, 3)
    V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
    B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
    op.set_local(V, B)
    op.set_atoms(s.atoms)
    return op, V, B


SMALL = lambda: synth.make_system("adjs", n_cells=(2, 3, 2), box=(4.0, 5.0, 4.0), p=3,
                                  kpts=[(0.1, -0.15, 0.05)], n_atoms=2, lmax=1, rcut_sigmas=5.0, n_vec=5)


@pytest.mark.parametrize("form", ["cell", "matrix_free"])
def test_apply_backward_matches_oracle_and_closed_form(form):
    from paper_2410_02754_amd.autograd import apply_h
    s = SMALL()
    mesh, H, MD, Vo, Bo = ham.build(s, synth.veff, synth.bxc)
    op, V, B = _setup(s, form)
    X0 = synth.random_block(3, s.n_dof, s.n_vec)
    X = torch.tensor(X0, device="cuda", requires_grad=True)
    Vr = V.clone().requires_grad_(True)
    Br = B.clone().requires_grad_(True)
    Y = apply_h(X, Vr, Br, op)
    L = (X.conj() * Y).real.sum()          # sum_n Re <x_n | H x_n>
    L.backward()
    rho, m = oadj.density_magnetisation(mesh, MD, X0)
    wJ = mesh.wq * mesh.J
    dV = Vr.grad.cpu().numpy()
    dB = Br.grad.cpu().numpy()
    print(f"[adjoint apply] |dV - wJ rho| {np.abs(dV - wJ * rho).max():.2e} (scale {np.abs(wJ * rho).max():.2e})")
    assert np.abs(dV - wJ * rho).max() < 1e-12 * np.abs(wJ * rho).max()
    assert np.abs(dB - wJ[None, :, None] * m).max() < 1e-12 * np.abs(wJ * rho).max()
    ref = 2 * (H @ X0)
    assert np.abs(X.grad.cpu().numpy() - ref).max() < 1e-12 * np.abs(ref).max()
    op.close()


@pytest.mark.parametrize("form", ["cell", "matrix_free"])
def test_filter_backward_matches_oracle(form):
    s = SMALL()
    mesh, H, MD, Vo, Bo = ham.build(s, synth.veff, synth.bxc)
    op, V, B = _setup(s, form)
    lam = np.linalg.eigvalsh(H.toarray())
    m, a, b, a0 = 7, float(lam[30]), float(lam[-1] + 1.0), float(lam[0])
    X0 = synth.random_block(4, s.n_dof, s.n_vec)
    G0 = synth.random_block(5, s.n_dof, s.n_vec)
    Xb_o, dV_o, dB_o = oadj.filter_backward(H, mesh, MD, X0, G0, m, a, b, a0)
    X = torch.tensor(X0, device="cuda")
    G = torch.tensor(G0, device="cuda")
    outs = []
    for ck in (1, 2, 3, 4, 16):
        Xb = torch.empty_like(X)
        dV = torch.zeros_like(V)
        dB = torch.zeros_like(B)
        op.cheb_filter_backward(X, G, Xb, dV, dB, m, a, b, a0, ckpt_every=ck)
        outs.append((Xb.cpu().numpy(), dV.cpu().numpy(), dB.cpu().numpy()))
    Xb, dV, dB = outs[0]
    ex = np.abs(Xb - Xb_o).max() / np.abs(Xb_o).max()
    ev = np.abs(dV - dV_o).max() / np.abs(dV_o).max()
    eb = np.abs(dB - dB_o).max() / np.abs(dB_o).max()
    print(f"[adjoint filter] rel err Xbar {ex:.2e} dV {ev:.2e} dB {eb:.2e}")
    assert ex < 1e-11 and ev < 1e-11 and eb < 1e-11
    for o in outs[1:]:                     # recomputation is bitwise reproducible
        assert all(np.array_equal(u, v) for u, v in zip(o, outs[0]))
    op.close()


def test_filter_autograd_finite_differences_on_gpu():
    """L = sum ||filter(X)||^2; central differences (h = 1e-6) of the GPU forward
    path along random directions of X, V and B."""
    from paper_2410_02754_amd.autograd import cheb_filter
    s = SMALL()
    op, V, B = _setup(s)
    mesh, H, _, _, _ = ham.build(s, synth.veff, synth.bxc)
    lam = np.linalg.eigvalsh(H.toarray())
    m, a, b, a0 = 6, float(lam[30]), float(lam[-1] + 1.0), float(lam[0])
    X = torch.tensor(synth.random_block(6, s.n_dof, s.n_vec), device="cuda", requires_grad=True)
    Vr = V.clone().requires_grad_(True)
    Br = B.clone().requires_grad_(True)
    Y = cheb_filter(X, Vr, Br, op, m, a, b, a0, ckpt_every=4)
    (Y.abs() ** 2).sum().backward()

    def L(Xp, Vp, Bp):
        with torch.no_grad():
            return float((cheb_filter(Xp, Vp, Bp, op, m, a, b, a0).abs() ** 2).sum())
    gen = torch.Generator(device="cuda").manual_seed(0)
    h = 1e-6
    D = torch.randn(X.shape, dtype=torch.complex128, device="cuda", generator=gen)
    fd = (L(X.detach() + h * D, V, B) - L(X.detach() - h * D, V, B)) / (2 * h)
    an = float(torch.real(torch.vdot(X.grad.flatten(), D.flatten())))
    assert abs(fd - an) < 1e-6 * abs(an)
    dVd = torch.randn(V.shape, dtype=torch.float64, device="cuda", generator=gen)
    fd = (L(X.detach(), V + h * dVd, B) - L(X.detach(), V - h * dVd, B)) / (2 * h)
    an = float((Vr.grad * dVd).sum())
    print(f"[adjoint fd] dV: fd {fd:.10e} analytic {an:.10e}")
    assert abs(fd - an) < 1e-6 * abs(an)
    dBd = torch.randn(B.shape, dtype=torch.float64, device="cuda", generator=gen)
    fd = (L(X.detach(), V, B + h * dBd) - L(X.detach(), V, B - h * dBd)) / (2 * h)
    an = float((Br.grad * dBd).sum())
    assert abs(fd - an) < 1e-6 * abs(an)
    op.close()


def test_adjoint_workload_size_closed_form():
    """The adjoint workload (10^3 cells, p=5, 250k dofs, N=256): the apply
    adjoint reproduces the density/magnetisation closed form, and the filter
    adjoint (m=16, checkpoints every 4) satisfies the adjoint identity
    Re <Ybar, p(H) Z> = Re <p(H) Ybar, Z> with Xbar = p(H) Ybar."""
    from paper_2410_02754_amd.autograd import apply_h
    s = synth.config("adjoint")
    op, V, B = _setup(s)
    mesh = ham.mesh_for(s)
    MD = mesh.lumped_mass()
    X0 = synth.start_block(s, s.n_dof)
    X = torch.tensor(X0, device="cuda", requires_grad=True)
    Vr = V.clone().requires_grad_(True)
    Br = B.clone().requires_grad_(True)
    L = (X.conj() * apply_h(X, Vr, Br, op)).real.sum()
    L.backward()
    rho, mm = oadj.density_magnetisation(mesh, MD, X0)
    wJ = mesh.wq * mesh.J
    scale = np.abs(wJ * rho).max()
    ev = np.abs(Vr.grad.cpu().numpy() - wJ * rho).max() / scale
    eb = np.abs(Br.grad.cpu().numpy() - wJ[None, :, None] * mm).max() / scale
    print(f"[adjoint workload] closed form rel err dV {ev:.2e} dB {eb:.2e}")
    assert ev < 1e-12 and eb < 1e-12
    # filter adjoint identity with the workload's degree and checkpointing
    v0 = torch.tensor(synth.lanczos_start(s, s.n_dof), device="cuda")
    lo, hi = op.lanczos_bounds(v0, 40)
    a, a0 = lo + 0.3 * (hi - lo), lo - 0.1
    G = torch.tensor(synth.random_block(9, s.n_dof, s.n_vec), device="cuda")
    Xb = torch.empty_like(G)
    dV = torch.zeros_like(V)
    dB = torch.zeros_like(B)
    import time
    torch.cuda.synchronize(); t = time.perf_counter()
    op.cheb_filter_backward(X.detach(), G, Xb, dV, dB, 16, a, hi, a0, ckpt_every=4)
    torch.cuda.synchronize(); tb = time.perf_counter() - t
    Z = X.detach().clone()
    W = torch.empty_like(Z)
    t = time.perf_counter()
    op.cheb_filter(Z, W, 16, a, hi, a0)
    torch.cuda.synchronize(); tf = time.perf_counter() - t
    lhs = torch.vdot(G.flatten(), Z.flatten())
    rhs = torch.vdot(Xb.flatten(), X.detach().flatten())
    rel = float((lhs - rhs).abs() / lhs.abs())
    print(f"[adjoint workload] forward {tf:.3f} s backward {tb:.3f} s adjoint identity rel {rel:.2e}")
    assert rel < 1e-10
    op.close()


def test_autograd_backward_uses_the_forward_fields():
    """Two forwards on different fields, then the backward of the first: the
    adjoint must run with the operator of its own forward (H(V1, B1)), not the
    one the context holds after the second forward."""
    from paper_2410_02754_amd.autograd import apply_h, cheb_filter
    s = SMALL()
    mesh, H1, MD, Vo, Bo = ham.build(s, synth.veff, synth.bxc)
    op, V, B = _setup(s)
    V2 = (1.5 * V + 0.2).contiguous()
    B2 = (-0.7 * B).contiguous()
    H2 = ham.build(s, synth.veff, synth.bxc, V=1.5 * Vo + 0.2, B=-0.7 * Bo)[1]
    lam = np.linalg.eigvalsh(H1.toarray())
    m, a, b, a0 = 5, float(lam[30]), float(lam[-1] + 2.0), float(lam[0])
    X0 = synth.random_block(11, s.n_dof, s.n_vec)
    G0 = synth.random_block(12, s.n_dof, s.n_vec)
    # apply: Xbar = H1 G
    X = torch.tensor(X0, device="cuda", requires_grad=True)
    V1r, B1r = V.clone().requires_grad_(True), B.clone().requires_grad_(True)
    Y1 = apply_h(X, V1r, B1r, op)
    Y2 = apply_h(X.detach(), V2, B2, op)
    Y1.backward(torch.tensor(G0, device="cuda"))
    ref = H1 @ G0
    err = np.abs(X.grad.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert np.abs(Y2.detach().cpu().numpy() - H2 @ X0).max() < 1e-12 * np.abs(H2 @ X0).max()
    print(f"[autograd fields] apply Xbar rel err {err:.2e}")
    assert err < 1e-12
    # filter: Xbar, dV, dB of the first forward against the oracle adjoint with H1
    Xb_o, dV_o, dB_o = oadj.filter_backward(H1, mesh, MD, X0, G0, m, a, b, a0)
    X = torch.tensor(X0, device="cuda", requires_grad=True)
    V1r, B1r = V.clone().requires_grad_(True), B.clone().requires_grad_(True)
    Z1 = cheb_filter(X, V1r, B1r, op, m, a, b, a0, ckpt_every=2)
    cheb_filter(X.detach(), V2, B2, op, m, a, b, a0)
    Z1.backward(torch.tensor(G0, device="cuda"))
    ex = np.abs(X.grad.cpu().numpy() - Xb_o).max() / np.abs(Xb_o).max()
    ev = np.abs(V1r.grad.cpu().numpy() - dV_o).max() / np.abs(dV_o).max()
    eb = np.abs(B1r.grad.cpu().numpy() - dB_o).max() / np.abs(dB_o).max()
    print(f"[autograd fields] filter rel err Xbar {ex:.2e} dV {ev:.2e} dB {eb:.2e}")
    assert ex < 1e-11 and ev < 1e-11 and eb < 1e-11
    op.close()
