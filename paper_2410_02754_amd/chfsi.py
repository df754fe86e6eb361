"""Thin wrapper of one chfsi context (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
from typing import Iterable, Optional, Sequence

import numpy as np

from . import _lib

PREC_FP64 = 0
PREC_MIXED = 1
FORMS = {"cell": 0, "matrix_free": 1}
_PREC = {"fp64": PREC_FP64, "mixed": PREC_MIXED, PREC_FP64: PREC_FP64, PREC_MIXED: PREC_MIXED}


def _torch():
    import torch
    return torch


def _block(t, name):
    """(pointer, ld, n_vec) of a row-major complex128 CUDA matrix or column block."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise ValueError(f"{name} must be contiguous")
        return t.data_ptr(), 1, 1
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D row-major block (unit column stride)")
    return t.data_ptr(), t.stride(0), t.shape[1]


class Operator:
    """H_hat^k = M_D^{-1/2} H^k M_D^{-1/2} on one GPU, with the ChFSI steps.

    All tensors must live on the current CUDA (HIP) device; every call is
    enqueued on the torch stream that was current when the operator was built.
    """

    def __init__(self, n_cells: Sequence[int], box: Sequence[float], p: int, quad: str = "gl",
                 n_q: Optional[int] = None, kpts=None, stream=None, form: str = "cell"):
        torch = _torch()
        self.lib = _lib.load()
        k = np.zeros((1, 3)) if kpts is None else np.ascontiguousarray(kpts, dtype=np.float64).reshape(-1, 3)
        self._kbuf = (C.c_double * k.size)(*k.ravel().tolist())
        d = _lib.MeshDesc()
        d.n_cells = (C.c_int * 3)(*[int(x) for x in n_cells])
        d.box = (C.c_double * 3)(*[float(x) for x in box])
        d.p = int(p)
        d.quad = 1 if quad == "gll" else 0
        d.n_q = int(n_q if n_q else p + 1)
        d.n_k = int(k.shape[0])
        d.kpts = C.cast(self._kbuf, C.POINTER(C.c_double))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        ctx = C.c_void_p()
        rc = self.lib.chfsi_create(C.byref(d), C.c_void_p(stream), C.byref(ctx))
        _lib.check(rc, None)
        self.ctx = ctx
        nn, nd = C.c_int64(), C.c_int64()
        ne, nq3, ncol = C.c_int(), C.c_int(), C.c_int()
        _lib.check(self.lib.chfsi_sizes(ctx, C.byref(nn), C.byref(nd), C.byref(ne), C.byref(nq3),
                                        C.byref(ncol)), ctx)
        self.n_nodes, self.n_dof = nn.value, nd.value
        self.n_cells, self.nq3, self.n_colours = ne.value, nq3.value, ncol.value
        self.n_k = int(k.shape[0])
        self.form = "cell"
        if form != "cell":
            self.set_form(form)

    def set_form(self, form: str):
        """"cell" (stored cell matrices) or "matrix_free" (sum factorisation);
        the local operator must be set again afterwards."""
        if form not in FORMS:
            raise ValueError(f"form must be one of {sorted(FORMS)}")
        self._chk(self.lib.chfsi_set_apply_form(self.ctx, FORMS[form]))
        self.form = form

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.chfsi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        _lib.check(rc, self.ctx)

    # ---------------------------------------------------------------- setup
    def quad_points(self) -> np.ndarray:
        out = np.zeros((self.n_cells, self.nq3, 3))
        self._chk(self.lib.chfsi_quad_points(self.ctx, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def set_local(self, V, B):
        torch = _torch()
        for t, shp in ((V, (self.n_cells, self.nq3)), (B, (self.n_cells, self.nq3, 3))):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
                raise ValueError(f"field must be a contiguous float64 CUDA tensor of shape {shp}")
        self._chk(self.lib.chfsi_set_local(self.ctx, C.c_void_p(V.data_ptr()), C.c_void_p(B.data_ptr())))

    def set_atoms(self, atoms: Iterable, delta_overrides=None):
        atoms = list(atoms)
        arr = (_lib.AtomDesc * max(1, len(atoms)))()
        keep = []
        for i, a in enumerate(atoms):
            arr[i].pos = (C.c_double * 3)(*[float(x) for x in a.pos])
            arr[i].lmax = int(a.lmax)
            arr[i].sigma = float(a.sigma)
            arr[i].rcut = float(a.rcut)
            d0 = list(a.d0) + [0.0] * (3 - len(a.d0))
            arr[i].d0 = (C.c_double * 3)(*d0[:3])
            arr[i].dso = float(a.dso)
            ov = None if delta_overrides is None else delta_overrides[i]
            if ov is not None:
                buf = np.ascontiguousarray(np.asarray(ov, dtype=np.complex128)).view(np.float64)
                keep.append(buf)
                arr[i].delta_override = buf.ctypes.data_as(C.POINTER(C.c_double))
            else:
                arr[i].delta_override = None
        self._chk(self.lib.chfsi_set_atoms(self.ctx, len(atoms), arr))

    # ---------------------------------------------------------------- hot path
    def apply_H(self, X, Y, ik: int = 0, prec="fp64"):
        px, ldx, n = _block(X, "X")
        py, ldy, ny = _block(Y, "Y")
        if ny != n or X.shape[0] != self.n_dof or Y.shape[0] != self.n_dof:
            raise ValueError("X and Y must both be [2M][n_vec]")
        self._chk(self.lib.chfsi_apply_H(self.ctx, ik, C.c_void_p(px), ldx, C.c_void_p(py), ldy, n,
                                         _PREC[prec]))
        return Y

    def cheb_filter(self, X, work, degree: int, a: float, b: float, a0: float, ik: int = 0,
                    prec="fp64"):
        px, ldx, n = _block(X, "X")
        pw, ldw, nw = _block(work, "work")
        if nw < n or X.shape[0] != self.n_dof or work.shape[0] != self.n_dof:
            raise ValueError("work must be [2M][>= n_vec]")
        self._chk(self.lib.chfsi_cheb_filter(self.ctx, ik, C.c_void_p(px), ldx, C.c_void_p(pw), ldw,
                                             n, int(degree), float(a), float(b), float(a0),
                                             _PREC[prec]))
        return X

    def cheb_filter_noalloc(self, X, work, degree: int, a: float, b: float, a0: float, ik: int = 0,
                            prec="fp64"):
        """cheb_filter with the library's fixed nonlocal scratch (no device allocation)."""
        px, ldx, n = _block(X, "X")
        pw, ldw, nw = _block(work, "work")
        if nw < n or X.shape[0] != self.n_dof or work.shape[0] != self.n_dof:
            raise ValueError("work must be [2M][>= n_vec]")
        self._chk(self.lib.chfsi_cheb_filter_noalloc(self.ctx, ik, C.c_void_p(px), ldx, C.c_void_p(pw), ldw,
                                                     n, int(degree), float(a), float(b), float(a0),
                                                     _PREC[prec]))
        return X

    def ritz_residual(self, X, W, theta):
        """W <- W - X diag(theta) (R = H X - X Theta when W = H X)."""
        px, ldx, n = _block(X, "X")
        pw, ldw, nw = _block(W, "W")
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if nw != n or th.size < n:
            raise ValueError("W and theta must match X")
        self._chk(self.lib.chfsi_ritz_residual(self.ctx, C.c_void_p(px), ldx, C.c_void_p(pw), ldw, n,
                                               th.ctypes.data_as(C.POINTER(C.c_double))))
        return W

    def cheb_filter_resid(self, X, R, theta, work, degree: int, a: float, b: float, a0: float,
                          ik: int = 0, prec="fp64"):
        """Residual form of the filter; work must be [2M][>= 2 n_vec]."""
        px, ldx, n = _block(X, "X")
        pr, ldr, nr = _block(R, "R")
        pw, ldw, nw = _block(work, "work")
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if nr != n or nw < 2 * n or th.size < n:
            raise ValueError("R must match X, work must be [2M][>= 2 n_vec]")
        self._chk(self.lib.chfsi_cheb_filter_resid(self.ctx, ik, C.c_void_p(px), ldx, C.c_void_p(pr), ldr,
                                                   th.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(pw), ldw,
                                                   n, int(degree), float(a), float(b), float(a0), _PREC[prec]))
        return X

    def chol_gs(self, X):
        px, ldx, n = _block(X, "X")
        bad = C.c_int(-1)
        rc = self.lib.chfsi_chol_gs(self.ctx, C.c_void_p(px), ldx, n, C.byref(bad))
        if rc != 0:
            err = _lib.ChfsiError(rc, self.lib.chfsi_last_error(self.ctx).decode())
            err.bad_col = bad.value
            raise err
        return X

    def overlap(self, X, Y) -> np.ndarray:
        """S = X^H Y (host complex128 [n][n])."""
        px, ldx, n = _block(X, "X")
        py, ldy, ny = _block(Y, "Y")
        if ny != n:
            raise ValueError("X and Y must have the same width")
        S = np.zeros((n, n), dtype=np.complex128)
        self._chk(self.lib.chfsi_overlap(self.ctx, C.c_void_p(px), ldx, C.c_void_p(py), ldy, n,
                                         S.ctypes.data_as(C.POINTER(C.c_double))))
        return S

    def workspace_bytes(self, n_vec: int, op: str, ik: int = 0) -> int:
        """Device bytes the library holds for one call ("apply", "filter", "chol_gs",
        "rayleigh_ritz", "density") on n_vec columns."""
        ops = {"apply": 0, "filter": 1, "chol_gs": 2, "rayleigh_ritz": 3, "density": 4}
        return int(self.lib.chfsi_workspace_bytes(self.ctx, int(ik), int(n_vec), ops[op]))

    def rayleigh_ritz(self, X, work, ik: int = 0, resid: bool = True):
        px, ldx, n = _block(X, "X")
        pw, ldw, nw = _block(work, "work")
        theta = np.zeros(n)
        r = np.zeros(n) if resid else None
        self._chk(self.lib.chfsi_rayleigh_ritz(
            self.ctx, ik, C.c_void_p(px), ldx, C.c_void_p(pw), ldw, n,
            theta.ctypes.data_as(C.POINTER(C.c_double)),
            r.ctypes.data_as(C.POINTER(C.c_double)) if resid else None))
        return theta, r

    def lanczos_bounds(self, v0, steps: int = 40, ik: int = 0):
        pv, _, _ = _block(v0, "v0")
        lo, hi = C.c_double(), C.c_double()
        self._chk(self.lib.chfsi_lanczos_bounds(self.ctx, ik, int(steps), C.c_void_p(pv),
                                                C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def fill_random(self, X, seed: int, row0: int = 0, col0: int = 0, n_total_cols=None):
        px, ld, n = _block(X, "X")
        ntc = n if n_total_cols is None else int(n_total_cols)
        self._chk(self.lib.chfsi_fill_random(self.ctx, C.c_void_p(px), X.shape[0], n, ld,
                                             C.c_uint64(seed), row0, col0, ntc))
        return X

    # ---------------------------------------------------------------- adjoint
    def _fields_grad(self, dV, dB):
        torch = _torch()
        for t, shp in ((dV, (self.n_cells, self.nq3)), (dB, (self.n_cells, self.nq3, 3))):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
                raise ValueError(f"gradient buffers must be contiguous float64 CUDA tensors {shp}")

    def apply_H_backward(self, X, Ybar, Xbar, dV, dB, ik: int = 0):
        """Xbar = H_hat Ybar; dV, dB += dL/dV, dL/dB (Ybar = 2 dL/d conj(Y))."""
        px, ldx, n = _block(X, "X")
        pg, ldg, ng = _block(Ybar, "Ybar")
        pb, ldb, nb = _block(Xbar, "Xbar")
        if not (n == ng == nb):
            raise ValueError("X, Ybar, Xbar must have the same width")
        self._fields_grad(dV, dB)
        self._chk(self.lib.chfsi_apply_H_backward(self.ctx, ik, C.c_void_p(px), ldx, C.c_void_p(pg), ldg,
                                                  C.c_void_p(pb), ldb, n, C.c_void_p(dV.data_ptr()),
                                                  C.c_void_p(dB.data_ptr())))
        return Xbar

    def filter_backward_workspace(self, n_vec: int, degree: int, ckpt_every: int) -> int:
        return int(self.lib.chfsi_filter_backward_workspace(self.ctx, n_vec, degree, ckpt_every))

    def cheb_filter_backward(self, X, Ybar, Xbar, dV, dB, degree, a, b, a0, ckpt_every: int = 4,
                             ik: int = 0, work=None):
        torch = _torch()
        px, ldx, n = _block(X, "X")
        pg, ldg, ng = _block(Ybar, "Ybar")
        pb, ldb, nb = _block(Xbar, "Xbar")
        if not (n == ng == nb):
            raise ValueError("X, Ybar, Xbar must have the same width")
        self._fields_grad(dV, dB)
        need = self.filter_backward_workspace(n, degree, ckpt_every)
        if work is None or work.numel() * work.element_size() < need:
            work = torch.empty(need // 16 + 1, dtype=torch.complex128, device=X.device)
        self._chk(self.lib.chfsi_cheb_filter_backward(
            self.ctx, ik, C.c_void_p(px), ldx, C.c_void_p(pg), ldg, C.c_void_p(pb), ldb, n, int(degree),
            float(a), float(b), float(a0), int(ckpt_every), C.c_void_p(work.data_ptr()),
            work.numel() * work.element_size(), C.c_void_p(dV.data_ptr()), C.c_void_p(dB.data_ptr())))
        return Xbar

    # ---------------------------------------------------------------- densities
    def density(self, X, occ, rho, mag):
        """rho += sum_n occ[n] u_n^H u_n, mag += sum_n occ[n] u_n^H sigma u_n at every
        quadrature point; rho [E, nq^3], mag [E, nq^3, 3] float64 CUDA tensors."""
        px, ldx, n = _block(X, "X")
        f = np.ascontiguousarray(np.asarray(occ, dtype=np.float64).reshape(-1))
        if f.shape[0] != n:
            raise ValueError("occ must hold one value per column of X")
        self._fields_grad(rho, mag)
        self._chk(self.lib.chfsi_density(self.ctx, C.c_void_p(px), ldx, n,
                                         f.ctypes.data_as(C.POINTER(C.c_double)),
                                         C.c_void_p(rho.data_ptr()), C.c_void_p(mag.data_ptr())))
        return rho, mag

    # ---------------------------------------------------------------- SCF fields
    def _qfield(self, t, name, vec=False):
        torch = _torch()
        shp = (self.n_cells, self.nq3, 3) if vec else (self.n_cells, self.nq3)
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or \
                not t.is_contiguous() or tuple(t.shape) != shp:
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {shp}")
        return C.c_void_p(t.data_ptr())

    def field_inner(self, r1, m1, r2, m2) -> float:
        """(1/2)(int r1 r2 + int m1 . m2) with the cell quadrature (m1 = m2 = None: charge part)."""
        out = C.c_double()
        pm1 = None if m1 is None else self._qfield(m1, "m1", True)
        pm2 = None if m2 is None else self._qfield(m2, "m2", True)
        self._chk(self.lib.chfsi_field_inner(self.ctx, self._qfield(r1, "r1"), pm1, self._qfield(r2, "r2"), pm2,
                                             C.byref(out)))
        return out.value

    def hartree(self, rho, vh, tol: float = 1e-13, max_iter: int = 20000) -> int:
        it = C.c_int()
        self._chk(self.lib.chfsi_hartree(self.ctx, self._qfield(rho, "rho"), self._qfield(vh, "vh"), float(tol),
                                         int(max_iter), C.byref(it)))
        return it.value

    def kerker(self, f, out, k0: float, tol: float = 1e-13, max_iter: int = 20000) -> int:
        it = C.c_int()
        self._chk(self.lib.chfsi_kerker(self.ctx, float(k0), self._qfield(f, "f"), self._qfield(out, "out"),
                                        float(tol), int(max_iter), C.byref(it)))
        return it.value

    def exchange(self, rho, m, vx, bx):
        self._chk(self.lib.chfsi_exchange(self.ctx, self._qfield(rho, "rho"), self._qfield(m, "m", True),
                                          self._qfield(vx, "vx"), self._qfield(bx, "bx", True)))
        return vx, bx

    def stats_enable(self, on: bool = True):
        self._chk(self.lib.chfsi_stats_enable(self.ctx, 1 if on else 0))

    def stats_reset(self):
        self._chk(self.lib.chfsi_stats_reset(self.ctx))

    def stats(self) -> dict:
        """Per-stage totals since the last reset: launches, ms, flops, exec_flops, bytes."""
        arr = (_lib.StageStats * len(_lib.STAGES))()
        self._chk(self.lib.chfsi_stats_read(self.ctx, arr))
        return {name: {f: getattr(arr[i], f) for f, _ in _lib.StageStats._fields_}
                for i, name in enumerate(_lib.STAGES)}

    def sync(self):
        self._chk(self.lib.chfsi_sync(self.ctx))


def interpolate_block(coarse: "Operator", fine: "Operator", Yc, Yf):
    """Move the degree-(p-1) block Yc of `coarse` to the degree-p nodes of `fine` (into Yf)."""
    pc, ldc, n = _block(Yc, "Yc")
    pf, ldf, nf = _block(Yf, "Yf")
    if nf != n or Yc.shape[0] != coarse.n_dof or Yf.shape[0] != fine.n_dof:
        raise ValueError("Yc must be [2M_c][n], Yf [2M_f][n]")
    _lib.check(fine.lib.chfsi_interpolate_block(coarse.ctx, fine.ctx, C.c_void_p(pc), ldc, C.c_void_p(pf), ldf, n),
               fine.ctx)
    return Yf


SCF_DEFAULTS = dict(passes_first=4, passes=1, depth=4, max_iter=40, max_coarse=20, lanczos_steps=40,
                    field_max_iter=20000, prec="fp64", alpha=0.5, k0=0.0, tol=1e-8, tol_coarse=1e-3,
                    field_tol=1e-13, seed=0, lanczos_seed=1, bounds=None, kweights=None, start_given=False)


def scf_run(fine: "Operator", vext, bext, rho, m, rho_out, m_out, X, n_electrons: float, kT: float,
            degree: int, coarse: Optional["Operator"] = None, max_hist: int = 1000, **kw):
    """The SCF loop of chfsi_scf_run.  rho, m (in: initial input densities; out: last
    input), rho_out, m_out (out) and X (out: the Ritz blocks; [2M][n_vec], or
    [n_k][2M][n_vec] for an operator with n_k k-points) are CUDA tensors; bounds
    (optional) the filter's upper bound per iteration and k-point (iteration-major),
    kweights the k-point weights (default equal); start_given: X holds the start
    blocks (a restart) instead of the seeded ones.  Returns (history records as dicts,
    theta, occupations, converged); theta and the occupations are [n_k][n_vec] with
    several k-points, [n_vec] with one."""
    o = dict(SCF_DEFAULTS)
    unknown = set(kw) - set(o)
    if unknown:
        raise TypeError(f"unknown SCF parameters {sorted(unknown)}")
    o.update(kw)
    nk = fine.n_k
    torch = _torch()
    if nk > 1:
        if not isinstance(X, torch.Tensor) or X.dim() != 3 or X.shape[0] != nk or not X.is_contiguous():
            raise ValueError("X must be a contiguous [n_k][2M][n_vec] tensor for several k-points")
        px, ldx, n = _block(X[0], "X")
    else:
        px, ldx, n = _block(X, "X")
    prm = _lib.ScfParams()
    prm.n_vec, prm.degree = n, int(degree)
    for f in ("passes_first", "passes", "depth", "max_iter", "max_coarse", "lanczos_steps", "field_max_iter"):
        setattr(prm, f, int(o[f]))
    prm.prec_mode = _PREC[o["prec"]]
    prm.n_electrons, prm.kT = float(n_electrons), float(kT)
    for f in ("alpha", "k0", "tol", "tol_coarse", "field_tol"):
        setattr(prm, f, float(o[f]))
    prm.seed, prm.lanczos_seed = int(o["seed"]), int(o["lanczos_seed"])
    prm.start_given = 1 if o["start_given"] else 0
    bnd = wk = None
    if o["bounds"] is not None:
        bnd = np.ascontiguousarray(np.asarray(o["bounds"], dtype=np.float64).reshape(-1))
        prm.bounds_h = bnd.ctypes.data_as(C.POINTER(C.c_double))
        prm.n_bounds = bnd.shape[0]
    if o["kweights"] is not None:
        wk = np.ascontiguousarray(np.asarray(o["kweights"], dtype=np.float64).reshape(-1))
        if wk.shape[0] != nk:
            raise ValueError("kweights needs one weight per k-point")
        prm.kweights_h = wk.ctypes.data_as(C.POINTER(C.c_double))
    th = np.zeros(nk * n)
    occ = np.zeros(nk * n)
    hist = (_lib.ScfRecord * max_hist)()
    nh, conv = C.c_int(), C.c_int()
    pd = C.POINTER(C.c_double)
    rc = fine.lib.chfsi_scf_run(fine.ctx, None if coarse is None else coarse.ctx, C.byref(prm),
                                fine._qfield(vext, "vext"), fine._qfield(bext, "bext", True),
                                fine._qfield(rho, "rho"), fine._qfield(m, "m", True),
                                fine._qfield(rho_out, "rho_out"), fine._qfield(m_out, "m_out", True),
                                C.c_void_p(px), ldx, th.ctypes.data_as(pd), occ.ctypes.data_as(pd), hist,
                                int(max_hist), C.byref(nh), C.byref(conv))
    _lib.check(rc, fine.ctx)
    recs = [{f: getattr(hist[i], f) for f, _ in _lib.ScfRecord._fields_} for i in range(min(nh.value, max_hist))]
    if nk > 1:
        th, occ = th.reshape(nk, n), occ.reshape(nk, n)
    return recs, th, occ, bool(conv.value)


BATCH_AUTOTUNE = 1
BATCH_GRAPH = 2


def fermi_dirac(eps, n_electrons: float, kT: float, weights=None):
    """(occupations, mu, E_ent) of the levels eps at temperature kT (Ha) holding
    n_electrons; weights are the levels' k-point weights (default 1)."""
    lib = _lib.load()
    e = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(-1))
    pd = C.POINTER(C.c_double)
    w = None
    if weights is not None:
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        if w.shape != e.shape:
            raise ValueError("weights must match eps")
    occ = np.empty_like(e)
    mu, ent = C.c_double(0.0), C.c_double(0.0)
    rc = lib.chfsi_fermi_dirac(e.shape[0], e.ctypes.data_as(pd), None if w is None else w.ctypes.data_as(pd),
                               float(n_electrons), float(kT), occ.ctypes.data_as(pd), C.byref(mu), C.byref(ent))
    _lib.check(rc)
    return occ, mu.value, ent.value


class Batch:
    """Batched filter of many (operator, k-point, block) tasks; see chfsi_batch_create.
    tasks: list of (Operator, ik, X, work) with X, work complex128 CUDA blocks."""

    def __init__(self, tasks, degree: int, prec="fp64", flags: int = BATCH_AUTOTUNE | BATCH_GRAPH):
        self.lib = _lib.load()
        self._keep = tasks
        arr = (_lib.BatchTask * len(tasks))()
        for i, (op, ik, X, W) in enumerate(tasks):
            px, ldx, n = _block(X, "X")
            pw, ldw, nw = _block(W, "work")
            if nw < n:
                raise ValueError("work narrower than X")
            arr[i].ctx = op.ctx
            arr[i].ik = int(ik)
            arr[i].X_d = px
            arr[i].ldx = ldx
            arr[i].work_d = pw
            arr[i].ldw = ldw
            arr[i].n_vec = n
        h = C.c_void_p()
        rc = self.lib.chfsi_batch_create(len(tasks), arr, int(degree), _PREC[prec], int(flags), C.byref(h))
        if rc != 0:
            raise _lib.ChfsiError(rc, "chfsi_batch_create failed (check contexts, buffers, stream)")
        self.h = h
        self.n = len(tasks)

    def filter(self, a, b, a0):
        arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (self.n,))) for v in (a, b, a0)]
        ptrs = [x.ctypes.data_as(C.POINTER(C.c_double)) for x in arrs]
        rc = self.lib.chfsi_batch_filter(self.h, *ptrs)
        if rc != 0:
            raise _lib.ChfsiError(rc, self.lib.chfsi_batch_last_error(self.h).decode())

    def tiles(self):
        cols = (C.c_int * self.n)()
        ms = np.zeros(3 * self.n)
        self.lib.chfsi_batch_tiles(self.h, cols, ms.ctypes.data_as(C.POINTER(C.c_double)))
        return list(cols), ms.reshape(self.n, 3)

    def graph_info(self) -> dict:
        """Captures, replays and host milliseconds of capture and instantiation."""
        nc, nr = C.c_int(), C.c_int()
        cms, ims = C.c_double(), C.c_double()
        rc = self.lib.chfsi_batch_graph_info(self.h, C.byref(nc), C.byref(nr), C.byref(cms), C.byref(ims))
        if rc != 0:
            raise _lib.ChfsiError(rc, "chfsi_batch_graph_info failed")
        return {"captures": nc.value, "replays": nr.value, "capture_ms": cms.value, "instantiate_ms": ims.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.chfsi_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
