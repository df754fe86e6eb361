#!/usr/bin/env python
"""ChFSI benchmark on one MI355X.

One step = one ChFSI pass over the whole block: the degree-m Chebyshev filter
of every 128-vector block, Cholesky-Gram-Schmidt and Rayleigh-Ritz (with
residual norms), all through the C ABI.  The default workload is the
large periodic system: 20^3 cells, p = 6 (3.456 M spinor dofs), 200-Gaussian
V_eff, noncollinear B_xc, 64 pseudo-atoms with l <= 2 spin-orbit projectors,
N = 512 vectors filtered in 4 blocks of 128, Chebyshev degree 24, Gamma point.

Printed JSON (one line, rank 0):
  value        FP64 filter throughput, TFLOP/s, algorithmic count (a complex
               multiply-add = 8 flops) over the filter sections of the timed passes
  ms_per_step  wall time per FP64 pass (filter + CholGS + RR), the K timed passes
  roofline     the FP64 cell-product kernel (dominant): algorithmic flops per
               launch / mean launch time from HIP events, against 78.6 TFLOP/s
  mixed        from the same FP64 prologue and warm-up, the timed passes with FP32
               cell/projector products in applies 1..m-1: per-pass time, speedup and
               the largest Ritz-value difference from the FP64 run
  mixed_resid  the same with the residual form of the filter (every correction
               product in FP32)
  cpu_baseline the FP64 oracle on a bounded sample (see `sample`)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6     # TFLOP/s, MI355X dense FP64 (vector = matrix)
PEAK_FP32 = 157.3    # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0    # GB/s, MI355X HBM3E
K_B_HA = 3.166811563e-6   # Boltzmann constant, Ha / K
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "cell_apply_fp64_scale_traffic.md")


MF_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "mf_apply_density_scale_traffic.md")
CELL_SOURCES = ("cell.hip", "mfma.h")
MF_SOURCES = ("matfree.hip", "sumfact.h", "mfma.h")


def kernel_fingerprint(sources=CELL_SOURCES):
    """sha256 over a kernel's sources and the device compile flags: a counter
    record taken for another build of the kernel does not apply."""
    import hashlib
    from paper_2410_02754_amd import build as b
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2410_02754_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(b.COMMON).encode())
    return h.hexdigest()


def cell_kernel_fingerprint():
    return kernel_fingerprint(CELL_SOURCES)


def measured_traffic(grid_wg, record=TRAFFIC_RECORD, sources=CELL_SOURCES):
    """HBM bytes per launch of a kernel from its committed counter record
    (calibrated FETCH_SIZE + WRITE_SIZE), or None when the record is missing, was
    taken on another launch shape or for other kernel sources."""
    try:
        with open(record) as fh:
            line = next(l for l in fh if l.startswith("traffic_record: "))
        rec = json.loads(line[len("traffic_record: "):])
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("source_sha256") != kernel_fingerprint(sources) or rec.get("grid_wg") != grid_wg:
        return None
    return float(rec["hbm_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_operator(s, torch, stream=None, form="cell"):
    import synth
    from paper_2410_02754_amd import Operator
    op = Operator(s.n_cells, s.box, s.p, s.quad, s.n_q, s.kpts,
                  stream=None if stream is None else stream.cuda_stream, form=form)
    t = time.perf_counter()
    pts = op.quad_points().reshape(-1, 3)
    V = torch.tensor(synth.veff(s, pts).reshape(op.n_cells, op.nq3), device="cuda")
    B = torch.tensor(synth.bxc(s, pts).reshape(op.n_cells, op.nq3, 3), device="cuda")
    log(f"[bench] fields at {pts.shape[0]} quadrature points: {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    op.set_local(V, B)
    del V, B
    log(f"[bench] cell operators: {time.perf_counter() - t:.1f} s")
    t = time.perf_counter()
    op.set_atoms(s.atoms)
    log(f"[bench] projectors ({len(s.atoms)} atoms): {time.perf_counter() - t:.1f} s")
    return op


def run_passes(op, s, X, W, Wf, b, theta, n_pass, prec, torch, label, resid_form=False):
    """n_pass passes; returns (theta, resid, per-pass seconds, filter seconds, filter stats).
    resid_form: filter through Hamiltonian-times-residual products (Wf is [2M][2*block]);
    W must then hold H X of the previous Rayleigh-Ritz."""
    times, ftimes = [], []
    fstats = {"flops": 0.0, "cell_flops": 0.0, "cell_exec": 0.0, "cell_ms": 0.0, "cell_launches": 0,
              "stage_ms": {}}
    cell_key = "cell_fp64" if prec == "fp64" else "cell_fp32"
    r = None
    for p in range(n_pass):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a, a0 = float(theta[-1]), float(theta[0])
        op.stats_reset()
        if resid_form:
            op.ritz_residual(X, W, theta)
        for c0 in range(0, s.n_vec, s.block):
            if resid_form:
                op.cheb_filter_resid(X[:, c0:c0 + s.block], W[:, c0:c0 + s.block], theta[c0:c0 + s.block], Wf,
                                     s.degree, a, b, a0, prec=prec)
            else:
                op.cheb_filter(X[:, c0:c0 + s.block], Wf[:, :s.block], s.degree, a, b, a0, prec=prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = op.stats()
        fstats["flops"] += sum(st[k]["flops"] for k in ("cell_fp64", "cell_fp32", "nonlocal"))
        # the dominant kernel: every cell launch of this precision (apply m is FP64 in mixed mode)
        fstats["cell_flops"] += st[cell_key]["flops"]
        fstats["cell_exec"] += st[cell_key]["exec_flops"]
        fstats["cell_ms"] += st[cell_key]["ms"]
        fstats["cell_launches"] += st[cell_key]["launches"]
        for k, v in st.items():
            fstats["stage_ms"]["filter_" + k] = fstats["stage_ms"].get("filter_" + k, 0.0) + v["ms"]
        op.stats_reset()
        op.chol_gs(X)
        theta, r = op.rayleigh_ritz(X, W)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for k, v in op.stats().items():
            fstats["stage_ms"]["rr_" + k] = fstats["stage_ms"].get("rr_" + k, 0.0) + v["ms"]
        times.append(t2 - t0)
        ftimes.append(t1 - t0)
        log(f"[bench] {label} pass {p + 1}/{n_pass}: {t2 - t0:.2f} s (filter {t1 - t0:.2f} s), "
            f"theta[0]={theta[0]:.10f} max resid {np.max(r):.2e}")
    return theta, r, times, ftimes, fstats


def start(op, s, X, W, torch):
    op.fill_random(X, s.seed, n_total_cols=s.n_vec)
    op.chol_gs(X)
    return op.rayleigh_ritz(X, W)


def cpu_baseline(s_name):
    """The oracle, as it is, on a bounded sample of the workload: one H_hat
    application to 64 vectors on a 3 x 3 x 3-cell periodic piece of the same
    mesh (same h and p), with one pseudo-atom of the same kind."""
    import synth
    from oracle import hamiltonian as ham
    big = synth.config(s_name)
    h = big.box[0] / big.n_cells[0]
    a0 = big.atoms[0]
    s = synth.make_system("sample", n_cells=(3, 3, 3), box=(3 * h, 3 * h, 3 * h), p=big.p,
                          n_gauss=2, n_atoms=1, lmax=a0.lmax, sigma=a0.sigma,
                          rcut_sigmas=a0.rcut / a0.sigma, n_vec=big.block, seed=5)
    t = time.perf_counter()
    _, H, _, _, _ = ham.build(s, synth.veff, synth.bxc)
    t_build = time.perf_counter() - t
    X = synth.start_block(s, s.n_dof)
    reps = 0
    t = time.perf_counter()
    while True:          # repeat the apply for about 10 s of CPU work
        Y = H @ X
        reps += 1
        if time.perf_counter() - t > 10.0 or reps >= 50:
            break
    t_apply = (time.perf_counter() - t) / reps
    n2 = 2 * (s.p + 1) ** 3
    flops = s.n_cell_total * 8.0 * n2 * n2 * s.n_vec
    for Ps, D in H.projs:
        nsup = int(np.count_nonzero(Ps.getnnz(axis=1))) // 2
        npj = D.shape[0] // 2
        flops += 2 * 8.0 * nsup * npj * 2 * s.n_vec + 8.0 * (2 * npj) ** 2 * s.n_vec
    del Y
    return {"value": flops / t_apply / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": (f"{reps} H_hat applies to {s.n_vec} vectors on a 3x3x3-cell periodic piece of the "
                       f"{s_name} mesh (p={s.p}, h={h:.2f} bohr, {s.n_dof} dofs, 1 atom l<={a0.lmax}); "
                       f"scipy CSR x dense is single-threaded; {t_apply:.2f} s per apply, "
                       f"{t_build:.1f} s assembly (untimed)"),
            "apply_s": t_apply}


def cell_alg_bytes(s):
    """Algorithmic HBM bytes of one filter launch (one colour, 128 columns):
    the Gamma-point Pauli-form operator (4 real (p+1)^3 x (p+1)^3 FP64 matrices
    per cell) read once, the cell's gathered input rows read once and its output
    rows read and written once."""
    n_colour_cells = int(np.prod(s.n_cells)) // 8
    nloc = (s.p + 1) ** 3
    return n_colour_cells * (4.0 * nloc * nloc * 8 + 3.0 * 2 * nloc * s.block * 16)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=os.environ.get("CHFSI_BENCH_WORKLOAD", "scale"),
                    help="scale (default), batch (k-grid + uneven systems) or adjoint")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-matfree", action="store_true")
    ap.add_argument("--eig-table", default=None,
                    help="write the per-eigenvalue FP64 / mixed table (text) to this path")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(k-points and systems would go one per GPU; a large system would be split into "
              "subdomains of cells with halo scatter-adds).", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload == "batch":
        out = bench_batch(args, torch)
    elif args.workload == "adjoint":
        out = bench_adjoint(args, torch)
    else:
        out = bench_scale(args, torch)
    print(json.dumps(out), flush=True)


def bench_density(op, s, X, theta, torch, reps=3):
    """Densities of the FP64 Ritz block (eqn:rho, eqn:mag) with Fermi-Dirac
    occupations at 500 K (Sec. V), the block holding 15% more states than
    electrons; HIP-event time of chfsi_density (quadrature-point kernel and the
    fixed-order group reduction) over the whole block."""
    from paper_2410_02754_amd import fermi_dirac
    n_e = float(round(0.85 * s.n_vec))
    kT = 500.0 * K_B_HA
    t = time.perf_counter()
    f, mu, ent = fermi_dirac(theta, n_e, kT)
    t_fd = time.perf_counter() - t
    rho = torch.zeros((op.n_cells, op.nq3), dtype=torch.float64, device="cuda")
    mag = torch.zeros((op.n_cells, op.nq3, 3), dtype=torch.float64, device="cuda")
    op.density(X, f, rho, mag)                    # first call sizes the partial-sum buffer
    ts = []
    for _ in range(reps):
        rho.zero_()
        mag.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        op.density(X, f, rho, mag)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = sum(ts) / len(ts)
    n_points = op.n_cells * op.nq3
    alg_bytes = s.n_dof * s.n_vec * 16 + n_points * 4 * 8          # block read once, rho and m written
    nq, np1 = s.n_q, s.p + 1
    # sum factorisation per column, cell and spin: three 1-D passes of complex x real MACs
    flops = 8.0 * (nq * np1 ** 3 + nq * nq * np1 ** 2 + nq ** 3 * np1) * op.n_cells * s.n_vec
    mnorm = torch.linalg.norm(mag, dim=-1)
    res = {"ms": round(ms, 3), "n_electrons": n_e, "kT_Ha": kT, "mu_Ha": mu, "E_ent_Ha": ent,
           "fermi_dirac_host_ms": round(1e3 * t_fd, 3),
           "algorithmic_bytes": alg_bytes, "achieved_GBs": round(alg_bytes / (ms * 1e-3) / 1e9, 1),
           "frac_of_hbm_8000GBs": round(alg_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM, 4),
           "interp_flops": flops, "achieved_fp64_tflops": round(flops / (ms * 1e-3) / 1e12, 3),
           "max_rho": float(rho.max()), "max_abs_m_over_rho": float((mnorm / rho.clamp_min(1e-300)).max())}
    log(f"[bench] densities: {ms:.2f} ms, mu {mu:.6f} Ha, E_ent {ent:.3e} Ha")
    del rho, mag
    return res


def fastest_pass(out, bar=1e-7):
    """The fastest of the measured pass forms whose Ritz values stay within bar
    (Ha) of the FP64 cell-matrix run (that run itself included)."""
    cands = [("cell matrices, FP64", out["s_per_pass"], 0.0)]
    for key, name in (("mixed", "cell matrices, FP32 applies 1..m-1"),
                      ("mixed_resid", "cell matrices, FP32 residual form")):
        if key in out:
            cands.append((name, out[key]["s_per_pass"], out[key]["max_dtheta_vs_fp64_Ha"]))
    mf = out.get("matrix_free")
    if mf:
        cands.append(("matrix-free, FP64", mf["s_per_pass"], mf["max_dtheta_vs_cell_fp64_Ha"]))
        for key, name in (("mixed", "matrix-free, FP32 applies 1..m-1"),
                          ("mixed_resid", "matrix-free, FP32 residual form")):
            if key in mf:
                cands.append((name, mf[key]["s_per_pass"], mf[key]["max_dtheta_vs_cell_fp64_Ha"]))
    ok = [c for c in cands if c[2] <= bar]
    name, sp, dth = min(ok, key=lambda c: c[1])
    return {"form": name, "s_per_pass": sp, "max_dtheta_vs_fp64_Ha": dth,
            "speedup_vs_cell_fp64": round(out["s_per_pass"] / sp, 3)}


def bench_matfree(args, s, X, W, Wf, b, theta_ref, torch, tables=None):
    """The same FP64 passes (same start block, bound and steps) with the
    matrix-free local operator instead of the stored cell matrices."""
    t = time.perf_counter()
    op = build_operator(s, torch, form="matrix_free")
    t_setup = time.perf_counter() - t
    op.stats_enable(True)
    theta, _ = start(op, s, X, W, torch)
    theta, _, _, _, _ = run_passes(op, s, X, W, Wf, b, theta, args.warmup, "fp64", torch, "matrix-free warmup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th, r, times, ftimes, fst = run_passes(op, s, X, W, Wf, b, theta, args.steps, "fp64", torch, "matrix-free")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    mixed = {}
    if not args.no_mixed:
        # the FP32 filters on the same state as the FP64 passes: plain (applies
        # 1..m-1 in FP32) and residual form (every correction product in FP32)
        for key, resid_form, form in (("mixed", False, "applies 1..m-1 with the FP32 matrix-free and projector "
                                                        "products, apply m FP64"),
                                      ("mixed_resid", True, "residual form, FP32 matrix-free and projector "
                                                            "products on the correction")):
            theta, _ = start(op, s, X, W, torch)
            theta, _, _, _, _ = run_passes(op, s, X, W, Wf, b, theta, args.warmup, "fp64", torch,
                                           f"matrix-free {key} fp64 warmup")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            thm, rm, _, mft, mst = run_passes(op, s, X, W, Wf, b, theta, args.steps, "mixed", torch,
                                              f"matrix-free {key}", resid_form)
            torch.cuda.synchronize()
            mtotal = time.perf_counter() - t1
            dthm = np.abs(thm - theta_ref)
            if tables is not None:
                tables[f"matrix_free {key}"] = (thm, dthm)
            mixed[key] = {"form": form,
                          "s_per_pass": round(mtotal / args.steps, 3),
                          "filter_s_per_pass": round(sum(mft) / args.steps, 3),
                          "speedup_pass_vs_matrix_free_fp64": round(total / mtotal, 3),
                          "max_dtheta_vs_cell_fp64_Ha": float(dthm.max()),
                          "within_1e-7_Ha": bool(dthm.max() <= 1e-7),
                          "fp32_launch_ms": round(mst["cell_ms"] / max(1, mst["cell_launches"]), 4),
                          "stage_ms_per_pass": {k: round(v / args.steps, 1) for k, v in mst["stage_ms"].items()
                                                if v > 0}}
            log(f"[bench] matrix-free {key}: {mixed[key]['s_per_pass']} s per pass, max |dtheta| "
                f"{dthm.max():.2e} Ha")
    op.close()
    n_l = max(1, fst["cell_launches"])
    ms = fst["cell_ms"] / n_l
    exec_per = fst["cell_exec"] / n_l
    dth = np.abs(th - theta_ref)
    # roofline of the local operator: algorithmic bytes (rows gathered, output rows read
    # and written, once per launch) over the mean filter launch
    n_colour_cells = int(np.prod(s.n_cells)) // 8
    alg = float(n_colour_cells * 2 * (s.p + 1) ** 3 * s.block * 16 * 3)
    grid_wg = n_colour_cells * ((s.block + 1) // 2)
    ach = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM, 4), "algorithmic_bytes_per_launch": alg,
            "traffic": measured_traffic(grid_wg, MF_TRAFFIC_RECORD, MF_SOURCES),
            "traffic_unit": "HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)"}
    res = {"form": "matrix-free sum factorisation, FP64 (n_q = p + 1 collocation)",
           "roofline": roof,
           "s_per_pass": round(total / args.steps, 3),
           "filter_s_per_pass": round(sum(ftimes) / args.steps, 3),
           "filter_tflops_cell_count": round(fst["flops"] / sum(ftimes) / 1e12, 4),
           "setup_s": round(t_setup, 2),
           "kernel": "mf_apply_kernel<7, false> (gather, 12 line contractions per spin, scatter-add)",
           "mean_launch_ms": round(ms, 4),
           # 12 dense 1-D contractions per spin (96 n_p^4 per cell and column); the even-odd
           # form issues about half of these multiply-adds
           "sumfact_flops_per_launch": exec_per,
           "sumfact_fp64_tflops": round(exec_per / (ms * 1e-3) / 1e12, 3) if ms > 0 else None,
           "sumfact_frac_of_78.6": round(exec_per / (ms * 1e-3) / 1e12 / PEAK_FP64, 4) if ms > 0 else None,
           "cell_form_flops_per_launch": fst["cell_flops"] / n_l,
           "max_dtheta_vs_cell_fp64_Ha": float(dth.max()), "max_resid": float(np.max(r)),
           "stage_ms_per_pass": {k: round(v / args.steps, 1) for k, v in fst["stage_ms"].items() if v > 0}}
    res.update(mixed)
    log(f"[bench] matrix-free: {res['s_per_pass']} s per pass, max |dtheta| vs cell {dth.max():.2e} Ha")
    return res


def bench_scale(args, torch):
    import synth
    s = synth.config(args.workload)
    log(f"[bench] workload {s.name}: {s.n_cells} cells p={s.p} 2M={s.n_dof} N={s.n_vec} "
        f"block={s.block} m={s.degree} atoms={len(s.atoms)}")
    t = time.perf_counter()
    op = build_operator(s, torch)
    op.stats_enable(True)
    t_setup = time.perf_counter() - t
    X = torch.empty((s.n_dof, s.n_vec), dtype=torch.complex128, device="cuda")
    W = torch.empty_like(X)
    Wf = torch.empty((s.n_dof, 2 * s.block), dtype=torch.complex128, device="cuda")
    v0 = torch.empty((s.n_dof, 1), dtype=torch.complex128, device="cuda")
    op.fill_random(v0, s.seed + 1)
    t = time.perf_counter()
    lo, b = op.lanczos_bounds(v0[:, 0], 40)
    t_lanczos = time.perf_counter() - t
    del v0
    log(f"[bench] Lanczos bounds ({t_lanczos:.2f} s): [{lo:.6f}, {b:.6f}]")

    # FP64 passes
    theta, _ = start(op, s, X, W, torch)
    theta, _, _, _, _ = run_passes(op, s, X, W, Wf, b, theta, args.warmup, "fp64", torch, "fp64 warmup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta64, r64, times, ftimes, fst = run_passes(op, s, X, W, Wf, b, theta, args.steps, "fp64", torch,
                                                  "fp64")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    filt_tflops = fst["flops"] / sum(ftimes) / 1e12
    cell_per_launch = fst["cell_flops"] / max(1, fst["cell_launches"])
    cell_ms = fst["cell_ms"] / max(1, fst["cell_launches"])
    achieved = cell_per_launch / (cell_ms * 1e-3) / 1e12 if cell_ms > 0 else 0.0
    exec_tf = fst["cell_exec"] / (fst["cell_ms"] * 1e-3) / 1e12 if fst["cell_ms"] > 0 else 0.0
    # filter launches: one colour of cells x row tiles x column tiles of 64
    n_colour_cells = int(np.prod(s.n_cells)) // 8
    nloc = (s.p + 1) ** 3
    grid_wg = n_colour_cells * (((nloc + 15) // 16 + 1) // 2) * ((s.block + 63) // 64)
    traffic = measured_traffic(grid_wg)

    out = {
        "metric": "ChFSI filter TFLOP/s + s per ChFSI pass; FP32 vs FP64 filter at 1e-7 Ha eigs",
        "value": round(filt_tflops, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * total / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{s.name}: periodic {s.n_cells[0]}x{s.n_cells[1]}x{s.n_cells[2]} cells, "
                               f"p={s.p}, {s.n_dof} spinor dofs, {len(s.atoms)} SOC atoms, "
                               f"N={s.n_vec} in blocks of {s.block}, degree {s.degree}, Gamma",
                   "n_dof": s.n_dof, "n_vec": s.n_vec, "block": s.block, "degree": s.degree,
                   "parallelism": "single GPU"},
        "s_per_pass": round(total / args.steps, 3),
        "filter_s_per_pass": round(sum(ftimes) / args.steps, 3),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64, 4),
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                     "algorithmic_bytes_per_launch": cell_alg_bytes(s),
                     "kernel": "cell_apply_kernel<double, 2, false> (gather + Pauli-form cell products + scatter-add, 64-column tiles)",
                     "flops_per_launch": cell_per_launch, "mean_launch_ms": round(cell_ms, 4),
                     "executed_mfma_tflops": round(exec_tf, 3),
                     "executed_frac": round(exec_tf / PEAK_FP64, 4)},
        "stage_ms_per_pass": {k: round(v / args.steps, 1) for k, v in fst["stage_ms"].items() if v > 0},
        "setup_s": round(t_setup, 2), "lanczos_s": round(t_lanczos, 3),
        "theta_min": float(theta64[0]), "theta_max": float(theta64[-1]), "max_resid": float(np.max(r64)),
    }

    out["density"] = bench_density(op, s, X, theta64, torch)

    tables = {}
    if not args.no_mixed:
        for key, resid_form in (("mixed", False), ("mixed_resid", True)):
            # the same FP64 prologue and warm-up passes as the FP64 run (bitwise the
            # same state: every kernel is deterministic); only the timed passes differ
            theta, _ = start(op, s, X, W, torch)
            theta, _, _, _, _ = run_passes(op, s, X, W, Wf, b, theta, args.warmup, "fp64", torch,
                                           key + " fp64 warmup")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            thetam, rm, mt, mft, mst = run_passes(op, s, X, W, Wf, b, theta, args.steps, "mixed", torch, key,
                                                  resid_form)
            torch.cuda.synchronize()
            mtotal = time.perf_counter() - t0
            dth = np.abs(thetam - theta64)
            tables[key] = (thetam, dth)
            m_ach = (mst["cell_flops"] / max(1, mst["cell_launches"])) / \
                ((mst["cell_ms"] / max(1, mst["cell_launches"])) * 1e-3) / 1e12 if mst["cell_ms"] > 0 else 0.0
            conv = r64 < 1e-1
            out[key] = {
                "form": ("FP32 cell/projector products in applies 1..m-1, FP64 apply m" if not resid_form else
                         "residual form: every H x correction product in FP32, recurrence and "
                         "combination in FP64"),
                "filter_tflops": round(mst["flops"] / sum(mft) / 1e12, 4),
                "s_per_pass": round(mtotal / args.steps, 3),
                "filter_s_per_pass": round(sum(mft) / args.steps, 3),
                "speedup_pass": round(total / mtotal, 3),
                "speedup_filter": round(sum(ftimes) / sum(mft), 3),
                "max_dtheta_vs_fp64_Ha": float(dth.max()),
                "median_dtheta_vs_fp64_Ha": float(np.median(dth)),
                "max_dtheta_resid_below_0.1_Ha": float(dth[conv].max()) if np.any(conv) else None,
                "n_resid_below_0.1": int(np.count_nonzero(conv)),
                "within_1e-7_Ha": bool(dth.max() <= 1e-7),
                "cell_fp32_achieved_tflops": round(m_ach, 3),
                "cell_fp32_frac_of_157.3": round(m_ach / PEAK_FP32, 4),
                "stage_ms_per_pass": {k: round(v / args.steps, 1) for k, v in mst["stage_ms"].items() if v > 0},
            }
            log(f"[bench] {key}: max |dtheta| vs fp64 = {dth.max():.3e} Ha")
    op.close()
    if not args.no_matfree and s.n_q == s.p + 1:
        out["matrix_free"] = bench_matfree(args, s, X, W, Wf, b, theta64, torch, tables)
    out["fastest_pass_within_1e-7_Ha"] = fastest_pass(out)
    del X, W, Wf
    if args.eig_table and tables:
        with open(args.eig_table, "w") as fh:
            fh.write("# i  theta_fp64 (Ha)  resid_fp64  " +
                     "  ".join(f"|dtheta| {k} (Ha)" for k in tables) + "\n")
            for i in range(len(theta64)):
                fh.write(f"{i:4d} {theta64[i]: .12f} {r64[i]:.3e} " +
                         " ".join(f"{tables[k][1][i]:.3e}" for k in tables) + "\n")
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle on a bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline(s.name)
        out["cpu_baseline"].pop("apply_s", None)
    return out


def _task_flops(op, ik, X, W):
    """Algorithmic flops of one H_hat application to X (cell + nonlocal stages),
    read from the library's stage counters."""
    op.stats_enable(True)
    op.stats_reset()
    op.apply_H(X, W, ik=ik)
    st = op.stats()
    op.stats_enable(False)
    return st["cell_fp64"]["flops"] + st["nonlocal"]["flops"]


def bench_batch(args, torch):
    """The batched workload: the 8 k-points of a 2x2x2 Monkhorst-Pack grid on a
    12^3-cell p=5 mesh (N=384) and 5 Gamma systems of 6^3..14^3 cells (N=64..320),
    filtered (degree 16) in one persistent launch per colour phase replayed from a
    hipGraph, tiles from the autotuner; then per-task CholGS + RR.  Timed: the
    batched filter (FP64 and mixed) and, for reference, the same filters issued
    task by task through chfsi_cheb_filter."""
    import synth
    from paper_2410_02754_amd import Batch
    kg = synth.config("kgrid")
    systems = [kg] + [synth.config(f"uneven{i}") for i in range(1, 6)]
    stream = torch.cuda.Stream()            # graph capture needs a non-default stream
    out = {}
    with torch.cuda.stream(stream):
        t = time.perf_counter()
        ops = [build_operator(sy, torch, stream) for sy in systems]
        t_setup = time.perf_counter() - t
        tasks, meta = [], []
        for j, sy in enumerate(systems):
            for ik in range(len(sy.kpts)):
                X = torch.empty((sy.n_dof, sy.n_vec), dtype=torch.complex128, device="cuda")
                W = torch.empty_like(X)
                ops[j].fill_random(X, sy.seed + 100 * ik, n_total_cols=sy.n_vec)
                tasks.append((ops[j], ik, X, W))
                meta.append((sy, j, ik))
        # bounds per task: Lanczos upper bound, prologue CholGS + RR for a, a0
        a, b, a0, flops = [], [], [], 0.0
        t = time.perf_counter()
        for (op, ik, X, W), (sy, j, _) in zip(tasks, meta):
            v0 = torch.empty((sy.n_dof, 1), dtype=torch.complex128, device="cuda")
            op.fill_random(v0, sy.seed + 1)
            lo, hi = op.lanczos_bounds(v0[:, 0], 40, ik=ik)
            op.chol_gs(X)
            theta, _ = op.rayleigh_ritz(X, W, ik=ik)
            a.append(float(theta[-1]))
            a0.append(float(theta[0]))
            b.append(hi)
            flops += sy.degree * _task_flops(op, ik, X, W)
        t_prologue = time.perf_counter() - t
        X0 = [x.clone() for _, _, x, _ in tasks]
        degree = kg.degree
        log(f"[bench] batch: {len(tasks)} tasks, setup {t_setup:.1f} s, prologue {t_prologue:.1f} s, "
            f"{flops / 1e12:.2f} TFLOP per batched filter")

        def restore():
            for (_, _, X, _), x0 in zip(tasks, X0):
                X.copy_(x0)
            torch.cuda.synchronize()

        res = {}
        for prec in (("fp64",) if args.no_mixed else ("fp64", "mixed")):
            batch = Batch(tasks, degree, prec=prec)
            cols, tune = batch.tiles()
            for _ in range(max(1, args.warmup)):
                restore()
                batch.filter(a, b, a0)
            torch.cuda.synchronize()
            times = []
            for _ in range(args.steps):
                restore()
                t0 = time.perf_counter()
                batch.filter(a, b, a0)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            Yb = [x.clone() for _, _, x, _ in tasks]
            if prec == "fp64":
                Yb64 = Yb
            batch.close()
            # the same filters, task by task
            seq = []
            for _ in range(args.steps):
                restore()
                t0 = time.perf_counter()
                for (op, ik, X, W), aa, bb, cc in zip(tasks, a, b, a0):
                    op.cheb_filter(X, W, degree, aa, bb, cc, prec=prec, ik=ik)
                torch.cuda.synchronize()
                seq.append(time.perf_counter() - t0)
            same = all(bool(torch.equal(y, x)) for y, (_, _, x, _) in zip(Yb, tasks))
            tb, ts = float(np.median(times)), float(np.median(seq))
            res[prec] = {"ms_per_filter": round(1e3 * tb, 2), "tflops": round(flops / tb / 1e12, 3),
                         "sequential_ms": round(1e3 * ts, 2), "speedup_vs_sequential": round(ts / tb, 3),
                         "bitwise_equal_to_sequential": same,
                         "tiles_cols": cols, "autotune_ms_per_cell_stage": tune.round(4).tolist()}
            log(f"[bench] batch {prec}: {1e3 * tb:.1f} ms per batched filter ({flops / tb / 1e12:.2f} TFLOP/s), "
                f"task by task {1e3 * ts:.1f} ms, bitwise equal {same}")
        # one full pass per task after the batched FP64 filter: CholGS + RR
        restore()
        batch = Batch(tasks, degree, prec="fp64")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.filter(a, b, a0)
        for (op, ik, X, W) in tasks:
            op.chol_gs(X)
            op.rayleigh_ritz(X, W, ik=ik)
        torch.cuda.synchronize()
        t_pass = time.perf_counter() - t0
        batch.close()
        for op in ops:
            op.close()
        # the same tasks with the matrix-free operator (per-task colour launches
        # inside the captured filter), same start blocks and bounds
        mf = {}
        if not args.no_matfree:
            t = time.perf_counter()
            opm = [build_operator(sy, torch, stream, form="matrix_free") for sy in systems]
            t_setup_mf = time.perf_counter() - t
            tasks_mf = [(opm[j], ik, X, W) for (_, ik, X, W), (_, j, _) in zip(tasks, meta)]
            for prec in (("fp64",) if args.no_mixed else ("fp64", "mixed")):
                batch = Batch(tasks_mf, degree, prec=prec)
                for _ in range(max(1, args.warmup)):
                    restore()
                    batch.filter(a, b, a0)
                torch.cuda.synchronize()
                times = []
                for _ in range(args.steps):
                    restore()
                    t0 = time.perf_counter()
                    batch.filter(a, b, a0)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                batch.close()
                tb = float(np.median(times))
                mf[prec] = {"ms_per_filter": round(1e3 * tb, 2),
                            "speedup_vs_cell_form": round(res[prec]["ms_per_filter"] / (1e3 * tb), 3)}
                if prec == "fp64":
                    mf[prec]["max_rel_diff_vs_cell_form"] = max(
                        float((x - y).abs().max() / y.abs().max()) for (_, _, x, _), y in zip(tasks_mf, Yb64))
                log(f"[bench] batch matrix-free {prec}: {1e3 * tb:.1f} ms per batched filter")
            mf["setup_s"] = round(t_setup_mf, 1)
            for op in opm:
                op.close()
    f64 = res["fp64"]
    out = {
        "metric": "batched ChFSI filter TFLOP/s (8 k-points + 5 uneven Gamma systems, persistent hipGraph launch)",
        "value": f64["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": f64["ms_per_filter"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch: 2x2x2 MP k-grid on 12^3 cells p=5 (N=384) + Gamma systems "
                               "6^3/8^3/10^3/12^3/14^3 cells p=5 (N=64..320), degree 16",
                   "n_tasks": len(tasks), "parallelism": "single GPU"},
        "flops_per_batched_filter": flops,
        "fp64": f64, "s_per_pass_batched_fp64": round(t_pass, 3),
        "setup_s": round(t_setup, 1), "prologue_s": round(t_prologue, 1),
    }
    if "mixed" in res:
        out["mixed"] = res["mixed"]
        out["speedup_mixed_vs_fp64"] = round(f64["ms_per_filter"] / res["mixed"]["ms_per_filter"], 3)
    if mf:
        out["matrix_free"] = mf
    return out


def _adjoint_run(args, s, op, torch):
    """Median forward and backward times of the degree-m filter and its adjoint on
    op, the adjoint identity of the last run, and its outputs (Xbar, dV, dB)."""
    X = torch.empty((s.n_dof, s.n_vec), dtype=torch.complex128, device="cuda")
    op.fill_random(X, s.seed, n_total_cols=s.n_vec)
    v0 = torch.empty((s.n_dof, 1), dtype=torch.complex128, device="cuda")
    op.fill_random(v0, s.seed + 1)
    lo, hi = op.lanczos_bounds(v0[:, 0], 40)
    a, a0 = lo + 0.3 * (hi - lo), lo - 0.1
    flops = s.degree * _task_flops(op, 0, X, torch.empty_like(X))
    G = torch.empty_like(X)
    op.fill_random(G, s.seed + 2, n_total_cols=s.n_vec)
    Y, W, Xb = torch.empty_like(X), torch.empty_like(X), torch.empty_like(X)
    dV = torch.zeros((op.n_cells, op.nq3), dtype=torch.float64, device="cuda")
    dB = torch.zeros((op.n_cells, op.nq3, 3), dtype=torch.float64, device="cuda")
    tf, tb = [], []
    for it in range(args.warmup + args.steps):
        Y.copy_(X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.cheb_filter(Y, W, s.degree, a, hi, a0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dV.zero_()
        dB.zero_()
        op.cheb_filter_backward(X, G, Xb, dV, dB, s.degree, a, hi, a0, ckpt_every=4)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if it >= args.warmup:
            tf.append(t1 - t0)
            tb.append(t2 - t1)
    # adjoint identity Re<G, p(H) X> = Re<p(H) G, X> as a consistency check of the timed run
    lhs = torch.vdot(G.flatten(), Y.flatten())
    rhs = torch.vdot(Xb.flatten(), X.flatten())
    rel = float((lhs - rhs).abs() / lhs.abs())
    ws = op.filter_backward_workspace(s.n_vec, s.degree, 4)
    return float(np.median(tf)), float(np.median(tb)), rel, flops, ws, (Xb, dV, dB)


def bench_adjoint(args, torch):
    """The differentiation workload: 10^3 cells, p=5 (250k spinor dofs), N=256,
    degree 16; forward filter and its adjoint (checkpoints every 4 steps) giving
    dL/dX, dL/dV_eff and dL/dB_xc at the quadrature points, with the stored cell
    matrices and with the matrix-free operator."""
    import synth
    s = synth.config("adjoint")
    op = build_operator(s, torch)
    tfm, tbm, rel, flops, ws, outs = _adjoint_run(args, s, op, torch)
    op.close()
    log(f"[bench] adjoint: forward {1e3 * tfm:.1f} ms, backward {1e3 * tbm:.1f} ms, identity rel {rel:.1e}")
    out = {
        "metric": "Chebyshev filter adjoint: dL/dX, dL/dV_eff, dL/dB_xc (checkpoints every 4 steps)",
        "value": round(1e3 * tbm, 2), "unit": "ms per backward", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * (tfm + tbm), 2), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "adjoint: 10^3 cells p=5 (250000 spinor dofs), 8 atoms l<=1, N=256, degree 16",
                   "parallelism": "single GPU"},
        "forward_ms": round(1e3 * tfm, 2), "forward_tflops": round(flops / tfm / 1e12, 3),
        "backward_over_forward": round(tbm / tfm, 3), "adjoint_identity_rel": rel,
        "workspace": ws,
    }
    if not args.no_matfree and s.n_q == s.p + 1:
        opm = build_operator(s, torch, form="matrix_free")
        tfm2, tbm2, rel2, _, _, outs2 = _adjoint_run(args, s, opm, torch)
        opm.close()
        diffs = [float((u - v).abs().max() / v.abs().max()) for u, v in zip(outs2, outs)]
        out["matrix_free"] = {"forward_ms": round(1e3 * tfm2, 2), "backward_ms": round(1e3 * tbm2, 2),
                              "adjoint_identity_rel": rel2,
                              "max_rel_diff_vs_cell_form": {"Xbar": diffs[0], "dV": diffs[1], "dB": diffs[2]}}
        log(f"[bench] adjoint matrix-free: forward {1e3 * tfm2:.1f} ms, backward {1e3 * tbm2:.1f} ms, "
            f"rel diff vs cell form {max(diffs):.1e}")
    return out


if __name__ == "__main__":
    main()
