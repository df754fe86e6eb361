// The self-consistent field loop (Sec. III.B, eqn:fixedpointmap): input
// densities -> (V_eff, B_xc) -> ChFSI -> Fermi-Dirac occupations -> output
// densities (eqn:rho, eqn:mag), mixed by Anderson's method in the inner product
// of eqn:innerPdt with a Kerker-preconditioned charge residual; optionally
// started on degree p-1 elements of the same cells and moved to degree p by
// interpolating the subspace (Sec. IV.A, eqn:FEWfnsCMesh).  Every field and
// block operation runs on the device; the host keeps the loop, the Anderson
// normal equations (depth x depth) and the occupations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <future>
#include <vector>

#include "internal.h"

using namespace chfsi;

namespace {

// dense solve A x = b (n small) by Gaussian elimination with partial pivoting
bool small_solve(std::vector<double> A, std::vector<double>& b, int n) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
    if (A[piv * n + k] == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double l = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
      b[i] -= l * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * b[j];
    b[k] = s / A[k * n + k];
  }
  return true;
}

void check_rc(int rc, chfsi_ctx* c, const char* what) {
  if (rc != CHFSI_OK)
    throw Error{rc, std::string(what) + ": " + (c ? c->last_error : std::string(chfsi_last_error(nullptr)))};
}

// Rayleigh-Ritz of a k-point's last pass with its host eigensolve on a helper
// thread: start() issues H X and the projected matrix (returning once that
// matrix is on the host) and hands it to the thread; the caller goes on with
// the next k-point's bound, filter and CholGS on the GPU; finish() takes the
// eigenpairs, rotates the block and stores the Ritz values.  Nothing between
// start() and finish() reads the block or the Ritz values of that k-point, and
// the rotation needs no H X (no residual norms here).
struct DeferredRR {
  chfsi_ctx* g = nullptr;
  void* X = nullptr;
  int64_t ldx = 0;
  int n = 0;
  double* theta = nullptr;
  std::vector<cplx> Hp, Q;
  std::vector<double> w;
  double ms = 0.0;
  std::future<void> job;        // last member: waited for before the vectors go

  void start(chfsi_ctx* ctx, int ik, void* Xb, int64_t ld, void* work, int64_t ldw, int nv, double* th) {
    g = ctx;
    X = Xb;
    ldx = ld;
    n = nv;
    theta = th;
    rr_project(g, ik, (const double2*)X, ldx, (double2*)work, ldw, n, Hp);
    job = std::async(std::launch::async, [this]() {
      const auto t0 = std::chrono::steady_clock::now();
      hermitian_eig(Hp, n, w, Q);
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    });
  }
  void finish() {
    if (!job.valid()) return;
    job.get();                  // rethrows a failure of the eigensolve
    stats_add_host(g, CHFSI_STAGE_HOST_DENSE, ms);
    rotate_inplace(g, (double2*)X, ldx, 2 * g->n_nodes, n, Q, false);
    for (int i = 0; i < n; ++i) theta[i] = w[i];
  }
};

}  // namespace

extern "C" {

int chfsi_field_inner(chfsi_ctx* c, const double* r1, const double* m1, const double* r2, const double* m2,
                      double* out) {
  if (!c) return CHFSI_EINVAL;
  try {
    CHFSI_CHECK(r1 && r2 && out, CHFSI_EINVAL, "field_inner: r1_d, r2_d and out must be non-NULL");
    CHFSI_CHECK((m1 == nullptr) == (m2 == nullptr), CHFSI_EINVAL, "field_inner: give both m1_d and m2_d or neither");
    *out = field_inner(c, r1, m1, r2, m2);
  } catch (const Error& e) {
    c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    c->last_error = e.what();
    return CHFSI_EINVAL;
  }
  return CHFSI_OK;
}

int chfsi_hartree(chfsi_ctx* c, const double* rho, double* vh, double tol, int max_iter, int* iters) {
  if (!c) return CHFSI_EINVAL;
  try {
    CHFSI_CHECK(rho && vh, CHFSI_EINVAL, "hartree: rho_d and vh_d must be non-NULL");
    CHFSI_CHECK(tol > 0.0 && max_iter >= 1, CHFSI_EINVAL, "hartree: need tol > 0 and max_iter >= 1");
    const int it = screened_poisson(c, 0.0, 4.0 * M_PI, rho, vh, tol, max_iter, nullptr);
    if (iters) *iters = it;
  } catch (const Error& e) {
    c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    c->last_error = e.what();
    return CHFSI_EINVAL;
  }
  return CHFSI_OK;
}

int chfsi_kerker(chfsi_ctx* c, double k0, const double* f, double* out, double tol, int max_iter, int* iters) {
  if (!c) return CHFSI_EINVAL;
  try {
    CHFSI_CHECK(f && out, CHFSI_EINVAL, "kerker: f_d and out_d must be non-NULL");
    CHFSI_CHECK(std::isfinite(k0) && k0 >= 0.0, CHFSI_EINVAL, "kerker: need k0 >= 0");
    CHFSI_CHECK(tol > 0.0 && max_iter >= 1, CHFSI_EINVAL, "kerker: need tol > 0 and max_iter >= 1");
    const int64_t np = (int64_t)c->n_cells * c->nq3;
    int it = 0;
    if (k0 == 0.0) {
      field_axpby(c, np, 1.0, f, 0.0, nullptr, out);
    } else {
      // w = (k0^2 - lap)^{-1} f in the FE space; K f = f - k0^2 w
      it = screened_poisson(c, k0 * k0, 1.0, f, out, tol, max_iter, nullptr);
      field_axpby(c, np, 1.0, f, -k0 * k0, out, out);
    }
    CHFSI_HIP(hipStreamSynchronize(c->stream));
    if (iters) *iters = it;
  } catch (const Error& e) {
    c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    c->last_error = e.what();
    return CHFSI_EINVAL;
  }
  return CHFSI_OK;
}

int chfsi_exchange(chfsi_ctx* c, const double* rho, const double* m, double* vx, double* bx) {
  if (!c) return CHFSI_EINVAL;
  try {
    CHFSI_CHECK(rho && m && vx && bx, CHFSI_EINVAL, "exchange: all arguments must be non-NULL");
    launch_exchange(c, (int64_t)c->n_cells * c->nq3, rho, m, nullptr, nullptr, vx, bx);
  } catch (const Error& e) {
    c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    c->last_error = e.what();
    return CHFSI_EINVAL;
  }
  return CHFSI_OK;
}

int chfsi_interpolate_block(chfsi_ctx* cc, chfsi_ctx* cf, const void* Yc, int64_t ldc, void* Yf, int64_t ldf,
                            int n_vec) {
  if (!cc || !cf) return CHFSI_EINVAL;
  try {
    CHFSI_CHECK(cf->p == cc->p + 1, CHFSI_EINVAL, "interpolate_block: the fine degree must be the coarse one + 1");
    for (int d = 0; d < 3; ++d) {
      CHFSI_CHECK(cc->nc[d] == cf->nc[d], CHFSI_EINVAL, "interpolate_block: the meshes must have the same cells");
      CHFSI_CHECK(cc->box[d] == cf->box[d], CHFSI_EINVAL, "interpolate_block: the meshes must have the same box");
    }
    CHFSI_CHECK(Yc && Yf && n_vec >= 1 && ldc >= n_vec && ldf >= n_vec, CHFSI_EINVAL,
                "interpolate_block: bad block arguments");
    CHFSI_CHECK(((uintptr_t)Yc % 16) == 0 && ((uintptr_t)Yf % 16) == 0, CHFSI_EINVAL,
                "interpolate_block: blocks must be 16-byte aligned");
    CHFSI_CHECK(cc->stream == cf->stream, CHFSI_EINVAL, "interpolate_block: the contexts must share a stream");
    interpolate_block(cc, cf, (const double2*)Yc, ldc, (double2*)Yf, ldf, n_vec);
  } catch (const Error& e) {
    cf->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    cf->last_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    cf->last_error = e.what();
    return CHFSI_EINVAL;
  }
  return CHFSI_OK;
}

int chfsi_scf_run(chfsi_ctx* fine, chfsi_ctx* coarse, const chfsi_scf_params* prm, const double* vext,
                  const double* bext, double* rho, double* mag, double* rho_out, double* mag_out, void* X,
                  int64_t ldx, double* theta_h, double* occ_h, chfsi_scf_record* hist, int max_hist, int* n_hist,
                  int* converged) {
  if (!fine) return CHFSI_EINVAL;
  try {
    CHFSI_CHECK(prm && vext && bext && rho && mag && rho_out && mag_out && X, CHFSI_EINVAL,
                "scf_run: a required pointer is NULL");
    const chfsi_scf_params& P = *prm;
    CHFSI_CHECK(P.n_vec >= 1 && ldx >= P.n_vec && P.degree >= 1 && P.passes >= 1 && P.passes_first >= 1 &&
                    P.depth >= 1 && P.depth <= 16 && P.max_iter >= 1 && P.max_coarse >= 1 && P.lanczos_steps >= 2,
                CHFSI_EINVAL, "scf_run: invalid counts in params");
    CHFSI_CHECK(P.tol > 0.0 && P.tol_coarse > 0.0 && P.field_tol > 0.0 && P.field_max_iter >= 1 &&
                    P.n_electrons > 0.0 && P.n_electrons < P.n_vec && P.kT > 0.0 && P.alpha > 0.0 && P.k0 >= 0.0,
                CHFSI_EINVAL, "scf_run: invalid tolerances, electron count, kT, alpha or k0 in params");
    CHFSI_CHECK(P.prec_mode == CHFSI_PREC_FP64 || P.prec_mode == CHFSI_PREC_MIXED, CHFSI_EINVAL,
                "scf_run: unknown precision");
    CHFSI_CHECK(((uintptr_t)X % 16) == 0, CHFSI_EINVAL, "scf_run: X_d must be 16-byte aligned");
    CHFSI_CHECK(P.start_given == 0 || (P.start_given == 1 && coarse == nullptr), CHFSI_EINVAL,
                "scf_run: start_given is 0 or 1, and a given start block needs no coarse grid");
    const int nk = (int)fine->kp.size();
    std::vector<chfsi_ctx*> grids;
    if (coarse) {
      CHFSI_CHECK(fine->p == coarse->p + 1, CHFSI_EINVAL, "scf_run: the coarse degree must be the fine one - 1");
      CHFSI_CHECK(coarse->nq == fine->nq && coarse->quad == fine->quad && coarse->n_cells == fine->n_cells,
                  CHFSI_EINVAL, "scf_run: both grids need the same cells and quadrature points");
      CHFSI_CHECK(coarse->stream == fine->stream, CHFSI_EINVAL, "scf_run: the contexts must share a stream");
      CHFSI_CHECK((int)coarse->kp.size() == nk, CHFSI_EINVAL, "scf_run: both grids need the same k-points");
      for (int ik = 0; ik < nk; ++ik)
        for (int d = 0; d < 3; ++d)
          CHFSI_CHECK(coarse->kp[ik]->k[d] == fine->kp[ik]->k[d], CHFSI_EINVAL,
                      "scf_run: both grids need the same k-points");
      grids.push_back(coarse);
    }
    grids.push_back(fine);
    // zone-average weights of the k-points
    std::vector<double> wk(nk, 1.0 / nk);
    if (P.kweights_h) {
      double ws = 0.0;
      for (int ik = 0; ik < nk; ++ik) {
        wk[ik] = P.kweights_h[ik];
        CHFSI_CHECK(std::isfinite(wk[ik]) && wk[ik] >= 0.0, CHFSI_EINVAL, "scf_run: k-point weights must be >= 0");
        ws += wk[ik];
      }
      CHFSI_CHECK(std::fabs(ws - 1.0) <= 1e-12, CHFSI_EINVAL, "scf_run: k-point weights must sum to 1");
    }
    chfsi_ctx* c = fine;
    const int N = P.n_vec;
    const int64_t np = (int64_t)c->n_cells * c->nq3;
    hipStream_t st = c->stream;
    // device work: potentials, output densities, Anderson history, blocks of the coarse grid
    DevBuf<double> V, B, Vh, Vb, ro, mo, fr, fm, xr, xm, kf;
    V.alloc(np);
    B.alloc(3 * np);
    Vh.alloc(np);
    Vb.alloc(np);
    ro.alloc(np);
    mo.alloc(3 * np);
    fr.alloc(np);
    fm.alloc(3 * np);
    xr.alloc(np);
    xm.alloc(3 * np);
    kf.alloc(np);
    std::vector<DevBuf<double>> hx(P.depth), hxm(P.depth), hf(P.depth), hfm(P.depth);
    for (int j = 0; j < P.depth; ++j) {
      hx[j].alloc(np);
      hxm[j].alloc(3 * np);
      hf[j].alloc(np);
      hfm[j].alloc(3 * np);
    }
    // mixed precision runs the residual form of the filter: its work blocks are two
    // columns wide per state, and the residual block R = H X - X diag(theta) is kept
    const bool resid_form = P.prec_mode == CHFSI_PREC_MIXED;
    const int wcols = resid_form ? 2 * N : N;
    DevBuf<double2> Xc, Wc, Wf, Rc, Rf, v0;
    if (coarse) {
      Xc.alloc((size_t)nk * 2 * coarse->n_nodes * N);
      Wc.alloc((size_t)2 * coarse->n_nodes * wcols);
      if (resid_form) Rc.alloc((size_t)2 * coarse->n_nodes * N);
    }
    Wf.alloc((size_t)2 * fine->n_nodes * wcols);
    if (resid_form) Rf.alloc((size_t)2 * fine->n_nodes * N);
    v0.alloc((size_t)2 * fine->n_nodes);
    // per k-point: Ritz values and occupations; occupations times weights
    std::vector<double> theta((size_t)nk * N), occ((size_t)nk * N), wts((size_t)nk * N), occw(N), rnorm(N);
    DeferredRR rr_late;
    for (int ik = 0; ik < nk; ++ik)
      for (int n = 0; n < N; ++n) wts[(size_t)ik * N + n] = wk[ik];
    int nh = 0, it = 0;
    bool conv = false;
    for (size_t gi = 0; gi < grids.size(); ++gi) {
      chfsi_ctx* g = grids[gi];
      c = g;                    // field solves in the FE space of the current grid
      const bool last = gi + 1 == grids.size();
      const int64_t ldg = last ? ldx : N;
      // block of k-point ik on this grid
      auto Xk = [&](int ik) -> void* {
        return last ? (void*)((double2*)X + (size_t)ik * 2 * fine->n_nodes * ldx)
                    : (void*)(Xc.ptr + (size_t)ik * 2 * coarse->n_nodes * N);
      };
      void* Wg = last ? (void*)Wf.ptr : (void*)Wc.ptr;
      void* Rg = last ? (void*)Rf.ptr : (void*)Rc.ptr;
      for (int ik = 0; ik < nk; ++ik) {
        if (gi == 0 && P.start_given) continue;   // the caller's blocks
        if (gi == 0)
          check_rc(chfsi_fill_random(g, Xk(ik), 2 * g->n_nodes, N, ldg, P.seed + 7919ull * (uint64_t)ik, 0, 0, N),
                   g, "scf_run: start block");
        else
          check_rc(chfsi_interpolate_block(grids[gi - 1], g, Xc.ptr + (size_t)ik * 2 * coarse->n_nodes * N, N,
                                           Xk(ik), ldg, N),
                   g, "scf_run: two-grid transfer");
      }
      int n_mix = 0;            // Anderson history is per grid
      int head = 0;             // ring slot of the next entry
      bool first = true;
      int n_here = 0;
      while (true) {
        ++it;
        ++n_here;
        // the map's first step: (V_eff, B_xc) of the input densities
        int cg_h = screened_poisson(c, 0.0, 4.0 * M_PI, rho, Vh.ptr, P.field_tol, P.field_max_iter, nullptr);
        field_axpby(c, np, 1.0, vext, 1.0, Vh.ptr, Vb.ptr);
        launch_exchange(c, np, rho, mag, Vb.ptr, bext, V.ptr, B.ptr);
        check_rc(chfsi_set_local(g, V.ptr, B.ptr), g, "scf_run: set_local");
        const int npass = (first && gi == 0) ? P.passes_first : P.passes;
        double b0 = 0.0;
        for (int ik = 0; ik < nk; ++ik) {
          double* th = theta.data() + (size_t)ik * N;
          double lo = 0.0, b = 0.0;
          const int64_t bi = (int64_t)(it - 1) * nk + ik;
          if (P.bounds_h && bi < P.n_bounds) {
            b = P.bounds_h[bi];
            CHFSI_CHECK(std::isfinite(b), CHFSI_EINVAL, "scf_run: non-finite upper bound in bounds_h");
          } else {
            check_rc(chfsi_fill_random(g, v0.ptr, 2 * g->n_nodes, 1, 1, P.lanczos_seed, 0, 0, 1), g,
                     "scf_run: Lanczos start");
            check_rc(chfsi_lanczos_bounds(g, ik, P.lanczos_steps, v0.ptr, &lo, &b), g, "scf_run: Lanczos");
          }
          if (ik == 0) b0 = b;
          void* Xg = Xk(ik);
          if (first) {
            int bad = -1;
            check_rc(chfsi_chol_gs(g, Xg, ldg, N, &bad), g, "scf_run: CholGS");
            check_rc(chfsi_rayleigh_ritz(g, ik, Xg, ldg, Wg, wcols, N, th, nullptr), g, "scf_run: RR");
          }
          if (resid_form) {
            // R = H X - X diag(theta) for this iteration's operator (FP64)
            check_rc(chfsi_apply_H(g, ik, Xg, ldg, Rg, N, N, CHFSI_PREC_FP64), g, "scf_run: residual apply");
            check_rc(chfsi_ritz_residual(g, Xg, ldg, Rg, N, N, th), g, "scf_run: residuals");
          }
          for (int p = 0; p < npass; ++p) {
            if (resid_form)
              check_rc(chfsi_cheb_filter_resid(g, ik, Xg, ldg, Rg, N, th, Wg, wcols, N, P.degree, th[N - 1], b, th[0],
                                               CHFSI_PREC_MIXED),
                       g, "scf_run: filter");
            else
              check_rc(chfsi_cheb_filter(g, ik, Xg, ldg, Wg, wcols, N, P.degree, th[N - 1], b, th[0], P.prec_mode), g,
                       "scf_run: filter");
            int bad = -1;
            check_rc(chfsi_chol_gs(g, Xg, ldg, N, &bad), g, "scf_run: CholGS");
            if (p + 1 < npass && resid_form) {
              // the next pass filters with R of the rotated block: H X into R, then
              // R = H X - X diag(theta)
              check_rc(chfsi_rayleigh_ritz(g, ik, Xg, ldg, Rg, N, N, th, rnorm.data()), g, "scf_run: RR");
              check_rc(chfsi_ritz_residual(g, Xg, ldg, Rg, N, N, th), g, "scf_run: residuals");
            } else if (p + 1 < npass) {
              // residual norms are not needed here: no rotation of H X
              check_rc(chfsi_rayleigh_ritz(g, ik, Xg, ldg, Wg, wcols, N, th, nullptr), g, "scf_run: RR");
            } else {
              // last pass of this k-point (in the residual form R is formed again
              // from the next iteration's operator): the eigensolve overlaps the
              // next k-point's GPU work
              rr_late.finish();
              rr_late.start(g, ik, Xg, ldg, Wg, wcols, N, th);
            }
          }
        }
        rr_late.finish();
        first = false;
        // one Fermi level for all (n, k); densities summed with the weights
        double mu = 0.0;
        check_rc(chfsi_fermi_dirac(nk * N, theta.data(), wts.data(), P.n_electrons, P.kT, occ.data(), &mu, nullptr),
                 nullptr, "scf_run: occupations");
        field_fill(c, np, 0.0, ro.ptr);
        field_fill(c, 3 * np, 0.0, mo.ptr);
        for (int ik = 0; ik < nk; ++ik) {
          for (int n = 0; n < N; ++n) occw[n] = wk[ik] * occ[(size_t)ik * N + n];
          check_rc(chfsi_density(g, Xk(ik), ldg, N, occw.data(), ro.ptr, mo.ptr), g, "scf_run: densities");
        }
        // hold exactly N_e electrons under the cell quadrature
        const double q = P.n_electrons / field_integral(c, ro.ptr);
        CHFSI_CHECK(std::isfinite(q) && q > 0.0, CHFSI_ENONFINITE, "scf_run: output density has no positive charge");
        field_axpby(c, np, q, ro.ptr, 0.0, nullptr, ro.ptr);
        field_axpby(c, 3 * np, q, mo.ptr, 0.0, nullptr, mo.ptr);
        field_axpby(c, np, 1.0, ro.ptr, -1.0, rho, fr.ptr);
        field_axpby(c, 3 * np, 1.0, mo.ptr, -1.0, mag, fm.ptr);
        const double nres = std::sqrt(field_inner(c, fr.ptr, fm.ptr, fr.ptr, fm.ptr));
        CHFSI_CHECK(std::isfinite(nres), CHFSI_ENONFINITE, "scf_run: non-finite density residual");
        double eband = 0.0, th0 = theta[0];
        for (int ik = 0; ik < nk; ++ik) {
          double e = 0.0;
          for (int n = 0; n < N; ++n) e += occ[(size_t)ik * N + n] * theta[(size_t)ik * N + n];
          eband += wk[ik] * e;
          th0 = std::min(th0, theta[(size_t)ik * N]);
        }
        if (hist && nh < max_hist)
          hist[nh] = chfsi_scf_record{g->p, nres, mu, eband, th0, cg_h, b0};
        ++nh;
        conv = nres < (last ? P.tol : P.tol_coarse);
        if (last && (conv || it >= P.max_iter)) {
          field_axpby(c, np, 1.0, ro.ptr, 0.0, nullptr, rho_out);
          field_axpby(c, 3 * np, 1.0, mo.ptr, 0.0, nullptr, mag_out);
          CHFSI_HIP(hipStreamSynchronize(st));
          if (theta_h) std::copy(theta.begin(), theta.end(), theta_h);
          if (occ_h) std::copy(occ.begin(), occ.end(), occ_h);
          if (n_hist) *n_hist = nh;
          if (converged) *converged = conv ? 1 : 0;
          return CHFSI_OK;
        }
        // Anderson: history entries oldest -> newest, at most depth of them
        field_axpby(c, np, 1.0, rho, 0.0, nullptr, hx[head].ptr);
        field_axpby(c, 3 * np, 1.0, mag, 0.0, nullptr, hxm[head].ptr);
        field_axpby(c, np, 1.0, fr.ptr, 0.0, nullptr, hf[head].ptr);
        field_axpby(c, 3 * np, 1.0, fm.ptr, 0.0, nullptr, hfm[head].ptr);
        head = (head + 1) % P.depth;
        n_mix = std::min(n_mix + 1, P.depth);
        std::vector<int> slot(n_mix);
        for (int j = 0; j < n_mix; ++j) slot[j] = (head - n_mix + j + 2 * P.depth) % P.depth;
        std::vector<double> A((size_t)n_mix * n_mix), cf(n_mix, 1.0);
        for (int j = 0; j < n_mix; ++j)
          for (int k = 0; k < n_mix; ++k)
            A[(size_t)j * n_mix + k] = field_inner(c, hf[slot[j]].ptr, hfm[slot[j]].ptr, hf[slot[k]].ptr,
                                                   hfm[slot[k]].ptr);
        CHFSI_CHECK(small_solve(A, cf, n_mix), CHFSI_ENONFINITE, "scf_run: singular Anderson matrix");
        double csum = 0.0;
        for (double v : cf) csum += v;
        for (double& v : cf) v /= csum;
        // x = sum b_j x_j, f = sum b_j f_j (in history order)
        for (int j = 0; j < n_mix; ++j) {
          const double bj = cf[j];
          const int s = slot[j];
          field_axpby(c, np, bj, hx[s].ptr, j ? 1.0 : 0.0, j ? xr.ptr : nullptr, xr.ptr);
          field_axpby(c, 3 * np, bj, hxm[s].ptr, j ? 1.0 : 0.0, j ? xm.ptr : nullptr, xm.ptr);
          field_axpby(c, np, bj, hf[s].ptr, j ? 1.0 : 0.0, j ? fr.ptr : nullptr, fr.ptr);
          field_axpby(c, 3 * np, bj, hfm[s].ptr, j ? 1.0 : 0.0, j ? fm.ptr : nullptr, fm.ptr);
        }
        // next input: x + alpha (K f_rho, f_m)
        check_rc(chfsi_kerker(c, P.k0, fr.ptr, kf.ptr, P.field_tol, P.field_max_iter, nullptr), c, "scf_run: Kerker");
        field_axpby(c, np, 1.0, xr.ptr, P.alpha, kf.ptr, rho);
        field_axpby(c, 3 * np, 1.0, xm.ptr, P.alpha, fm.ptr, mag);
        if (!last && (conv || n_here >= P.max_coarse || it >= P.max_iter)) break;
      }
    }
    throw Error{CHFSI_ESTATE, "scf_run: loop ended without the fine grid"};
  } catch (const Error& e) {
    fine->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    fine->last_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    fine->last_error = e.what();
    return CHFSI_EINVAL;
  }
}

}  // extern "C"
