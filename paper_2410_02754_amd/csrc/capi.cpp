// extern "C" entry points of the ChFSI library: argument validation, context
// lifetime, and the host-side sequencing of the device steps.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <chrono>
#include <new>

#include "internal.h"

using namespace chfsi;

namespace chfsi {
void tridiag_eigvals(std::vector<double> d, std::vector<double> e, std::vector<double>& w);
}

static std::string g_create_error;

#define API_BEGIN(ctx) \
  try {
#define API_END(ctx)                                           \
  }                                                            \
  catch (const chfsi::Error& e) {                              \
    if (ctx) (ctx)->last_error = e.msg;                        \
    return e.code;                                             \
  }                                                            \
  catch (const std::bad_alloc&) {                              \
    if (ctx) (ctx)->last_error = "host allocation failed";     \
    return CHFSI_ENOMEM;                                       \
  }                                                            \
  catch (const std::exception& e) {                            \
    if (ctx) (ctx)->last_error = e.what();                     \
    return CHFSI_EINVAL;                                       \
  }                                                            \
  return CHFSI_OK;

static KPoint& kpoint(chfsi_ctx* c, int ik) {
  CHFSI_CHECK(ik >= 0 && ik < (int)c->kp.size(), CHFSI_EINVAL, "k-point index out of range");
  return *c->kp[ik];
}

static void check_block(const chfsi_ctx* c, const void* p, int64_t ld, int n_vec, const char* what) {
  CHFSI_CHECK(p != nullptr, CHFSI_EINVAL, std::string(what) + " is NULL");
  CHFSI_CHECK(n_vec >= 1, CHFSI_EINVAL, "n_vec must be >= 1");
  CHFSI_CHECK(ld >= n_vec, CHFSI_EINVAL, std::string("ld of ") + what + " must be >= n_vec");
  CHFSI_CHECK(((uintptr_t)p % 16) == 0, CHFSI_EINVAL, std::string(what) + " must be 16-byte aligned");
  (void)c;
}

static void require_operator(const chfsi_ctx* c) {
  CHFSI_CHECK(c->have_local, CHFSI_ESTATE, "chfsi_set_local has not been called");
}

namespace chfsi {
void rr_project(chfsi_ctx* c, int ik, const double2* X, int64_t ldx, double2* work, int64_t ldw, int n_vec,
                std::vector<cplx>& Hp) {
  KPoint& kp = kpoint(c, ik);
  apply_H(c, kp, X, ldx, work, ldw, n_vec, CHFSI_PREC_FP64, 1.0, 0.0, 0.0);
  gram(c, X, ldx, work, ldw, 2 * c->n_nodes, n_vec, Hp, true);
  for (const auto& v : Hp)
    CHFSI_CHECK(std::isfinite(v.real()) && std::isfinite(v.imag()), CHFSI_ENONFINITE, "projected H has NaN/Inf");
}
}  // namespace chfsi


extern "C" {

const char* chfsi_version(void) { return "chfsi-mi355x 0.1"; }

const char* chfsi_last_error(const chfsi_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

int chfsi_create(const chfsi_mesh_desc* d, void* stream, chfsi_ctx** out) {
  chfsi_ctx* c = nullptr;
  try {
    CHFSI_CHECK(d != nullptr && out != nullptr, CHFSI_EINVAL, "desc and out must be non-NULL");
    for (int k = 0; k < 3; ++k) {
      CHFSI_CHECK(d->n_cells[k] >= 2 && d->n_cells[k] <= 4096, CHFSI_EINVAL, "n_cells must be in [2, 4096]");
      CHFSI_CHECK(d->box[k] > 0.0 && std::isfinite(d->box[k]), CHFSI_EINVAL, "box lengths must be > 0");
    }
    CHFSI_CHECK(d->p >= 1 && d->p <= kMaxP, CHFSI_EINVAL, "p must be in [1, 8]");
    CHFSI_CHECK(d->quad == CHFSI_QUAD_GL || d->quad == CHFSI_QUAD_GLL, CHFSI_EINVAL, "unknown quadrature");
    if (d->quad == CHFSI_QUAD_GL)
      CHFSI_CHECK(d->n_q >= 1 && d->n_q <= kMaxNq, CHFSI_EINVAL, "n_q must be in [1, 12]");
    CHFSI_CHECK(d->n_k >= 1 && d->kpts != nullptr, CHFSI_EINVAL, "need n_k >= 1 k-points");
    const int64_t nodes = (int64_t)d->n_cells[0] * d->p * d->n_cells[1] * d->p * d->n_cells[2] * d->p;
    CHFSI_CHECK(nodes < ((int64_t)1 << 30), CHFSI_EINVAL, "mesh too large for 32-bit node ids");
    c = new chfsi_ctx();
    for (int k = 0; k < 3; ++k) {
      c->nc[k] = d->n_cells[k];
      c->box[k] = d->box[k];
    }
    c->p = d->p;
    c->np1 = d->p + 1;
    c->quad = d->quad;
    c->stream = (hipStream_t)stream;
    CHFSI_HIP(hipGetDevice(&c->device));
    noalloc_scratch_init();
    c->ref = make_ref(d->p, d->quad, d->n_q);
    c->nq = c->ref.nq;
    build_mesh(c);
    build_uniform_mats(c);
    for (int ik = 0; ik < d->n_k; ++ik) {
      KPoint* kp = new KPoint();
      for (int k = 0; k < 3; ++k) kp->k[k] = d->kpts[3 * ik + k];
      kp->gamma = kp->k[0] == 0.0 && kp->k[1] == 0.0 && kp->k[2] == 0.0;
      kp->nmat = kp->gamma ? 4 : 5;
      c->kp.push_back(kp);
    }
    CHFSI_HIP(hipStreamSynchronize(c->stream));
    *out = c;
    return CHFSI_OK;
  } catch (const chfsi::Error& e) {
    g_create_error = e.msg;
    if (c) chfsi_destroy(c);
    return e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    if (c) chfsi_destroy(c);
    return CHFSI_ENOMEM;
  }
}

int chfsi_destroy(chfsi_ctx* c) {
  if (!c) return CHFSI_OK;
  (void)hipStreamSynchronize(c->stream);
  for (auto* k : c->kp) delete k;
  delete c;
  return CHFSI_OK;
}

int chfsi_sizes(const chfsi_ctx* c, int64_t* n_nodes, int64_t* n_dof, int* n_cells, int* nq3, int* n_colours) {
  if (!c) return CHFSI_EINVAL;
  if (n_nodes) *n_nodes = c->n_nodes;
  if (n_dof) *n_dof = 2 * c->n_nodes;
  if (n_cells) *n_cells = c->n_cells;
  if (nq3) *nq3 = c->nq3;
  if (n_colours) *n_colours = c->n_colours;
  return CHFSI_OK;
}

int chfsi_quad_points(const chfsi_ctx* c, double* xyz) {
  if (!c || !xyz) return CHFSI_EINVAL;
  const int nq = c->nq;
  for (int e = 0; e < c->n_cells; ++e) {
    const int cc[3] = {e % c->nc[0], (e / c->nc[0]) % c->nc[1], e / (c->nc[0] * c->nc[1])};
    for (int q = 0; q < c->nq3; ++q) {
      const int qa[3] = {q % nq, (q / nq) % nq, q / (nq * nq)};
      for (int d = 0; d < 3; ++d)
        xyz[((size_t)e * c->nq3 + q) * 3 + d] = cc[d] * c->h[d] + (c->ref.xq[qa[d]] + 1.0) * 0.5 * c->h[d];
    }
  }
  return CHFSI_OK;
}

int chfsi_set_apply_form(chfsi_ctx* c, int form) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  CHFSI_CHECK(form == CHFSI_FORM_CELL_MATRIX || form == CHFSI_FORM_MATRIX_FREE, CHFSI_EINVAL, "unknown form");
  if (form == CHFSI_FORM_MATRIX_FREE) {
    CHFSI_CHECK(mf_supported(c), CHFSI_EINVAL, "matrix-free form needs n_q = p + 1");
    mf_prepare(c);
  }
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  // drop the other form's data; the operator is rebuilt by the next set_local
  for (auto* kp : c->kp) {
    kp->cell64.release();
    kp->cell32.release();
  }
  c->mf_qd.release();
  c->mf_qd32.release();
  c->form = form;
  c->have_local = false;
  ++c->gen;
  API_END(c)
}

int chfsi_set_local(chfsi_ctx* c, const double* V, const double* B) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  CHFSI_CHECK(V && B, CHFSI_EINVAL, "veff_d and bxc_d must be non-NULL");
  CHFSI_CHECK(check_finite(c, V, (int64_t)c->n_cells * c->nq3), CHFSI_ENONFINITE, "veff has NaN/Inf");
  CHFSI_CHECK(check_finite(c, B, (int64_t)c->n_cells * c->nq3 * 3), CHFSI_ENONFINITE, "bxc has NaN/Inf");
  ++c->gen;
  if (c->form == CHFSI_FORM_MATRIX_FREE) {
    mf_set_local(c, V, B);
    c->have_local = true;
    return CHFSI_OK;
  }
  const int N = c->nloc;
  for (auto* kp : c->kp) {
    // uniform parts of the cell operator for this k:
    //   U0 = kinetic + |k|^2/2 mass;  S = -(C - C^T)/2 with C = sum_d k_d C_d
    // (the k-gradient term -i C of eqn:FEHloc, skew-symmetrised per cell; the
    // symmetric part of C sums to zero over the periodic mesh)
    const double k2 = kp->k[0] * kp->k[0] + kp->k[1] * kp->k[1] + kp->k[2] * kp->k[2];
    std::vector<double> U0((size_t)N * N), S((size_t)N * N, 0.0);
    for (size_t t = 0; t < U0.size(); ++t) U0[t] = c->Kin[t] + 0.5 * k2 * c->Mcons[t];
    if (!kp->gamma)
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          double cij = 0.0, cji = 0.0;
          for (int d = 0; d < 3; ++d) {
            cij += kp->k[d] * c->Cgrad[d][(size_t)i * N + j];
            cji += kp->k[d] * c->Cgrad[d][(size_t)j * N + i];
          }
          S[(size_t)i * N + j] = -0.5 * (cij - cji);
        }
    DevBuf<double> dU, dS;
    dU.upload(U0.data(), U0.size(), c->stream);
    dS.upload(S.data(), S.size(), c->stream);
    launch_cell_setup(c, *kp, V, B, dU.ptr, dS.ptr);
    launch_cell_to_f32(c, *kp);
    CHFSI_HIP(hipStreamSynchronize(c->stream));
  }
  // the matrix-free quadrature data as well (w_q J (V, B) per point, 32 B): the
  // single-column applies of the Lanczos bounds use it instead of streaming the
  // cell operators for one column
  if (mf_supported(c)) mf_set_local(c, V, B);
  c->have_local = true;
  API_END(c)
}

int chfsi_set_atoms(chfsi_ctx* c, int n_atoms, const chfsi_atom_desc* atoms) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  CHFSI_CHECK(n_atoms >= 0 && (n_atoms == 0 || atoms != nullptr), CHFSI_EINVAL, "bad atom list");
  for (int a = 0; a < n_atoms; ++a) {
    const auto& at = atoms[a];
    CHFSI_CHECK(at.lmax >= 0 && at.lmax <= 2, CHFSI_EINVAL, "lmax must be in [0, 2]");
    CHFSI_CHECK(at.sigma > 0.0 && at.rcut > 0.0, CHFSI_EINVAL, "sigma and rcut must be > 0");
    for (int d = 0; d < 3; ++d) CHFSI_CHECK(std::isfinite(at.pos[d]), CHFSI_ENONFINITE, "atom position NaN/Inf");
    if (at.delta_override) {
      const int nd = 2 * (at.lmax + 1) * (at.lmax + 1);
      for (int i = 0; i < nd; ++i)
        for (int j = 0; j < nd; ++j) {
          const double* a1 = at.delta_override + 2 * ((size_t)i * nd + j);
          const double* a2 = at.delta_override + 2 * ((size_t)j * nd + i);
          CHFSI_CHECK(std::isfinite(a1[0]) && std::isfinite(a1[1]), CHFSI_ENONFINITE, "Delta has NaN/Inf");
          CHFSI_CHECK(std::fabs(a1[0] - a2[0]) <= 1e-12 * (1 + std::fabs(a1[0])) &&
                          std::fabs(a1[1] + a2[1]) <= 1e-12 * (1 + std::fabs(a1[1])),
                      CHFSI_ENONHERM, "Delta override is not Hermitian");
        }
    }
  }
  ++c->gen;
  for (auto* kp : c->kp) build_nonlocal(c, *kp, n_atoms, atoms);
  API_END(c)
}

int chfsi_apply_H(chfsi_ctx* c, int ik, const void* X, int64_t ldx, void* Y, int64_t ldy, int n_vec, int prec) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  require_operator(c);
  check_block(c, X, ldx, n_vec, "X");
  check_block(c, Y, ldy, n_vec, "Y");
  CHFSI_CHECK(X != Y, CHFSI_EINVAL, "X and Y must be distinct");
  CHFSI_CHECK(prec == CHFSI_PREC_FP64 || prec == CHFSI_PREC_MIXED, CHFSI_EINVAL, "unknown precision");
  KPoint& kp = kpoint(c, ik);
  apply_H(c, kp, (const double2*)X, ldx, (double2*)Y, ldy, n_vec, prec, 1.0, 0.0, 0.0);
  API_END(c)
}

}  // extern "C"

namespace chfsi {
KPoint& kpoint_of(chfsi_ctx* c, int ik) { return kpoint(c, ik); }

void check_filter_args(chfsi_ctx* c, void* X, int64_t ldx, void* work, int64_t ldw, int n_vec, int degree,
                       double a, double b, double a0, int prec_mode) {
  require_operator(c);
  check_block(c, X, ldx, n_vec, "X");
  check_block(c, work, ldw, n_vec, "work");
  CHFSI_CHECK(X != work, CHFSI_EINVAL, "X and work must be distinct");
  CHFSI_CHECK(degree >= 1, CHFSI_EINVAL, "degree must be >= 1");
  CHFSI_CHECK(std::isfinite(a) && std::isfinite(b) && std::isfinite(a0) && a0 < a && a < b, CHFSI_EINVAL,
              "filter bounds must satisfy a0 < a < b");
  CHFSI_CHECK(prec_mode == CHFSI_PREC_FP64 || prec_mode == CHFSI_PREC_MIXED, CHFSI_EINVAL, "unknown precision");
}

// the scaled recurrence of chfsi_cheb_filter (arguments already checked)
void cheb_filter_run(chfsi_ctx* c, KPoint& kp, void* X, int64_t ldx, void* work, int64_t ldw, int n_vec,
                     int degree, double a, double b, double a0, int prec_mode) {
  const double e = 0.5 * (b - a), cc = 0.5 * (b + a);
  const double sigma1 = e / (a0 - cc);
  double sigma = sigma1;
  double2* bufs[2] = {(double2*)X, (double2*)work};
  const int64_t lds[2] = {ldx, ldw};
  // Y_1 = (sigma_1/e)(H - c) X -> work
  {
    const double al = sigma1 / e;
    const int prec = (prec_mode == CHFSI_PREC_MIXED && degree > 1) ? CHFSI_PREC_MIXED : CHFSI_PREC_FP64;
    apply_H(c, kp, bufs[0], lds[0], bufs[1], lds[1], n_vec, prec, al, 0.0, -cc * al);
  }
  int cur = 1;   // buffer holding Y_k
  for (int k = 2; k <= degree; ++k) {
    const double sn = 1.0 / (2.0 / sigma1 - sigma);
    const double al = 2.0 * sn / e;
    const double be = -sigma * sn;
    const int prec = (prec_mode == CHFSI_PREC_MIXED && k < degree) ? CHFSI_PREC_MIXED : CHFSI_PREC_FP64;
    // Y_{k} = al (H - c) Y_{k-1} + be Y_{k-2}, written over Y_{k-2}
    apply_H(c, kp, bufs[cur], lds[cur], bufs[cur ^ 1], lds[cur ^ 1], n_vec, prec, al, be, -cc * al);
    cur ^= 1;
    sigma = sn;
  }
  if (cur == 1) launch_copy_rows(c, bufs[0], ldx, bufs[1], ldw, 2 * c->n_nodes, n_vec);
}
}  // namespace chfsi

extern "C" {

int chfsi_cheb_filter(chfsi_ctx* c, int ik, void* X, int64_t ldx, void* work, int64_t ldw, int n_vec,
                      int degree, double a, double b, double a0, int prec_mode) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  check_filter_args(c, X, ldx, work, ldw, n_vec, degree, a, b, a0, prec_mode);
  KPoint& kp = kpoint(c, ik);
  cheb_filter_run(c, kp, X, ldx, work, ldw, n_vec, degree, a, b, a0, prec_mode);
  API_END(c)
}

int chfsi_ritz_residual(chfsi_ctx* c, const void* X, int64_t ldx, void* W, int64_t ldw, int n_vec,
                        const double* theta) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  check_block(c, X, ldx, n_vec, "X");
  check_block(c, W, ldw, n_vec, "W");
  CHFSI_CHECK(theta != nullptr, CHFSI_EINVAL, "theta_h must be non-NULL");
  std::vector<double> ab(2 * (size_t)n_vec);
  for (int i = 0; i < n_vec; ++i) {
    ab[i] = 1.0;
    ab[n_vec + i] = -theta[i];
  }
  DevBuf<double> d;
  d.upload(ab.data(), ab.size(), c->stream);
  launch_cols_axpby(c, (double2*)W, ldw, (const double2*)X, ldx, 2 * c->n_nodes, n_vec, d.ptr, d.ptr + n_vec);
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  API_END(c)
}

int chfsi_cheb_filter_resid(chfsi_ctx* c, int ik, void* X, int64_t ldx, const void* R, int64_t ldr,
                            const double* theta, void* work, int64_t ldw, int n_vec, int degree, double a, double b,
                            double a0, int prec_mode) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  require_operator(c);
  check_block(c, X, ldx, n_vec, "X");
  check_block(c, R, ldr, n_vec, "R");
  CHFSI_CHECK(work != nullptr && ldw >= 2 * (int64_t)n_vec && ((uintptr_t)work % 16) == 0, CHFSI_EINVAL,
              "work must be [2M][>= 2 n_vec], 16-byte aligned");
  CHFSI_CHECK(theta != nullptr, CHFSI_EINVAL, "theta_h must be non-NULL");
  CHFSI_CHECK(degree >= 1, CHFSI_EINVAL, "degree must be >= 1");
  CHFSI_CHECK(std::isfinite(a) && std::isfinite(b) && std::isfinite(a0) && a0 < a && a < b, CHFSI_EINVAL,
              "filter bounds must satisfy a0 < a < b");
  CHFSI_CHECK(prec_mode == CHFSI_PREC_FP64 || prec_mode == CHFSI_PREC_MIXED, CHFSI_EINVAL, "unknown precision");
  KPoint& kp = kpoint(c, ik);
  const int m = degree, n = n_vec;
  const int64_t rows = 2 * c->n_nodes;
  const double e = 0.5 * (b - a), cc = 0.5 * (b + a), s1 = e / (a0 - cc);
  std::vector<double> al(m + 1, 0.0), be(m + 1, 0.0);
  double sg = s1;
  al[1] = s1 / e;
  for (int k = 2; k <= m; ++k) {
    const double sn = 1.0 / (2.0 / s1 - sg);
    al[k] = 2.0 * sn / e;
    be[k] = -sg * sn;
    sg = sn;
  }
  // scalar recurrences p_k(theta_i), k = 0..m; table of source scales
  // src[k][i] = al[k] p_{k-1}(theta_i) for k = 2..m, and the final p_m
  std::vector<double> tab((size_t)(m + 2) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double pkm1 = 1.0, pk = al[1] * (theta[i] - cc);   // p_0, p_1
    for (int k = 2; k <= m; ++k) {
      tab[(size_t)k * n + i] = al[k] * pk;              // al_k p_{k-1}
      const double pn = al[k] * (theta[i] - cc) * pk + be[k] * pkm1;
      pkm1 = pk;
      pk = pn;
    }
    tab[(size_t)(m + 1) * n + i] = (m >= 1) ? pk : 1.0;  // p_m(theta_i)
    tab[i] = 1.0;                                        // ones for the final combination
  }
  DevBuf<double> dt;
  dt.upload(tab.data(), tab.size(), c->stream);
  double2* Z[2] = {(double2*)work, (double2*)work + n};
  // Z_1 = al_1 R
  launch_axpby_rows(c, Z[0], ldw, (const double2*)R, ldr, rows, n, 0.0, al[1]);
  int cur = 0;
  for (int k = 2; k <= m; ++k) {
    // Z_k = al_k (H - c) Z_{k-1} + be_k Z_{k-2} + al_k R p_{k-1}(Theta), written over Z_{k-2}
    apply_H3(c, kp, Z[cur], ldw, Z[cur ^ 1], ldw, Z[cur ^ 1], ldw, n, prec_mode, al[k], k == 2 ? 0.0 : be[k],
             -cc * al[k], (const double2*)R, ldr, dt.ptr + (size_t)k * n);
    cur ^= 1;
  }
  // X <- X p_m(Theta) + Z_m
  launch_cols_axpby(c, (double2*)X, ldx, Z[cur], ldw, rows, n, dt.ptr + (size_t)(m + 1) * n, dt.ptr);
  CHFSI_HIP(hipStreamSynchronize(c->stream));   // dt leaves scope
  API_END(c)
}

int chfsi_chol_gs(chfsi_ctx* c, void* X, int64_t ldx, int n_vec, int* bad_col) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  check_block(c, X, ldx, n_vec, "X");
  if (bad_col) *bad_col = -1;
  const int64_t rows = 2 * c->n_nodes;
  std::vector<cplx> S;
  gram(c, (const double2*)X, ldx, (const double2*)X, ldx, rows, n_vec, S, true);
  for (const auto& v : S)
    CHFSI_CHECK(std::isfinite(v.real()) && std::isfinite(v.imag()), CHFSI_ENONFINITE, "Gram matrix has NaN/Inf");
  auto t0 = std::chrono::steady_clock::now();
  // diagonal pre-scaling: S' = D S D with D = diag(S)^{-1/2} (unit diagonal), S' = L' L'^H,
  // X <- X D L'^{-H}.  In exact arithmetic D^{-1} L' is the Cholesky factor of S, so the
  // result is the unscaled one; columns of very different norms no longer set the
  // factor's conditioning.
  std::vector<double> dsc(n_vec);
  for (int j = 0; j < n_vec; ++j) {
    const double sjj = S[(size_t)j * n_vec + j].real();
    if (!(sjj > 0.0)) {
      if (bad_col) *bad_col = j;
      throw Error{CHFSI_ENOTPD, "Gram matrix not positive definite at column " + std::to_string(j)};
    }
    dsc[j] = 1.0 / std::sqrt(sjj);
  }
  for (int i = 0; i < n_vec; ++i)
    for (int j = 0; j < n_vec; ++j) S[(size_t)i * n_vec + j] *= dsc[i] * dsc[j];
  const int bad = cholesky_lower(S, n_vec);
  if (bad >= 0) {
    if (bad_col) *bad_col = bad;
    throw Error{CHFSI_ENOTPD, "Gram matrix not positive definite at column " + std::to_string(bad)};
  }
  std::vector<cplx> Linv, R((size_t)n_vec * n_vec);
  lower_inverse(S, n_vec, Linv);
  for (int i = 0; i < n_vec; ++i)
    for (int j = 0; j < n_vec; ++j) R[(size_t)i * n_vec + j] = dsc[i] * std::conj(Linv[(size_t)j * n_vec + i]);
  stats_add_host(c, CHFSI_STAGE_HOST_DENSE,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  rotate_inplace(c, (double2*)X, ldx, rows, n_vec, R, true);
  API_END(c)
}

int chfsi_overlap(chfsi_ctx* c, const void* X, int64_t ldx, const void* Y, int64_t ldy, int n_vec, double* S_h) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  check_block(c, X, ldx, n_vec, "X");
  check_block(c, Y, ldy, n_vec, "Y");
  CHFSI_CHECK(S_h != nullptr, CHFSI_EINVAL, "S_h is NULL");
  std::vector<cplx> S;
  gram(c, (const double2*)X, ldx, (const double2*)Y, ldy, 2 * c->n_nodes, n_vec, S, false);
  std::memcpy(S_h, S.data(), S.size() * sizeof(cplx));
  API_END(c)
}

size_t chfsi_workspace_bytes(const chfsi_ctx* c, int ik, int n_vec, int op) {
  if (!c || n_vec < 1 || ik < 0 || ik >= (int)c->kp.size()) return 0;
  auto cdiv = [](int64_t a, int64_t b) { return (int)((a + b - 1) / b); };
  const size_t n = (size_t)n_vec;
  const int64_t rows = 2 * c->n_nodes;
  // gram(): partial tiles of one resident round + the reduced matrix + tile list
  const int nti = cdiv(n_vec, 128), ntj = cdiv(n_vec, 64);
  const size_t ntl = (size_t)nti * ntj;
  const int64_t n_chunks = std::max<int64_t>(1, (rows + 255) / 256);
  const size_t n_groups = (size_t)std::max<int64_t>(1, std::min<int64_t>(n_chunks, 512 / (int64_t)ntl));
  const size_t gram_b = (2 * (n_groups * n * n + n * n) + ntl) * sizeof(double);
  // rotate_inplace(): a row panel of at most 128 MiB + the n x n rotation
  int64_t prow = std::max<int64_t>(128, ((int64_t)1 << 27) / ((int64_t)n * 16));
  prow = std::min<int64_t>(prow, rows);
  prow = (prow + 127) / 128 * 128;
  const size_t rot_b = ((size_t)prow * n + n * n) * sizeof(double2);
  const size_t resid_b = (256 * n + n) * sizeof(double);
  const size_t nl_b = nonlocal_scratch_bytes(*c->kp[ik], n_vec);
  switch (op) {
    case CHFSI_OP_APPLY:
    case CHFSI_OP_FILTER:
      return nl_b;
    case CHFSI_OP_CHOL_GS:
      return gram_b + rot_b;
    case CHFSI_OP_RAYLEIGH_RITZ:
      return std::max(std::max(nl_b, gram_b), resid_b) + rot_b;
    case CHFSI_OP_DENSITY: {
      const int want = std::max(1, cdiv(4096, std::max(1, c->n_cells)));
      int64_t groups;
      size_t order = 0;
      if (c->nq == c->np1) {
        // sum-factorised kernel: 4-column chunks, at least two interleaved groups,
        // and the tiled cell order it keeps
        groups = std::max<int64_t>(1, std::min<int64_t>(cdiv(n_vec, 4), std::max(2, want)));
        order = (size_t)c->n_cells * sizeof(int32_t);
      } else {
        groups = std::min<int64_t>(n_vec, want);
      }
      return (size_t)groups * c->n_cells * c->nq3 * 4 * sizeof(double) + n * sizeof(double) + order;
    }
    default:
      return 0;
  }
}


int chfsi_rayleigh_ritz(chfsi_ctx* c, int ik, void* X, int64_t ldx, void* work, int64_t ldw, int n_vec,
                        double* ritz, double* resid) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  require_operator(c);
  check_block(c, X, ldx, n_vec, "X");
  check_block(c, work, ldw, n_vec, "work");
  CHFSI_CHECK(ritz != nullptr, CHFSI_EINVAL, "ritz_h must be non-NULL");
  CHFSI_CHECK(X != work, CHFSI_EINVAL, "X and work must be distinct");
  const int64_t rows = 2 * c->n_nodes;
  std::vector<cplx> Hp;
  rr_project(c, ik, (const double2*)X, ldx, (double2*)work, ldw, n_vec, Hp);
  std::vector<double> w;
  std::vector<cplx> Q;
  auto t0 = std::chrono::steady_clock::now();
  hermitian_eig(Hp, n_vec, w, Q);
  stats_add_host(c, CHFSI_STAGE_HOST_DENSE,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  rotate_inplace(c, (double2*)X, ldx, rows, n_vec, Q, false);
  for (int i = 0; i < n_vec; ++i) ritz[i] = w[i];
  if (resid) {
    rotate_inplace(c, (double2*)work, ldw, rows, n_vec, Q, false);
    column_resid_norms(c, (const double2*)work, ldw, (const double2*)X, ldx, rows, n_vec, w.data(), resid);
  }
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  API_END(c)
}

int chfsi_lanczos_bounds(chfsi_ctx* c, int ik, int steps, const void* v0, double* lo, double* hi) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  require_operator(c);
  CHFSI_CHECK(v0 && lo && hi, CHFSI_EINVAL, "v0_d, lo and hi must be non-NULL");
  CHFSI_CHECK(steps >= 1 && steps <= 10000, CHFSI_EINVAL, "steps must be in [1, 10000]");
  KPoint& kp = kpoint(c, ik);
  const int64_t rows = 2 * c->n_nodes;
  DevBuf<double2> vb;
  vb.alloc((size_t)3 * rows);
  double2* v = vb.ptr;
  double2* w = v + rows;
  double2* vp = w + rows;
  const double n0 = std::sqrt(dot_re(c, (const double2*)v0, (const double2*)v0, rows));
  CHFSI_CHECK(n0 > 0.0 && std::isfinite(n0), CHFSI_EINVAL, "v0 must be finite and nonzero");
  launch_axpby_rows(c, v, 1, (const double2*)v0, 1, rows, 1, 0.0, 1.0 / n0);
  launch_axpby_rows(c, vp, 1, v, 1, rows, 1, 0.0, 0.0);
  double beta = 0.0;
  std::vector<double> al, be;
  // one column per apply: with the matrix-free data of the current fields at
  // hand the local part takes the matrix-free product (the same operator up to
  // rounding), which reads no cell matrices
  struct FormGuard {
    chfsi_ctx* c;
    int form;
    ~FormGuard() { c->form = form; }
  } fg{c, c->form};
  if (c->form == CHFSI_FORM_CELL_MATRIX && c->mf_gen == c->gen) c->form = CHFSI_FORM_MATRIX_FREE;
  for (int j = 0; j < steps; ++j) {
    apply_H(c, kp, v, 1, w, 1, 1, CHFSI_PREC_FP64, 1.0, 0.0, 0.0);
    const double alpha = dot_re(c, v, w, rows);
    launch_axpby_rows(c, w, 1, v, 1, rows, 1, 1.0, -alpha);
    launch_axpby_rows(c, w, 1, vp, 1, rows, 1, 1.0, -beta);
    const double bn = std::sqrt(dot_re(c, w, w, rows));
    al.push_back(alpha);
    if (j < steps - 1) be.push_back(bn);
    std::swap(vp, v);                                   // vp <- v
    if (bn > 0.0) launch_axpby_rows(c, v, 1, w, 1, rows, 1, 0.0, 1.0 / bn);
    beta = bn;
    if (!(bn > 0.0)) break;
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  std::vector<double> th;
  tridiag_eigvals(al, be, th);
  *lo = th.front();
  *hi = th.back() + beta;
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  API_END(c)
}

// Fermi-Dirac occupation of one level: 1 / (1 + exp((eps - mu) / kT)) in a form
// that neither overflows nor loses the small tail.
static double fermi_occ(double eps, double mu, double kT) {
  const double x = (eps - mu) / kT;
  if (x > 0.0) {
    const double t = std::exp(-x);
    return t / (1.0 + t);
  }
  return 1.0 / (1.0 + std::exp(x));
}

static double fermi_count(int n, const double* eps, const double* w, double mu, double kT) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += (w ? w[i] : 1.0) * fermi_occ(eps[i], mu, kT);
  return s;
}

int chfsi_fermi_dirac(int n, const double* eps, const double* w, double n_electrons, double kT, double* occ,
                      double* mu_out, double* e_ent_out) {
  try {
    CHFSI_CHECK(n >= 1 && eps && occ, CHFSI_EINVAL, "fermi_dirac: need n >= 1 and non-NULL eps, occ");
    CHFSI_CHECK(std::isfinite(kT) && kT > 0.0, CHFSI_EINVAL, "fermi_dirac: kT must be positive");
    double wsum = 0.0, lo = eps[0], hi = eps[0];
    for (int i = 0; i < n; ++i) {
      CHFSI_CHECK(std::isfinite(eps[i]), CHFSI_EINVAL, "fermi_dirac: non-finite eigenvalue");
      const double wi = w ? w[i] : 1.0;
      CHFSI_CHECK(std::isfinite(wi) && wi >= 0.0, CHFSI_EINVAL, "fermi_dirac: weights must be >= 0");
      wsum += wi;
      lo = std::min(lo, eps[i]);
      hi = std::max(hi, eps[i]);
    }
    CHFSI_CHECK(n_electrons > 0.0 && n_electrons < wsum, CHFSI_EINVAL,
                "fermi_dirac: need 0 < n_electrons < sum of weights");
    // bracket: the count rises monotonically in mu from 0 to sum w
    lo -= 50.0 * kT;
    hi += 50.0 * kT;
    for (int it = 0; it < 64 && fermi_count(n, eps, w, lo, kT) >= n_electrons; ++it) lo -= (hi - lo);
    for (int it = 0; it < 64 && fermi_count(n, eps, w, hi, kT) <= n_electrons; ++it) hi += (hi - lo);
    double mu = 0.5 * (lo + hi);
    for (int it = 0; it < 400; ++it) {
      mu = 0.5 * (lo + hi);
      if (fermi_count(n, eps, w, mu, kT) < n_electrons)
        lo = mu;
      else
        hi = mu;
      if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(mu))) break;
    }
    mu = 0.5 * (lo + hi);
    double ent = 0.0;
    for (int i = 0; i < n; ++i) {
      const double f = fermi_occ(eps[i], mu, kT);
      occ[i] = f;
      if (f > 0.0 && f < 1.0) ent += (w ? w[i] : 1.0) * (f * std::log(f) + (1.0 - f) * std::log1p(-f));
    }
    if (mu_out) *mu_out = mu;
    if (e_ent_out) *e_ent_out = kT * ent;
  } catch (const chfsi::Error& e) {
    g_create_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return CHFSI_EINVAL;
  }
  return CHFSI_OK;
}

int chfsi_density(chfsi_ctx* c, const void* X, int64_t ldx, int n_vec, const double* occ, double* rho,
                  double* mag) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  check_block(c, X, ldx, n_vec, "X");
  CHFSI_CHECK(occ != nullptr, CHFSI_EINVAL, "occ_h is NULL");
  CHFSI_CHECK(rho && mag, CHFSI_EINVAL, "rho_d and mag_d must be non-NULL");
  for (int n = 0; n < n_vec; ++n)
    CHFSI_CHECK(std::isfinite(occ[n]), CHFSI_EINVAL, "occ_h holds a non-finite value");
  c->occ.upload(occ, (size_t)n_vec, c->stream);
  densities(c, (const double2*)X, ldx, n_vec, c->occ.ptr, rho, mag);
  API_END(c)
}

int chfsi_apply_H_backward(chfsi_ctx* c, int ik, const void* X, int64_t ldx, const void* Ybar, int64_t ldyb,
                           void* Xbar, int64_t ldxb, int n_vec, double* dV, double* dB) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  require_operator(c);
  check_block(c, X, ldx, n_vec, "X");
  check_block(c, Ybar, ldyb, n_vec, "Ybar");
  check_block(c, Xbar, ldxb, n_vec, "Xbar");
  CHFSI_CHECK(dV && dB, CHFSI_EINVAL, "dV_d and dB_d must be non-NULL");
  CHFSI_CHECK(Xbar != Ybar && Xbar != X, CHFSI_EINVAL, "Xbar must not alias X or Ybar");
  KPoint& kp = kpoint(c, ik);
  apply_H(c, kp, (const double2*)Ybar, ldyb, (double2*)Xbar, ldxb, n_vec, CHFSI_PREC_FP64, 1.0, 0.0, 0.0);
  cross_density(c, (const double2*)Ybar, ldyb, (const double2*)X, ldx, n_vec, 1.0, dV, dB);
  API_END(c)
}

static int filter_n_segments(int degree, int ck) { return (degree + ck - 1) / ck; }

size_t chfsi_filter_backward_workspace(const chfsi_ctx* c, int n_vec, int degree, int ck) {
  if (!c || n_vec < 1 || degree < 1 || ck < 1) return 0;
  const size_t blk = (size_t)2 * c->n_nodes * n_vec * sizeof(double2);
  return blk * (2 * (size_t)filter_n_segments(degree, ck) + std::max(ck, 3) + 2);
}

int chfsi_cheb_filter_backward(chfsi_ctx* c, int ik, const void* X, int64_t ldx, const void* Ybar, int64_t ldyb,
                               void* Xbar, int64_t ldxb, int n_vec, int degree, double a, double b, double a0,
                               int ck, void* work, size_t work_bytes, double* dV, double* dB) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  require_operator(c);
  check_block(c, X, ldx, n_vec, "X");
  check_block(c, Ybar, ldyb, n_vec, "Ybar");
  check_block(c, Xbar, ldxb, n_vec, "Xbar");
  CHFSI_CHECK(dV && dB && work, CHFSI_EINVAL, "dV_d, dB_d and work_d must be non-NULL");
  CHFSI_CHECK(degree >= 1 && ck >= 1, CHFSI_EINVAL, "degree and ckpt_every must be >= 1");
  CHFSI_CHECK(std::isfinite(a) && std::isfinite(b) && std::isfinite(a0) && a0 < a && a < b, CHFSI_EINVAL,
              "filter bounds must satisfy a0 < a < b");
  CHFSI_CHECK(work_bytes >= chfsi_filter_backward_workspace(c, n_vec, degree, ck), CHFSI_EINVAL,
              "workspace too small");
  KPoint& kp = kpoint(c, ik);
  const int m = degree;
  const int64_t rows = 2 * c->n_nodes;
  const size_t blk = (size_t)rows * n_vec;
  const int J = filter_n_segments(m, ck);
  const int nseg = std::max(ck, 3);
  double2* base = (double2*)work;
  auto ckp = [&](int j, int which) { return base + (2 * (size_t)j + which) * blk; };
  auto seg = [&](int i) { return base + (2 * (size_t)J + i) * blk; };
  double2* lam[2] = {base + (2 * (size_t)J + nseg) * blk, base + (2 * (size_t)J + nseg + 1) * blk};
  // recurrence coefficients: Y_k = al_k (H - c) Y_{k-1} + be_k Y_{k-2}, k = 1..m
  const double e = 0.5 * (b - a), cc = 0.5 * (b + a);
  const double s1 = e / (a0 - cc);
  std::vector<double> al(m + 2, 0.0), be(m + 2, 0.0);
  double sg = s1;
  al[1] = s1 / e;
  for (int k = 2; k <= m; ++k) {
    const double sn = 1.0 / (2.0 / s1 - sg);
    al[k] = 2.0 * sn / e;
    be[k] = -sg * sn;
    sg = sn;
  }
  // state k lives in checkpoint j = k / ck (slot 0 or 1) or in seg[k % ck]
  auto slot = [&](int k) -> double2* {
    const int j = k / ck, i = k % ck;
    return i < 2 ? ckp(j, i) : seg(i);
  };
  auto step = [&](int k) {            // computes state k (2 <= k) from k-1, k-2 into its slot
    apply_H2(c, kp, slot(k - 1), n_vec, slot(k), n_vec, slot(k - 2), n_vec, n_vec, CHFSI_PREC_FP64, al[k],
             be[k], -cc * al[k]);
  };
  // forward: checkpoint pairs (Y_{jc}, Y_{jc+1}) for states 0 .. m-1
  launch_copy_rows(c, slot(0), n_vec, (const double2*)X, ldx, rows, n_vec);
  if (m >= 2)
    apply_H(c, kp, slot(0), n_vec, slot(1), n_vec, n_vec, CHFSI_PREC_FP64, al[1], 0.0, -cc * al[1]);
  for (int k = 2; k <= m - 1; ++k) step(k);
  // backward
  launch_copy_rows(c, lam[0], n_vec, (const double2*)Ybar, ldyb, rows, n_vec);
  int cur = 0;                        // lam[cur] = Lam_k, lam[cur ^ 1] = Lam_{k+1}
  for (int j = J - 1; j >= 0; --j) {
    const int k_lo = j * ck;          // states k_lo .. k_hi-1 are needed as Y_{k-1}
    const int k_hi = std::min(k_lo + ck, m);
    for (int k = k_lo + 2; k <= k_hi - 1; ++k) step(k);   // recompute this segment
    for (int k = k_hi; k >= k_lo + 1; --k) {
      cross_density(c, lam[cur], n_vec, slot(k - 1), n_vec, n_vec, al[k], dV, dB);
      const double bn = (k < m) ? be[k + 1] : 0.0;
      apply_H(c, kp, lam[cur], n_vec, lam[cur ^ 1], n_vec, n_vec, CHFSI_PREC_FP64, al[k], bn, -cc * al[k]);
      cur ^= 1;
    }
  }
  launch_copy_rows(c, (double2*)Xbar, ldxb, lam[cur], n_vec, rows, n_vec);
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  API_END(c)
}

int chfsi_fill_random(chfsi_ctx* c, void* X, int64_t n_rows, int n_vec, int64_t ld, uint64_t seed, int64_t row0,
                      int col0, int64_t ntc) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  check_block(c, X, ld, n_vec, "X");
  CHFSI_CHECK(n_rows >= 0 && row0 >= 0 && col0 >= 0 && ntc >= col0 + n_vec, CHFSI_EINVAL, "bad fill extents");
  launch_fill_random(c, (double2*)X, n_rows, n_vec, ld, seed, row0, col0, ntc);
  API_END(c)
}

int chfsi_sync(chfsi_ctx* c) {
  if (!c) return CHFSI_EINVAL;
  API_BEGIN(c)
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  API_END(c)
}

}  // extern "C"
