// Host-side finite-element setup: 1-D rules and Lagrange tables, periodic mesh
// numbering, cell colouring, lumped GLL mass, the uniform reference-cell
// matrices, and the Bloch-phased pseudo-atom projector tables.
//
// Paper: Sec. III.A (eqn:FEWfns, eqn:FEHloc, eqn:CMat, eqn:OvlapMap,
// eqn:cellIntegrals), Sec. III.B.2 (diagonal M_D from GLL quadrature at the
// nodes), Sec. IV.B (cell-level matrices, restriction maps).
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <thread>

#include "internal.h"

namespace chfsi {

// ---------------------------------------------------------------- Legendre
// P_n(x) and P_{n-1}(x) by the three-term recurrence.
static void legendre_pair(int n, double x, double& pn, double& pnm1) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { pn = 1.0; pnm1 = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pnm1 = p0;
}

// Gauss-Legendre: roots of P_n, weights 2 / ((1 - x^2) P_n'(x)^2), with
// P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1).
void gl_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, pm;
      legendre_pair(n, t, pn, pm);
      double dp = n * (t * pn - pm) / (t * t - 1.0);
      double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double pn, pm;
    legendre_pair(n, t, pn, pm);
    double dp = n * (t * pn - pm) / (t * t - 1.0);
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// Gauss-Lobatto-Legendre: -1, +1 and the roots of P_p'.  Newton on P_p' with
// (1 - x^2) P_p'' = 2 x P_p' - p (p+1) P_p; weights 2 / (p (p+1) P_p(x)^2).
void gll_rule(int p, std::vector<double>& x, std::vector<double>& w) {
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double pn, pm;
      legendre_pair(p, t, pn, pm);
      double d1 = p * (t * pn - pm) / (t * t - 1.0);
      double d2 = (2.0 * t * d1 - p * (p + 1) * pn) / (1.0 - t * t);
      double dt = d1 / d2;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = t;
  }
  for (int i = 0; i <= p; ++i) {
    double pn, pm;
    legendre_pair(p, x[i], pn, pm);
    w[i] = 2.0 / (p * (p + 1) * pn * pn);
  }
}

// Barycentric Lagrange interpolation (Berrut and Trefethen 2004):
// l_j(t) = (b_j / (t - x_j)) / sum_k b_k / (t - x_k),  b_j = 1 / prod_{k != j} (x_j - x_k);
// l_j'(t) = l_j(t) sum_{k != j} 1 / (t - x_k) off the nodes; at node x_i the
// differentiation matrix D_ij = (b_j / b_i) / (x_i - x_j), D_ii = -sum_{j != i} D_ij.
void lagrange_on(const std::vector<double>& xn, const std::vector<double>& pts,
                 std::vector<double>& B, std::vector<double>& D) {
  const int n = (int)xn.size(), m = (int)pts.size();
  std::vector<double> bw(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) bw[j] /= (xn[j] - xn[k]);
  B.assign((size_t)n * m, 0.0);
  D.assign((size_t)n * m, 0.0);
  for (int q = 0; q < m; ++q) {
    const double t = pts[q];
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if (std::fabs(t - xn[j]) < 1e-14) hit = j;
    if (hit >= 0) {
      double diag = 0.0;
      for (int j = 0; j < n; ++j) {
        if (j == hit) continue;
        double dij = (bw[j] / bw[hit]) / (xn[hit] - xn[j]);
        D[(size_t)j * m + q] = dij;
        diag -= dij;
      }
      D[(size_t)hit * m + q] = diag;
      B[(size_t)hit * m + q] = 1.0;
      continue;
    }
    double den = 0.0;
    for (int k = 0; k < n; ++k) den += bw[k] / (t - xn[k]);
    for (int j = 0; j < n; ++j) {
      double lj = (bw[j] / (t - xn[j])) / den;
      double s = 0.0;
      for (int k = 0; k < n; ++k)
        if (k != j) s += 1.0 / (t - xn[k]);
      B[(size_t)j * m + q] = lj;
      D[(size_t)j * m + q] = lj * s;
    }
  }
}

RefElement make_ref(int p, int quad, int nq) {
  RefElement r;
  r.p = p;
  r.np1 = p + 1;
  gll_rule(p, r.xi, r.wgll);
  if (quad == CHFSI_QUAD_GLL) {
    r.xq = r.xi;
    r.wq = r.wgll;
  } else {
    gl_rule(nq, r.xq, r.wq);
  }
  r.nq = (int)r.xq.size();
  lagrange_on(r.xi, r.xq, r.B, r.D);
  return r;
}

// ---------------------------------------------------------------- mesh
// Colour of a cell coordinate along one periodic direction of n cells: two
// colours alternate; an odd count gives the last cell a third colour, so that
// cells sharing a node (including across the periodic wrap) never share a colour.
static int dir_colour(int c, int n) {
  if (n % 2 == 0) return c % 2;
  return (c == n - 1) ? 2 : c % 2;
}
static int dir_ncolours(int n) { return (n % 2 == 0) ? 2 : 3; }

void build_mesh(chfsi_ctx* c) {
  const int np1 = c->np1, p = c->p;
  c->nloc = np1 * np1 * np1;
  for (int d = 0; d < 3; ++d) {
    c->h[d] = c->box[d] / c->nc[d];
    c->Nd[d] = c->nc[d] * p;
  }
  c->J = c->h[0] * c->h[1] * c->h[2] / 8.0;
  c->n_nodes = (int64_t)c->Nd[0] * c->Nd[1] * c->Nd[2];
  c->n_cells = c->nc[0] * c->nc[1] * c->nc[2];
  c->nq3 = c->nq * c->nq * c->nq;
  // restriction maps: local node a = ax + np (ay + np az) of cell (cx, cy, cz)
  c->cell_nodes_h.resize((size_t)c->n_cells * c->nloc);
  for (int cz = 0; cz < c->nc[2]; ++cz)
    for (int cy = 0; cy < c->nc[1]; ++cy)
      for (int cx = 0; cx < c->nc[0]; ++cx) {
        const int e = cx + c->nc[0] * (cy + c->nc[1] * cz);
        for (int az = 0; az < np1; ++az)
          for (int ay = 0; ay < np1; ++ay)
            for (int ax = 0; ax < np1; ++ax) {
              int ix = (cx * p + ax) % c->Nd[0];
              int iy = (cy * p + ay) % c->Nd[1];
              int iz = (cz * p + az) % c->Nd[2];
              c->cell_nodes_h[(size_t)e * c->nloc + ax + np1 * (ay + np1 * az)] =
                  (int32_t)(ix + (int64_t)c->Nd[0] * (iy + (int64_t)c->Nd[1] * iz));
            }
      }
  // colouring for conflict-free scatter-add
  int nc3[3] = {dir_ncolours(c->nc[0]), dir_ncolours(c->nc[1]), dir_ncolours(c->nc[2])};
  c->n_colours = nc3[0] * nc3[1] * nc3[2];
  std::vector<std::vector<int32_t>> byc(c->n_colours);
  for (int e = 0; e < c->n_cells; ++e) {
    int cx = e % c->nc[0], cy = (e / c->nc[0]) % c->nc[1], cz = e / (c->nc[0] * c->nc[1]);
    int col = dir_colour(cx, c->nc[0]) +
              nc3[0] * (dir_colour(cy, c->nc[1]) + nc3[1] * dir_colour(cz, c->nc[2]));
    byc[col].push_back(e);
  }
  c->colour_off.assign(c->n_colours + 1, 0);
  std::vector<int32_t> order;
  for (int k = 0; k < c->n_colours; ++k) {
    c->colour_off[k + 1] = c->colour_off[k] + (int)byc[k].size();
    order.insert(order.end(), byc[k].begin(), byc[k].end());
  }
  // lumped GLL mass: M_I = sum_{cells containing I} w_ax w_ay w_az J
  std::vector<double> M(c->n_nodes, 0.0);
  const auto& w = c->ref.wgll;
  for (int e = 0; e < c->n_cells; ++e)
    for (int a = 0; a < c->nloc; ++a) {
      int ax = a % np1, ay = (a / np1) % np1, az = a / (np1 * np1);
      M[c->cell_nodes_h[(size_t)e * c->nloc + a]] += w[ax] * w[ay] * w[az] * c->J;
    }
  c->minv_sqrt_h.resize(c->n_nodes);
  for (int64_t i = 0; i < c->n_nodes; ++i) c->minv_sqrt_h[i] = 1.0 / std::sqrt(M[i]);
  c->nrb = (c->nloc + kRowBlk - 1) / kRowBlk;
  c->nkb = c->nrb * (kRowBlk / kKStep);
  c->cell_nodes.upload(c->cell_nodes_h.data(), c->cell_nodes_h.size(), c->stream);
  c->colour_cells.upload(order.data(), order.size(), c->stream);
  c->minv_sqrt.upload(c->minv_sqrt_h.data(), c->minv_sqrt_h.size(), c->stream);
}

// ---------------------------------------------------------------- uniform cell matrices
// With a tensor-product basis and a tensor quadrature rule every constant-
// coefficient cell matrix is a Kronecker product of 1-D matrices:
//   M1[a][b] = sum_q w_q l_a l_b,  S1[a][b] = sum_q w_q l_a' l_b',  G1[a][b] = sum_q w_q l_a l_b'
//   kinetic  K = (J/2) sum_d (2/h_d)^2 (S1 in direction d, M1 in the others)
//   mass     Mc = J M1 x M1 x M1
//   k-grad   C_d = J (2/h_d) (G1 in direction d, M1 in the others),  C = sum_d k_d C_d
// where C[i][j] = int N_i (k . grad N_j) (the k-term of eqn:FEHloc is -i C).
void build_uniform_mats(chfsi_ctx* c) {
  const auto& r = c->ref;
  const int n = r.np1, nq = r.nq, N = c->nloc;
  std::vector<double> M1(n * n, 0.0), S1(n * n, 0.0), G1(n * n, 0.0);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int q = 0; q < nq; ++q) {
        M1[a * n + b] += r.wq[q] * r.B[a * nq + q] * r.B[b * nq + q];
        S1[a * n + b] += r.wq[q] * r.D[a * nq + q] * r.D[b * nq + q];
        G1[a * n + b] += r.wq[q] * r.B[a * nq + q] * r.D[b * nq + q];
      }
  c->Kin.assign((size_t)N * N, 0.0);
  c->Mcons.assign((size_t)N * N, 0.0);
  for (int d = 0; d < 3; ++d) c->Cgrad[d].assign((size_t)N * N, 0.0);
  const double s[3] = {2.0 / c->h[0], 2.0 / c->h[1], 2.0 / c->h[2]};
  for (int i = 0; i < N; ++i) {
    int ia[3] = {i % n, (i / n) % n, i / (n * n)};
    for (int j = 0; j < N; ++j) {
      int ja[3] = {j % n, (j / n) % n, j / (n * n)};
      double m[3], st[3], g[3];
      for (int d = 0; d < 3; ++d) {
        m[d] = M1[ia[d] * n + ja[d]];
        st[d] = S1[ia[d] * n + ja[d]];
        g[d] = G1[ia[d] * n + ja[d]];
      }
      const size_t ij = (size_t)i * N + j;
      c->Kin[ij] = 0.5 * c->J *
                   (s[0] * s[0] * st[0] * m[1] * m[2] + s[1] * s[1] * m[0] * st[1] * m[2] +
                    s[2] * s[2] * m[0] * m[1] * st[2]);
      c->Mcons[ij] = c->J * m[0] * m[1] * m[2];
      c->Cgrad[0][ij] = c->J * s[0] * g[0] * m[1] * m[2];
      c->Cgrad[1][ij] = c->J * s[1] * m[0] * g[1] * m[2];
      c->Cgrad[2][ij] = c->J * s[2] * m[0] * m[1] * g[2];
    }
  }
}

// ---------------------------------------------------------------- angular momentum
// Real harmonics: l=1 in the (x, y, z) basis, where L_c x_a = sum_b (L_c)_{ba} x_b
// with (L_c)_{ba} = -i eps_{cba}.  For l=2 a quadratic harmonic is
// phi_T(r) = r^T T r with T symmetric traceless; L_c is a derivation, so
// L_c phi_T = phi_{T'} with T' = L1_c T + T L1_c^T, and the five real d
// harmonics correspond to the Frobenius-orthonormal tensors below (their
// sphere normalisations are all equal, so the matrix elements are the
// Frobenius products).
void angular_momentum_real(int l, std::vector<cplx>& L) {
  const int n = 2 * l + 1;
  L.assign((size_t)3 * n * n, cplx(0.0, 0.0));
  if (l == 0) return;
  // L1[c][b][a] = -i eps_{c b a}
  cplx L1[3][3][3];
  for (int cc = 0; cc < 3; ++cc)
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        int e = 0;
        if (cc != b && b != a && cc != a) e = ((b - cc + 3) % 3 == 1) ? 1 : -1;
        L1[cc][b][a] = cplx(0.0, -(double)e);
      }
  if (l == 1) {
    for (int cc = 0; cc < 3; ++cc)
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) L[((size_t)cc * 3 + b) * 3 + a] = L1[cc][b][a];
    return;
  }
  // l == 2: basis tensors xy, yz, 3z^2-r^2, xz, x^2-y^2
  double T[5][3][3] = {};
  const double r2 = 1.0 / std::sqrt(2.0), r6 = 1.0 / std::sqrt(6.0);
  T[0][0][1] = T[0][1][0] = r2;
  T[1][1][2] = T[1][2][1] = r2;
  T[2][2][2] = 2.0 * r6; T[2][0][0] = -r6; T[2][1][1] = -r6;
  T[3][0][2] = T[3][2][0] = r2;
  T[4][0][0] = r2; T[4][1][1] = -r2;
  for (int cc = 0; cc < 3; ++cc)
    for (int mp = 0; mp < 5; ++mp) {
      cplx Tp[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          cplx s(0.0, 0.0);
          for (int k = 0; k < 3; ++k) s += L1[cc][a][k] * T[mp][k][b] + T[mp][a][k] * L1[cc][b][k];
          Tp[a][b] = s;
        }
      for (int m = 0; m < 5; ++m) {
        cplx s(0.0, 0.0);
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) s += T[m][a][b] * Tp[a][b];
        L[((size_t)cc * 5 + m) * 5 + mp] = s;
      }
    }
}

// ---------------------------------------------------------------- projectors
// r^l Y_lm real harmonics (orthonormal on the sphere), same order as chfsi.h.
static int eval_harmonics(int lmax, double x, double y, double z, double* out) {
  int k = 0;
  out[k++] = 0.5 / std::sqrt(M_PI);
  if (lmax >= 1) {
    const double c1 = std::sqrt(3.0 / (4.0 * M_PI));
    out[k++] = c1 * x;
    out[k++] = c1 * y;
    out[k++] = c1 * z;
  }
  if (lmax >= 2) {
    const double c = 0.5 * std::sqrt(15.0 / M_PI);
    const double cz = 0.25 * std::sqrt(5.0 / M_PI);
    const double cx = 0.25 * std::sqrt(15.0 / M_PI);
    out[k++] = c * x * y;
    out[k++] = c * y * z;
    out[k++] = cz * (2.0 * z * z - x * x - y * y);
    out[k++] = c * x * z;
    out[k++] = cx * (x * x - y * y);
  }
  return k;
}

static const cplx kPauli[3][2][2] = {
    {{cplx(0, 0), cplx(1, 0)}, {cplx(1, 0), cplx(0, 0)}},
    {{cplx(0, 0), cplx(0, -1)}, {cplx(0, 1), cplx(0, 0)}},
    {{cplx(1, 0), cplx(0, 0)}, {cplx(0, 0), cplx(-1, 0)}}};

struct AtomWork {
  std::vector<int32_t> nodes;   // support nodes, sorted
  std::vector<cplx> P;          // [n_sup][n_pj] scaled projector values
  std::vector<cplx> delta;      // [2 n_pj]^2
  int n_pj = 0;
};

static void atom_tables(const chfsi_ctx* c, const double* k, const chfsi_atom_desc& at,
                        AtomWork& out) {
  const auto& r = c->ref;
  const int np1 = c->np1, nq = r.nq, nq3 = c->nq3, nloc = c->nloc;
  const int npj = (at.lmax + 1) * (at.lmax + 1);
  out.n_pj = npj;
  const double rc2 = at.rcut * at.rcut;
  int nimg[3];
  for (int d = 0; d < 3; ++d) nimg[d] = (int)std::ceil(at.rcut / c->box[d]) + 1;
  double cl[3];
  for (int l = 0; l <= at.lmax; ++l)
    cl[l] = std::sqrt(2.0 / (std::tgamma(l + 1.5) * std::pow(at.sigma, 2 * l + 3)));
  // support cells: cell box within rcut of some image of the atom
  std::vector<int> cells;
  for (int e = 0; e < c->n_cells; ++e) {
    int cc[3] = {e % c->nc[0], (e / c->nc[0]) % c->nc[1], e / (c->nc[0] * c->nc[1])};
    bool hit = false;
    for (int ix = -nimg[0]; ix <= nimg[0] && !hit; ++ix)
      for (int iy = -nimg[1]; iy <= nimg[1] && !hit; ++iy)
        for (int iz = -nimg[2]; iz <= nimg[2] && !hit; ++iz) {
          const int sh[3] = {ix, iy, iz};
          double d2 = 0.0;
          for (int d = 0; d < 3; ++d) {
            double R = at.pos[d] + sh[d] * c->box[d];
            double lo = cc[d] * c->h[d], hi = lo + c->h[d];
            double g = std::max(0.0, std::max(lo - R, R - hi));
            d2 += g * g;
          }
          hit = d2 < rc2;
        }
    if (hit) cells.push_back(e);
  }
  std::vector<int32_t> nodes;
  for (int e : cells)
    for (int a = 0; a < nloc; ++a) nodes.push_back(c->cell_nodes_h[(size_t)e * nloc + a]);
  std::sort(nodes.begin(), nodes.end());
  nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
  out.nodes = nodes;
  out.P.assign(nodes.size() * npj, cplx(0.0, 0.0));
  std::vector<cplx> F((size_t)nq3 * npj), T1((size_t)nq * nq * np1 * npj), T2((size_t)nq * np1 * np1 * npj);
  std::vector<double> hv(9);
  for (int e : cells) {
    int cc[3] = {e % c->nc[0], (e / c->nc[0]) % c->nc[1], e / (c->nc[0] * c->nc[1])};
    // F[q][chi] = w_q J beta_chi(r_q),  beta = sum_L exp(-i k.(r - L)) p(r - R - L)
    for (int q = 0; q < nq3; ++q) {
      int qa[3] = {q % nq, (q / nq) % nq, q / (nq * nq)};
      double rq[3];
      for (int d = 0; d < 3; ++d) rq[d] = cc[d] * c->h[d] + (r.xq[qa[d]] + 1.0) * 0.5 * c->h[d];
      const double wJ = r.wq[qa[0]] * r.wq[qa[1]] * r.wq[qa[2]] * c->J;
      cplx acc[9];
      for (int x = 0; x < npj; ++x) acc[x] = 0.0;
      for (int ix = -nimg[0]; ix <= nimg[0]; ++ix)
        for (int iy = -nimg[1]; iy <= nimg[1]; ++iy)
          for (int iz = -nimg[2]; iz <= nimg[2]; ++iz) {
            const double L[3] = {ix * c->box[0], iy * c->box[1], iz * c->box[2]};
            double dv[3], d2 = 0.0;
            for (int d = 0; d < 3; ++d) {
              dv[d] = rq[d] - at.pos[d] - L[d];
              d2 += dv[d] * dv[d];
            }
            if (d2 >= rc2) continue;
            const double g = std::exp(-d2 / (2.0 * at.sigma * at.sigma));
            eval_harmonics(at.lmax, dv[0], dv[1], dv[2], hv.data());
            const double ph = -(k[0] * (rq[0] - L[0]) + k[1] * (rq[1] - L[1]) + k[2] * (rq[2] - L[2]));
            const cplx phase(std::cos(ph), std::sin(ph));
            int x = 0;
            for (int l = 0; l <= at.lmax; ++l)
              for (int m = 0; m < 2 * l + 1; ++m, ++x) acc[x] += phase * (cl[l] * g * hv[x]);
          }
      for (int x = 0; x < npj; ++x) F[(size_t)q * npj + x] = wJ * acc[x];
    }
    // P_cell[a][chi] = sum_q N_a(q) F[q][chi] by sum factorisation over z, y, x
    std::fill(T1.begin(), T1.end(), cplx(0.0, 0.0));
    for (int qx = 0; qx < nq; ++qx)
      for (int qy = 0; qy < nq; ++qy)
        for (int az = 0; az < np1; ++az)
          for (int qz = 0; qz < nq; ++qz) {
            const double b = r.B[az * nq + qz];
            const cplx* f = &F[((size_t)qx + nq * (qy + nq * qz)) * npj];
            cplx* t = &T1[(((size_t)qx * nq + qy) * np1 + az) * npj];
            for (int x = 0; x < npj; ++x) t[x] += b * f[x];
          }
    std::fill(T2.begin(), T2.end(), cplx(0.0, 0.0));
    for (int qx = 0; qx < nq; ++qx)
      for (int ay = 0; ay < np1; ++ay)
        for (int qy = 0; qy < nq; ++qy) {
          const double b = r.B[ay * nq + qy];
          for (int az = 0; az < np1; ++az) {
            const cplx* t1 = &T1[(((size_t)qx * nq + qy) * np1 + az) * npj];
            cplx* t2 = &T2[(((size_t)qx * np1 + ay) * np1 + az) * npj];
            for (int x = 0; x < npj; ++x) t2[x] += b * t1[x];
          }
        }
    for (int a = 0; a < nloc; ++a) {
      int ax = a % np1, ay = (a / np1) % np1, az = a / (np1 * np1);
      const int32_t node = c->cell_nodes_h[(size_t)e * nloc + a];
      const size_t s = std::lower_bound(nodes.begin(), nodes.end(), node) - nodes.begin();
      for (int qx = 0; qx < nq; ++qx) {
        const double b = r.B[ax * nq + qx];
        const cplx* t2 = &T2[(((size_t)qx * np1 + ay) * np1 + az) * npj];
        for (int x = 0; x < npj; ++x) out.P[s * npj + x] += b * t2[x];
      }
    }
  }
  for (size_t s = 0; s < nodes.size(); ++s)
    for (int x = 0; x < npj; ++x) out.P[s * npj + x] *= c->minv_sqrt_h[nodes[s]];
  // Delta: D0_l within each shell + dso L.S (S = sigma/2), index 2 chi + alpha
  const int nd = 2 * npj;
  out.delta.assign((size_t)nd * nd, cplx(0.0, 0.0));
  if (at.delta_override) {
    for (int i = 0; i < nd * nd; ++i) out.delta[i] = cplx(at.delta_override[2 * i], at.delta_override[2 * i + 1]);
    return;
  }
  int off = 0;
  for (int l = 0; l <= at.lmax; ++l) {
    const int n = 2 * l + 1;
    std::vector<cplx> L;
    angular_momentum_real(l, L);
    for (int m = 0; m < n; ++m)
      for (int al = 0; al < 2; ++al) out.delta[(size_t)(2 * (off + m) + al) * nd + 2 * (off + m) + al] += at.d0[l];
    for (int cc = 0; cc < 3; ++cc)
      for (int m = 0; m < n; ++m)
        for (int mp = 0; mp < n; ++mp)
          for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be)
              out.delta[(size_t)(2 * (off + m) + al) * nd + 2 * (off + mp) + be] +=
                  at.dso * 0.5 * L[((size_t)cc * n + m) * n + mp] * kPauli[cc][al][be];
    off += n;
  }
}

template <class F>
static void parallel_for(int n, F f) {
  int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
  nt = std::min(nt, std::max(1, n));
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int i = t; i < n; i += nt) f(i);
    });
  for (auto& x : th) x.join();
}

void build_nonlocal(chfsi_ctx* c, KPoint& kp, int n_atoms, const chfsi_atom_desc* atoms) {
  NonlocalK& nl = kp.nl;
  nl.n_atoms = n_atoms;
  nl.atoms.assign(n_atoms, AtomTables{});
  nl.n_entries = 0;
  nl.max_pj = 1;
  nl.n_chunks = 0;
  nl.n_pairs = 0;
  nl.real_proj = false;
  if (n_atoms == 0) return;
  std::vector<AtomWork> work(n_atoms);
  parallel_for(n_atoms, [&](int a) { atom_tables(c, kp.k, atoms[a], work[a]); });
  for (int a = 0; a < n_atoms; ++a) nl.max_pj = std::max(nl.max_pj, work[a].n_pj);
  const int mp = nl.max_pj;
  std::vector<int32_t> atom_off(n_atoms + 1, 0), atom_npj(n_atoms);
  for (int a = 0; a < n_atoms; ++a) {
    atom_off[a + 1] = atom_off[a] + (int32_t)work[a].nodes.size();
    atom_npj[a] = work[a].n_pj;
    nl.atoms[a].n_pj = work[a].n_pj;
    nl.atoms[a].n_sup = (int)work[a].nodes.size();
    nl.atoms[a].node_off = atom_off[a];
    nl.atoms[a].delta = work[a].delta;
  }
  nl.n_entries = atom_off[n_atoms];
  nl.real_proj = true;
  for (int a = 0; a < n_atoms && nl.real_proj; ++a)
    for (const cplx& v : work[a].P)
      if (v.imag() != 0.0) {
        nl.real_proj = false;
        break;
      }
  std::vector<int32_t> sup(nl.n_entries);
  std::vector<double2> proj((size_t)nl.n_entries * mp, double2{0.0, 0.0});
  std::vector<float2> proj32((size_t)nl.n_entries * mp, float2{0.0f, 0.0f});
  std::vector<double2> delta((size_t)n_atoms * 4 * mp * mp, double2{0.0, 0.0});
  for (int a = 0; a < n_atoms; ++a) {
    const auto& w = work[a];
    for (size_t s = 0; s < w.nodes.size(); ++s) {
      sup[atom_off[a] + s] = w.nodes[s];
      for (int x = 0; x < w.n_pj; ++x) {
        cplx v = w.P[s * w.n_pj + x];
        proj[(atom_off[a] + s) * mp + x] = double2{v.real(), v.imag()};
        proj32[(atom_off[a] + s) * mp + x] = float2{(float)v.real(), (float)v.imag()};
      }
    }
    const int nd = 2 * w.n_pj;
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j) {
        cplx v = w.delta[(size_t)i * nd + j];
        delta[((size_t)a * 2 * mp + i) * 2 * mp + j] = double2{v.real(), v.imag()};
      }
  }
  // chunks for the reduction C = P^H X (support entries are sorted by node)
  std::vector<int32_t> ch_atom, ch_b, ch_e, ch_win, atom_chunk0(n_atoms + 1, 0);
  for (int a = 0; a < n_atoms; ++a) {
    atom_chunk0[a] = (int32_t)ch_atom.size();
    for (int s = atom_off[a]; s < atom_off[a + 1];) {
      const int win = sup[s] / kNlWindow;
      int e = s;
      while (e < atom_off[a + 1] && e - s < kNlChunk && sup[e] / kNlWindow == win) ++e;
      ch_atom.push_back(a);
      ch_b.push_back(s);
      ch_e.push_back(e);
      ch_win.push_back(win);
      s = e;
    }
  }
  atom_chunk0[n_atoms] = (int32_t)ch_atom.size();
  nl.n_chunks = (int)ch_atom.size();
  std::vector<int32_t> ch_order(nl.n_chunks);
  for (int i = 0; i < nl.n_chunks; ++i) ch_order[i] = i;
  std::stable_sort(ch_order.begin(), ch_order.end(), [&](int x, int y) {
    return ch_win[x] != ch_win[y] ? ch_win[x] < ch_win[y] : ch_atom[x] < ch_atom[y];
  });
  // run lists for the back-product (deterministic, no atomics)
  std::vector<std::array<int32_t, 3>> trip(nl.n_entries);
  for (int a = 0; a < n_atoms; ++a)
    for (int s = atom_off[a]; s < atom_off[a + 1]; ++s) trip[s] = {sup[s], a, s};
  std::sort(trip.begin(), trip.end());
  const int64_t n_runs = (c->n_nodes + kNlRun - 1) / kNlRun;
  std::vector<int32_t> run_off(n_runs + 1, 0), pair_atom, pair_ent;
  std::vector<int32_t> here;
  size_t t = 0;
  for (int64_t r = 0; r < n_runs; ++r) {
    run_off[r] = (int32_t)pair_atom.size();
    const int64_t node_end = std::min<int64_t>((r + 1) * kNlRun, c->n_nodes);
    here.clear();
    for (size_t u = t; u < trip.size() && trip[u][0] < node_end; ++u) here.push_back(trip[u][1]);
    std::sort(here.begin(), here.end());
    here.erase(std::unique(here.begin(), here.end()), here.end());
    const size_t base = pair_atom.size();
    pair_atom.insert(pair_atom.end(), here.begin(), here.end());
    pair_ent.resize(pair_atom.size() * kNlRun, -1);
    for (; t < trip.size() && trip[t][0] < node_end; ++t) {
      const size_t k = std::lower_bound(here.begin(), here.end(), trip[t][1]) - here.begin();
      pair_ent[(base + k) * kNlRun + (trip[t][0] - r * kNlRun)] = trip[t][2];
    }
  }
  run_off[n_runs] = (int32_t)pair_atom.size();
  nl.n_pairs = (int64_t)pair_atom.size();
  hipStream_t s = c->stream;
  nl.sup_node.upload(sup.data(), sup.size(), s);
  nl.proj.upload(proj.data(), proj.size(), s);
  nl.proj32.upload(proj32.data(), proj32.size(), s);
  nl.delta.upload(delta.data(), delta.size(), s);
  nl.atom_off.upload(atom_off.data(), atom_off.size(), s);
  nl.atom_npj.upload(atom_npj.data(), atom_npj.size(), s);
  nl.chunk_atom.upload(ch_atom.data(), ch_atom.size(), s);
  nl.chunk_begin.upload(ch_b.data(), ch_b.size(), s);
  nl.chunk_end.upload(ch_e.data(), ch_e.size(), s);
  nl.chunk_order.upload(ch_order.data(), ch_order.size(), s);
  nl.atom_chunk0.upload(atom_chunk0.data(), atom_chunk0.size(), s);
  nl.run_off.upload(run_off.data(), run_off.size(), s);
  nl.pair_atom.upload(pair_atom.data(), pair_atom.size(), s);
  nl.pair_ent.upload(pair_ent.data(), pair_ent.size(), s);
  CHFSI_HIP(hipStreamSynchronize(s));   // host vectors go out of scope
}

}  // namespace chfsi
