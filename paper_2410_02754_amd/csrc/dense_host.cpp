// Small dense Hermitian linear algebra on the host for the T x T projected
// problems of the Rayleigh-Ritz step and the Cholesky factor of the Gram
// matrix (Sec. III.B.2).  T <= a few thousand; O(T^3) textbook algorithms:
//  - Cholesky S = L L^H (lower, positive real diagonal),
//  - forward-substitution inverse of a lower-triangular matrix,
//  - Hermitian eigendecomposition: Householder reduction to a Hermitian
//    tridiagonal matrix (Golub and Van Loan, Sec. 8.3), a diagonal phase
//    change that makes it real, then the implicit QL iteration with shifts on
//    the real tridiagonal (Bowdler, Martin, Reinsch and Wilkinson, 1968),
//    accumulating the rotations, and back-transformation.
// All matrices are row-major std::vector<cplx> of size n*n.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

#include "internal.h"

namespace chfsi {

static int n_threads(size_t work) {
  int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (work < (size_t)1 << 16) return 1;
  return nt;
}

template <class F>
static void par_rows(int n, size_t work_per_row, F f) {
  int nt = n_threads((size_t)n * work_per_row);
  nt = std::min(nt, std::max(1, n));
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (int i = t; i < n; i += nt) f(i);
    });
  for (auto& x : th) x.join();
}

int cholesky_lower(std::vector<cplx>& S, int n) {
  // in place: lower triangle of S becomes L, upper triangle zeroed
  for (int j = 0; j < n; ++j) {
    double d = S[(size_t)j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(S[(size_t)j * n + k]);
    if (!(d > 0.0) || !std::isfinite(d)) return j;
    const double ljj = std::sqrt(d);
    S[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      cplx s = S[(size_t)i * n + j];
      const cplx* Li = &S[(size_t)i * n];
      const cplx* Lj = &S[(size_t)j * n];
      for (int k = 0; k < j; ++k) s -= Li[k] * std::conj(Lj[k]);
      S[(size_t)i * n + j] = s / ljj;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) S[(size_t)i * n + j] = 0.0;
  return -1;
}

void lower_inverse(const std::vector<cplx>& L, int n, std::vector<cplx>& X) {
  X.assign((size_t)n * n, cplx(0.0, 0.0));
  // column j of X solves L x = e_j; columns are independent
  std::vector<std::vector<cplx>> cols(n);
  par_rows(n, (size_t)n * n / 2, [&](int j) {
    std::vector<cplx> x(n, 0.0);
    x[j] = 1.0 / L[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      cplx s = 0.0;
      const cplx* Li = &L[(size_t)i * n];
      for (int k = j; k < i; ++k) s += Li[k] * x[k];
      x[i] = -s / L[(size_t)i * n + i];
    }
    cols[j].swap(x);
  });
  for (int j = 0; j < n; ++j)
    for (int i = j; i < n; ++i) X[(size_t)i * n + j] = cols[j][i];
}

// Implicit QL on the real symmetric tridiagonal (d, e), e[i] couples i, i+1.
// Zt[i][:] accumulates eigenvector i (rows), starting from the identity.
static void tridiag_ql(std::vector<double>& d, std::vector<double>& e, std::vector<double>* Zt, int n) {
  if (n == 0) return;
  e.resize(n);
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    while (true) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == l) break;
      if (++iter > 200) break;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = m - 1;
      bool deflated = false;
      for (; i >= l; --i) {
        double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        if (Zt) {
          double* zi = &(*Zt)[(size_t)i * n];
          double* zj = &(*Zt)[(size_t)(i + 1) * n];
          for (int k = 0; k < n; ++k) {
            const double t = zj[k];
            zj[k] = s * zi[k] + c * t;
            zi[k] = c * zi[k] - s * t;
          }
        }
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
}

void hermitian_eig(const std::vector<cplx>& Ain, int n, std::vector<double>& w, std::vector<cplx>& V) {
  std::vector<cplx> A = Ain;
  // use the lower triangle; make A exactly Hermitian from it
  for (int i = 0; i < n; ++i) {
    A[(size_t)i * n + i] = A[(size_t)i * n + i].real();
    for (int j = 0; j < i; ++j) A[(size_t)j * n + i] = std::conj(A[(size_t)i * n + j]);
  }
  std::vector<std::vector<cplx>> vs(std::max(0, n - 2));
  std::vector<cplx> offd(std::max(0, n - 1), 0.0);
  std::vector<cplx> p(n), q(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;         // size of the trailing block
    std::vector<cplx> v(m);
    double xn2 = 0.0;
    for (int i = 0; i < m; ++i) {
      v[i] = A[(size_t)(k + 1 + i) * n + k];
      xn2 += std::norm(v[i]);
    }
    const double xn = std::sqrt(xn2);
    if (xn == 0.0) {
      offd[k] = 0.0;
      continue;
    }
    const cplx phase = (std::abs(v[0]) > 0.0) ? v[0] / std::abs(v[0]) : cplx(1.0, 0.0);
    const cplx alpha = -phase * xn;
    v[0] -= alpha;
    double vn = 0.0;
    for (int i = 0; i < m; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    for (int i = 0; i < m; ++i) v[i] /= vn;
    // p = A_sub v ; rho = v^H p ; q = p - rho v ; A_sub -= 2 (v q^H + q v^H)
    par_rows(m, (size_t)m, [&](int i) {
      cplx s = 0.0;
      const cplx* Ai = &A[(size_t)(k + 1 + i) * n + k + 1];
      for (int j = 0; j < m; ++j) s += Ai[j] * v[j];
      p[i] = s;
    });
    cplx rho = 0.0;
    for (int i = 0; i < m; ++i) rho += std::conj(v[i]) * p[i];
    for (int i = 0; i < m; ++i) q[i] = p[i] - rho.real() * v[i];
    par_rows(m, (size_t)m, [&](int i) {
      cplx* Ai = &A[(size_t)(k + 1 + i) * n + k + 1];
      const cplx vi = v[i], qi = q[i];
      for (int j = 0; j < m; ++j) Ai[j] -= 2.0 * (vi * std::conj(q[j]) + qi * std::conj(v[j]));
    });
    offd[k] = alpha;
    for (int i = 1; i < m; ++i) {
      A[(size_t)(k + 1 + i) * n + k] = 0.0;
      A[(size_t)k * n + k + 1 + i] = 0.0;
    }
    A[(size_t)(k + 1) * n + k] = alpha;
    A[(size_t)k * n + k + 1] = std::conj(alpha);
    vs[k].swap(v);
  }
  if (n >= 2) offd[n - 2] = A[(size_t)(n - 1) * n + n - 2];
  std::vector<double> d(n), e(std::max(1, n));
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i].real();
  // phases phi_0 = 1, phi_{k+1} = phi_k e_k / |e_k| make the tridiagonal real
  std::vector<cplx> phi(n, 1.0);
  for (int k = 0; k + 1 < n; ++k) {
    const double a = std::abs(offd[k]);
    e[k] = a;
    phi[k + 1] = (a > 0.0) ? phi[k] * offd[k] / a : phi[k];
  }
  std::vector<double> Zt((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
  tridiag_ql(d, e, &Zt, n);
  // sort ascending
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
  w.resize(n);
  // V[:, j] = Q (phi .* z_order[j]); build Y = D Z column-sorted, then apply Q
  V.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    w[j] = d[order[j]];
    const double* z = &Zt[(size_t)order[j] * n];
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = phi[i] * z[i];
  }
  // Q = H_0 H_1 ... H_{n-3}; apply in reverse to the rows k+1.. of V
  for (int k = n - 3; k >= 0; --k) {
    const auto& v = vs[k];
    if (v.empty()) continue;
    const int m = n - k - 1;
    std::vector<cplx> t(n, 0.0);     // t = v^H V_sub
    for (int i = 0; i < m; ++i) {
      const cplx cv = std::conj(v[i]);
      const cplx* Vi = &V[(size_t)(k + 1 + i) * n];
      for (int j = 0; j < n; ++j) t[j] += cv * Vi[j];
    }
    par_rows(m, (size_t)n, [&](int i) {
      cplx* Vi = &V[(size_t)(k + 1 + i) * n];
      const cplx vi = 2.0 * v[i];
      for (int j = 0; j < n; ++j) Vi[j] -= vi * t[j];
    });
  }
}

void tridiag_eigvals(std::vector<double> d, std::vector<double> e, std::vector<double>& w) {
  const int n = (int)d.size();
  tridiag_ql(d, e, nullptr, n);
  std::sort(d.begin(), d.end());
  w = d;
}

}  // namespace chfsi
