// Small dense Hermitian linear algebra on the host for the T x T projected
// problems of the Rayleigh-Ritz step and the Cholesky factor of the Gram
// matrix (Sec. III.B.2).  T <= a few thousand; O(T^3) textbook algorithms:
//  - Cholesky S = L L^H (lower, positive real diagonal),
//  - forward-substitution inverse of a lower-triangular matrix,
//  - Hermitian eigendecomposition: Householder reduction to a Hermitian
//    tridiagonal matrix (Golub and Van Loan, Sec. 8.3), a diagonal phase
//    change that makes it real, then the implicit QL iteration with shifts on
//    the real tridiagonal (Bowdler, Martin, Reinsch and Wilkinson, 1968),
//    accumulating the rotations, and back-transformation by blocks of
//    reflectors in the compact WY form I - Y T Y^H (Schreiber and Van Loan,
//    1989).
// All matrices are row-major std::vector<cplx> of size n*n.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <functional>
#include <numeric>
#include <thread>

#include "internal.h"

namespace chfsi {

// Fixed set of worker threads for the O(n^3) loops below.  run(f) calls f(t, nt)
// on every worker t (the caller is worker 0) and returns when all are done; the
// workers spin briefly, then yield, between calls, so the many short parallel
// phases of one factorisation pay no thread start-up.
class Pool {
 public:
  explicit Pool(size_t work) {
    nt_ = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (work < ((size_t)1 << 16)) nt_ = 1;
    for (int t = 1; t < nt_; ++t) th_.emplace_back([this, t]() { loop(t); });
  }
  ~Pool() {
    stop_.store(true);
    gen_.fetch_add(1);
    for (auto& x : th_) x.join();
  }
  int size() const { return nt_; }
  void run(const std::function<void(int, int)>& f) {
    if (nt_ == 1) {
      f(0, 1);
      return;
    }
    f_ = &f;
    done_.store(0);
    gen_.fetch_add(1, std::memory_order_release);
    f(0, nt_);
    for (int spin = 0; done_.load(std::memory_order_acquire) != nt_ - 1; ++spin)
      if (spin > 4096) std::this_thread::yield();
  }
  // [lo, hi) share of n items for worker t of nt
  static void range(int n, int t, int nt, int& lo, int& hi) {
    lo = (int)((int64_t)n * t / nt);
    hi = (int)((int64_t)n * (t + 1) / nt);
  }

 private:
  void loop(int t) {
    unsigned seen = 0;
    while (true) {
      unsigned g;
      for (int spin = 0; (g = gen_.load(std::memory_order_acquire)) == seen; ++spin)
        if (spin > 4096) std::this_thread::yield();
      seen = g;
      if (stop_.load()) return;
      (*f_)(t, nt_);
      done_.fetch_add(1, std::memory_order_acq_rel);
    }
  }
  int nt_ = 1;
  std::vector<std::thread> th_;
  std::atomic<unsigned> gen_{0};
  std::atomic<int> done_{0};
  std::atomic<bool> stop_{false};
  const std::function<void(int, int)>* f_ = nullptr;
};

int cholesky_lower(std::vector<cplx>& S, int n) {
  // in place, left-looking by rows of columns: lower triangle of S becomes L,
  // upper triangle zeroed; the updates of the rows below column j run in parallel
  Pool pool((size_t)n * n * n / 3);
  for (int j = 0; j < n; ++j) {
    double d = S[(size_t)j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(S[(size_t)j * n + k]);
    if (!(d > 0.0) || !std::isfinite(d)) return j;
    const double ljj = std::sqrt(d);
    S[(size_t)j * n + j] = ljj;
    const int rows = n - j - 1;
    auto body = [&](int t, int nt) {
      int lo, hi;
      Pool::range(rows, t, nt, lo, hi);
      const cplx* Lj = &S[(size_t)j * n];
      for (int i = j + 1 + lo; i < j + 1 + hi; ++i) {
        cplx s = S[(size_t)i * n + j];
        const cplx* Li = &S[(size_t)i * n];
        for (int k = 0; k < j; ++k) s -= Li[k] * std::conj(Lj[k]);
        S[(size_t)i * n + j] = s / ljj;
      }
    };
    if ((size_t)rows * j > 4096) pool.run(body);
    else body(0, 1);
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) S[(size_t)i * n + j] = 0.0;
  return -1;
}

void lower_inverse(const std::vector<cplx>& L, int n, std::vector<cplx>& X) {
  X.assign((size_t)n * n, cplx(0.0, 0.0));
  // column j of X solves L x = e_j; columns are independent (interleaved over
  // the workers, since column j costs ~(n - j)^2)
  Pool pool((size_t)n * n * n / 6);
  pool.run([&](int t, int nt) {
    std::vector<cplx> x(n);
    for (int j = t; j < n; j += nt) {
      x[j] = 1.0 / L[(size_t)j * n + j];
      for (int i = j + 1; i < n; ++i) {
        cplx s = 0.0;
        const cplx* Li = &L[(size_t)i * n];
        for (int k = j; k < i; ++k) s += Li[k] * x[k];
        x[i] = -s / L[(size_t)i * n + i];
      }
      for (int i = j; i < n; ++i) X[(size_t)i * n + j] = x[i];
    }
  });
}

// Implicit QL on the real symmetric tridiagonal (d, e), e[i] couples i, i+1.
// Zt[i][:] accumulates eigenvector i (rows), starting from the identity.  The
// rotations only act on Zt, so they are recorded in order and applied after the
// iteration, each worker applying all of them to its own range of columns.  One
// QL step is a chain of rotations of rows (i, i+1), i = m-1 down to l; along the
// chain the updated row i is the next rotation's row i+1, so it stays in
// registers ("carry") and each rotation costs one row load and one row store.
static void tridiag_ql(std::vector<double>& d, std::vector<double>& e, std::vector<double>* Zt, int n,
                       Pool* pool) {
  if (n == 0) return;
  e.resize(n);
  e[n - 1] = 0.0;
  std::vector<int> ch_m, ch_len;           // chain: rotations of rows (i, i+1), i = m-1 .. m-len
  std::vector<double> rc, rs;
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
      const size_t first = rc.size();
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
          rc.push_back(c);
          rs.push_back(s);
        }
      }
      if (Zt && rc.size() > first) {
        ch_m.push_back(m);
        ch_len.push_back((int)(rc.size() - first));
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  if (!Zt || rc.empty()) return;
  auto body = [&](int t, int nt) {
    int lo, hi;
    Pool::range(n, t, nt, lo, hi);
    double* Z = Zt->data();
    constexpr int B = 8;
    for (int k0 = lo; k0 < hi; k0 += B) {
      const int w = std::min(B, hi - k0);
      size_t q = 0;
      for (size_t ch = 0; ch < ch_m.size(); ++ch) {
        const int m = ch_m[ch], len = ch_len[ch];
        double carry[B];
        const double* zm = Z + (size_t)m * n + k0;
        for (int u = 0; u < B; ++u) carry[u] = u < w ? zm[u] : 0.0;
        for (int r = 0; r < len; ++r, ++q) {
          const int i = m - 1 - r;
          double* __restrict__ zi = Z + (size_t)i * n + k0;
          double* __restrict__ zj = zi + n;
          const double c = rc[q], s = rs[q];
          if (w == B) {
            for (int u = 0; u < B; ++u) {
              const double a = zi[u];
              zj[u] = s * a + c * carry[u];
              carry[u] = c * a - s * carry[u];
            }
          } else {
            for (int u = 0; u < w; ++u) {
              const double a = zi[u];
              zj[u] = s * a + c * carry[u];
              carry[u] = c * a - s * carry[u];
            }
          }
        }
        double* zl = Z + (size_t)(m - len) * n + k0;
        for (int u = 0; u < w; ++u) zl[u] = carry[u];
      }
    }
  };
  if (pool) pool->run(body);
  else body(0, 1);
}

void hermitian_eig(const std::vector<cplx>& Ain, int n, std::vector<double>& w, std::vector<cplx>& V) {
  Pool pool((size_t)n * n * n);
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
    const bool par = (size_t)m * m > 8192;
    auto matvec = [&](int t, int nt) {
      int lo, hi;
      Pool::range(m, t, nt, lo, hi);
      const double* vv = reinterpret_cast<const double*>(v.data());
      for (int i = lo; i < hi; ++i) {
        const double* Ai = reinterpret_cast<const double*>(&A[(size_t)(k + 1 + i) * n + k + 1]);
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < m; ++j) {
          sr += Ai[2 * j] * vv[2 * j] - Ai[2 * j + 1] * vv[2 * j + 1];
          si += Ai[2 * j] * vv[2 * j + 1] + Ai[2 * j + 1] * vv[2 * j];
        }
        p[i] = cplx(sr, si);
      }
    };
    if (par) pool.run(matvec);
    else matvec(0, 1);
    cplx rho = 0.0;
    for (int i = 0; i < m; ++i) rho += std::conj(v[i]) * p[i];
    for (int i = 0; i < m; ++i) q[i] = p[i] - rho.real() * v[i];
    auto update = [&](int t, int nt) {
      int lo, hi;
      Pool::range(m, t, nt, lo, hi);
      const double* vv = reinterpret_cast<const double*>(v.data());
      const double* qq = reinterpret_cast<const double*>(q.data());
      for (int i = lo; i < hi; ++i) {
        double* Ai = reinterpret_cast<double*>(&A[(size_t)(k + 1 + i) * n + k + 1]);
        const double vr = 2.0 * v[i].real(), vim = 2.0 * v[i].imag();
        const double qr = 2.0 * q[i].real(), qim = 2.0 * q[i].imag();
        for (int j = 0; j < m; ++j) {
          // vi conj(q_j) + qi conj(v_j)
          const double ar = vr * qq[2 * j] + vim * qq[2 * j + 1] + qr * vv[2 * j] + qim * vv[2 * j + 1];
          const double ai = vim * qq[2 * j] - vr * qq[2 * j + 1] + qim * vv[2 * j] - qr * vv[2 * j + 1];
          Ai[2 * j] -= ar;
          Ai[2 * j + 1] -= ai;
        }
      }
    };
    if (par) pool.run(update);
    else update(0, 1);
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
  tridiag_ql(d, e, &Zt, n, &pool);
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
  // Q = H_0 H_1 ... H_{n-3} applied to V, H_k = I - 2 v_k v_k^H (v_k unit, nonzero
  // from row k+1).  The reflectors go in blocks of kWY consecutive ones, each block
  // H_k1 ... H_k2 = I - Y T Y^H (compact WY form: Y = [v_k1 .. v_k2], T upper
  // triangular, T_ii = 2, T[0:i, i] = -2 T[0:i, 0:i] (Y[:, 0:i]^H v_i)), applied as
  // V_sub -= Y (T (Y^H V_sub)), last block first; each worker takes its own range of
  // columns (the columns are independent).
  constexpr int kWY = 32;
  const int nref = std::max(0, n - 2);
  struct Blk {
    int k1, k2;                 // reflectors k1..k2
    std::vector<cplx> Y;        // [m1][nb], rows k1+1 .. n-1 (zero above each v's start)
    std::vector<cplx> T;        // [nb][nb] upper
  };
  std::vector<Blk> blks;
  for (int k1 = 0; k1 < nref; k1 += kWY) {
    Blk B;
    B.k1 = k1;
    B.k2 = std::min(nref, k1 + kWY) - 1;
    const int nb = B.k2 - B.k1 + 1, m1 = n - k1 - 1;
    B.Y.assign((size_t)m1 * nb, 0.0);
    for (int j = 0; j < nb; ++j) {
      const auto& v = vs[k1 + j];
      if (v.empty()) continue;
      for (size_t i = 0; i < v.size(); ++i) B.Y[(size_t)(j + i) * nb + j] = v[i];   // v_k starts at row k+1
    }
    B.T.assign((size_t)nb * nb, 0.0);
    std::vector<cplx> g(nb);
    for (int i = 0; i < nb; ++i) {
      if (vs[k1 + i].empty()) continue;      // H = I: zero column of Y, T_ii = 0
      // g[0:i] = Y[:, 0:i]^H v_i
      for (int j = 0; j < i; ++j) {
        cplx acc = 0.0;
        for (int r = i; r < m1; ++r) acc += std::conj(B.Y[(size_t)r * nb + j]) * B.Y[(size_t)r * nb + i];
        g[j] = acc;
      }
      for (int j = 0; j < i; ++j) {
        cplx acc = 0.0;
        for (int l = j; l < i; ++l) acc += B.T[(size_t)j * nb + l] * g[l];
        B.T[(size_t)j * nb + i] = -2.0 * acc;
      }
      B.T[(size_t)i * nb + i] = 2.0;
    }
    blks.push_back(std::move(B));
  }
  pool.run([&](int t, int nt) {
    int lo, hi;
    Pool::range(n, t, nt, lo, hi);
    if (lo >= hi) return;
    const int w = hi - lo, w2 = 2 * w;
    std::vector<double> W((size_t)kWY * w2), W2((size_t)kWY * w2);
    for (int bi = (int)blks.size() - 1; bi >= 0; --bi) {
      const Blk& B = blks[bi];
      const int nb = B.k2 - B.k1 + 1, m1 = n - B.k1 - 1, r0 = B.k1 + 1;
      // W = Y^H V_sub (interleaved re, im)
      std::fill(W.begin(), W.begin() + (size_t)nb * w2, 0.0);
      for (int r = 0; r < m1; ++r) {
        const double* __restrict__ Vr = reinterpret_cast<const double*>(&V[(size_t)(r0 + r) * n + lo]);
        const cplx* Yr = &B.Y[(size_t)r * nb];
        const int jmax = std::min(nb, r + 1);      // v_{k1+j} starts at row j of the block
        for (int j = 0; j < jmax; ++j) {
          const double yr = Yr[j].real(), yi = -Yr[j].imag();
          double* __restrict__ Wj = &W[(size_t)j * w2];
          for (int c = 0; c < w2; c += 2) {
            Wj[c] += yr * Vr[c] - yi * Vr[c + 1];
            Wj[c + 1] += yr * Vr[c + 1] + yi * Vr[c];
          }
        }
      }
      // W2 = T W
      for (int j = 0; j < nb; ++j) {
        double* __restrict__ W2j = &W2[(size_t)j * w2];
        std::fill(W2j, W2j + w2, 0.0);
        for (int l = j; l < nb; ++l) {
          const double tr = B.T[(size_t)j * nb + l].real(), ti = B.T[(size_t)j * nb + l].imag();
          const double* __restrict__ Wl = &W[(size_t)l * w2];
          for (int c = 0; c < w2; c += 2) {
            W2j[c] += tr * Wl[c] - ti * Wl[c + 1];
            W2j[c + 1] += tr * Wl[c + 1] + ti * Wl[c];
          }
        }
      }
      // V_sub -= Y W2
      for (int r = 0; r < m1; ++r) {
        double* __restrict__ Vr = reinterpret_cast<double*>(&V[(size_t)(r0 + r) * n + lo]);
        const cplx* Yr = &B.Y[(size_t)r * nb];
        const int jmax = std::min(nb, r + 1);
        for (int j = 0; j < jmax; ++j) {
          const double yr = Yr[j].real(), yi = Yr[j].imag();
          const double* __restrict__ W2j = &W2[(size_t)j * w2];
          for (int c = 0; c < w2; c += 2) {
            Vr[c] -= yr * W2j[c] - yi * W2j[c + 1];
            Vr[c + 1] -= yr * W2j[c + 1] + yi * W2j[c];
          }
        }
      }
    }
  });
}

void tridiag_eigvals(std::vector<double> d, std::vector<double> e, std::vector<double>& w) {
  const int n = (int)d.size();
  tridiag_ql(d, e, nullptr, n, nullptr);
  std::sort(d.begin(), d.end());
  w = d;
}

}  // namespace chfsi
