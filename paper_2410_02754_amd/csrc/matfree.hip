// Matrix-free local part of H_hat: the tensor-structured multivector product
// that the paper names as future work (Sec. VI), for 2-component spinors.
//
// Per cell e and column n the product of the cell operator of eqn:FEHlocEl with
// the gathered, M_D^{-1/2}-scaled spinor u = (u_up, u_dn) is evaluated without
// forming the cell matrix:
//   1. U = (B (x) B (x) B)^T u        values at the quadrature points (3 passes)
//   2. W = w_q J [(V + |k|^2/2) U + (B_xc . sigma) U]          pointwise
//   3. for each direction d: G_d = D_d U (collocation derivative along d),
//        W += D_d^T (w_q J G_d / 2) - i k_d w_q J G_d              (2 passes each)
//   4. y = (B (x) B (x) B) W            back to the nodes (3 passes)
// and y, scaled by M_D^{-1/2}, is added into the output rows of the cell's nodes.
// B[a][q] = l_a(x_q) is the 1-D GLL-node Lagrange basis at the quadrature points
// and D_d = (2/h_d) Dq with Dq[q][r] = l~_r'(x_q) the derivative of the Lagrange
// basis on the quadrature points.  With n_q = p + 1 points per direction both
// are exact for the degree-p fields of the cell, so the result equals the
// product with the assembled cell matrices (kinetic K, mass, k-gradient C,
// potential and field matrices) up to rounding: same quadrature, different
// order of summation.  Work per cell and column is 12 line contractions of
// n_p^4 complex-by-real multiply-adds per spin, against 4 (2 n_p^3)^2 for the
// dense cell product, and no cell matrices are stored.
//
// FP64, or FP32 (mixed precision: tables, quadrature data, LDS fields and
// arithmetic in FP32, rows converted on gather and added into the FP64 output).
//
// Launch: one workgroup of 256 (FP64) or 512 (FP32) threads per (cell of one
// colour, chunk of CW columns).  Both spins of CW columns live in two LDS buffers of n_p^3 complex
// values per field; each thread owns one line (along the pass direction) of
// one (column, spin) field, keeps it in registers and writes the contracted
// line, so every LDS value read feeds n_p multiply-adds.  Within a colour no
// two cells share a node, so the scatter is a plain read-add-write.
#include <functional>

#include "mfma.h"
#include "sumfact.h"

namespace chfsi {

namespace {

template <class T> struct MfT;
template <> struct MfT<double> {
  typedef double2 C2;
  typedef double4 Q4;
  static constexpr int NT = 256;
};
template <> struct MfT<float> {
  typedef float2 C2;
  typedef float4 Q4;
  static constexpr int NT = 512;
};
// columns per workgroup: the same LDS bytes in both precisions
template <class T>
constexpr int mf_cw(int NP) { return sizeof(T) == 8 ? sf_cols(NP) : 2 * sf_cols(NP); }

// Kinetic and k-gradient terms along DIM, added into W:
//   G = Dq U,  W += a_d Dq^T (wJ G) - i b_d wJ G,
// a_d = (2/h_d)^2 / 2, b_d = k_d (2/h_d), wJ = J w_x w_y w_z at each point.
// BWD: W along the line is then complete (the other directions ran before), so
// the backward interpolation along DIM (W -> B W) is applied in place.
// eo: even-odd tables of Dq (G = Dq U), Dq^T (the transposed contraction) and
// B^T (points -> nodes), see sf_eo.
// In FP32 the kinetic weights a_d wJ come per point from kin (formed in FP64 and
// rounded once): products of the shared 1-D weights rounded in FP32 would bias
// the operator the same way in every cell.
template <class T, int NP, int CW, int DIM, bool KT, bool BWD>
__device__ __forceinline__ void grad_pass(const T* __restrict__ eoDf, const T* __restrict__ eoDb,
                                          const T* __restrict__ eoBb, const T* __restrict__ w1, T J, T a_d, T b_d,
                                          const T* __restrict__ kin, const typename MfT<T>::C2* __restrict__ U,
                                          typename MfT<T>::C2* __restrict__ W) {
  typedef typename MfT<T>::C2 C2;
  constexpr int NT = MfT<T>::NT;
  constexpr int N2 = NP * NP, N3 = N2 * NP;
  constexpr int S = DIM == 0 ? 1 : DIM == 1 ? NP : N2;
  for (int t = threadIdx.x; t < N2 * 2 * CW; t += NT) {
    const int l = t % N2, f = t / N2;
    const int lb = sf_line_base<NP, DIM>(l);
    const int base = f * N3 + lb;
    // the two coordinates held fixed along the line are l % NP and l / NP
    const T wl = J * w1[l % NP] * w1[l / NP];
    T kw[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) kw[q] = (sizeof(T) == 4) ? kin[lb + q * S] : a_d * wl * w1[q];
    C2 u[NP], g[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) u[j] = U[base + j * S];
    sf_eo<T, NP, true>(eoDf, u, g);
    C2 fk[NP], dw[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) fk[q] = C2{kw[q] * g[q].x, kw[q] * g[q].y};
    sf_eo<T, NP, true>(eoDb, fk, dw);
    C2 wv[NP];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      C2 acc = W[base + r * S];
      acc.x += dw[r].x;
      acc.y += dw[r].y;
      if constexpr (KT) {
        // -i b wJ g = b wJ g.y - i b wJ g.x
        const T s = b_d * wl * w1[r];
        acc.x = fma(s, g[r].y, acc.x);
        acc.y = fma(-s, g[r].x, acc.y);
      }
      wv[r] = acc;
    }
    if constexpr (BWD) {
      C2 o[NP];
      sf_eo<T, NP, false>(eoBb, wv, o);
#pragma unroll
      for (int r = 0; r < NP; ++r) W[base + r * S] = o[r];
    } else {
#pragma unroll
      for (int r = 0; r < NP; ++r) W[base + r * S] = wv[r];
    }
  }
}

// tab: [B: NP*NP][Dq: NP*NP][w: NP][even-odd tables of B, B^T, Dq, Dq^T], qd:
// [E][NP^3] of (wJ V, wJ Bx, wJ By, wJ Bz), both in the arithmetic type T.
//
// One workgroup per work item (cell of the colour, chunk of CW columns); items
// are cell major and consecutive items run on one XCD (workgroup b on XCD b % 8),
// so the column chunks of a cell share its rows in that XCD's L2.  Each thread
// owns at most one (column, spin, z-line) task of the first and last phases
// (2 CW n_p^2 <= NT for every n_p) and issues all of that task's global loads
// before it uses any of them.
template <class T, int NP, bool KT>
__global__ __launch_bounds__(MfT<T>::NT) void mf_apply_kernel(
    const T* __restrict__ tab, const typename MfT<T>::Q4* __restrict__ qd, const int32_t* __restrict__ cell_nodes,
    const int32_t* __restrict__ cells, int total, int n_chunks, const double* __restrict__ minv_sqrt,
    const double2* __restrict__ X, int64_t ldx, double2* __restrict__ Y, int64_t ldy, int n_vec, double alpha,
    T J, T half_k2, T a0, T a1, T a2, T b0, T b1, T b2, const T* __restrict__ kin,
    const double* __restrict__ alpha_d) {
  typedef typename MfT<T>::C2 C2;
  typedef typename MfT<T>::Q4 Q4;
  constexpr int NT = MfT<T>::NT;
  constexpr int CW = mf_cw<T>(NP);
  constexpr int N2 = NP * NP, N3 = N2 * NP;
  static_assert(2 * CW * N2 <= NT, "one edge task per thread");
  extern __shared__ double2 mf_sm_raw[];
  C2* bufA = reinterpret_cast<C2*>(mf_sm_raw);   // [CW][2][N3]
  C2* bufB = bufA + CW * 2 * N3;                 // [CW][2][N3]
  const T* w1 = tab + 2 * N2;
  const T* eoBf = tab + 2 * N2 + NP;
  const T* eoBb = eoBf + sf_eo_size(NP);
  const T* eoDf = eoBb + sf_eo_size(NP);
  const T* eoDb = eoDf + sf_eo_size(NP);
  const int tid = threadIdx.x;

  const int per_xcd = (total + 7) / 8;
  const int item = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (item >= total) return;
  // edge task: column fastest, then spin, then the z-line (x, y), so that
  // neighbouring lanes read one row
  const bool edge = tid < 2 * CW * N2;
  const int tc = tid % CW, ts = (tid / CW) % 2, tl = tid / (2 * CW);
  const int e = cells[item / n_chunks];
  const int col = (item % n_chunks) * CW + tc;
  const int32_t* nodes = cell_nodes + (size_t)e * N3;
  const bool ok = edge && col < n_vec;

  // gather M^{-1/2} x along the task's z-line (addresses clamped in bounds) and
  // interpolate along z into bufB
  if (edge) {
    const int cc = ok ? col : 0;
    int64_t I[NP];
#pragma unroll
    for (int z = 0; z < NP; ++z) I[z] = nodes[tl + z * N2];
    double xs[NP];
    double2 xr[NP];
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      xs[z] = minv_sqrt[I[z]];
      xr[z] = X[(2 * I[z] + ts) * ldx + cc];
    }
    C2 u[NP];
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      const double f = ok ? xs[z] : 0.0;
      u[z] = C2{(T)(f * xr[z].x), (T)(f * xr[z].y)};
    }
    C2* out = bufB + (tc * 2 + ts) * N3 + tl;
    C2 r[NP];
    sf_eo<T, NP, false>(eoBf, u, r);
#pragma unroll
    for (int o = 0; o < NP; ++o) out[o * N2] = r[o];
  }
  lds_barrier();
  sf_line_pass<NP, 2 * CW, 1, NT, T>(eoBf, bufB, bufB);   // in place: a thread owns its line
  lds_barrier();
  sf_line_pass<NP, 2 * CW, 0, NT, T>(eoBf, bufB, bufB);   // U in bufB
  lds_barrier();

  // potential and field terms at the points
  for (int t = tid; t < N3 * CW; t += NT) {
    const int q = t % N3, c = t / N3;
    const T wj = J * w1[q % NP] * w1[(q / NP) % NP] * w1[q / N2];
    const Q4 d = qd[(size_t)e * N3 + q];
    const C2 u0 = bufB[(c * 2) * N3 + q], u1 = bufB[(c * 2 + 1) * N3 + q];
    const T s = d.x + half_k2 * wj;
    // up:   (s + Bz) u0 + (Bx - i By) u1;  down: (s - Bz) u1 + (Bx + i By) u0
    C2 w0, w2;
    w0.x = (s + d.w) * u0.x + d.y * u1.x + d.z * u1.y;
    w0.y = (s + d.w) * u0.y + d.y * u1.y - d.z * u1.x;
    w2.x = (s - d.w) * u1.x + d.y * u0.x - d.z * u0.y;
    w2.y = (s - d.w) * u1.y + d.y * u0.y + d.z * u0.x;
    bufA[(c * 2) * N3 + q] = w0;
    bufA[(c * 2 + 1) * N3 + q] = w2;
  }
  lds_barrier();
  grad_pass<T, NP, CW, 2, KT, false>(eoDf, eoDb, eoBb, w1, J, a2, b2, kin + 2 * N3, bufB, bufA);
  lds_barrier();
  grad_pass<T, NP, CW, 1, KT, false>(eoDf, eoDb, eoBb, w1, J, a1, b1, kin + 1 * N3, bufB, bufA);
  lds_barrier();
  grad_pass<T, NP, CW, 0, KT, true>(eoDf, eoDb, eoBb, w1, J, a0, b0, kin + 0 * N3, bufB, bufA);   // and W -> B W along x
  lds_barrier();
  sf_line_pass<NP, 2 * CW, 1, NT, T>(eoBb, bufA, bufA);
  lds_barrier();

  // last backward contraction along z, then Y[rows] += alpha M^{-1/2} y (the
  // rows' indices, factors and old values loaded together before the stores)
  if (ok) {
    const C2* in = bufA + (tc * 2 + ts) * N3 + tl;
    C2 v[NP], y[NP];
    double2 r[NP];
#pragma unroll
    for (int z = 0; z < NP; ++z) v[z] = in[z * N2];
    sf_eo<T, NP, false>(eoBb, v, y);
#pragma unroll
    for (int o = 0; o < NP; ++o) r[o] = double2{(double)y[o].x, (double)y[o].y};
    int64_t I[NP];
#pragma unroll
    for (int o = 0; o < NP; ++o) I[o] = nodes[tl + o * N2];
    double sc[NP];
    double2 yo[NP];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      sc[o] = (alpha_d ? *alpha_d : alpha) * minv_sqrt[I[o]];
      yo[o] = Y[(2 * I[o] + ts) * ldy + col];
    }
#pragma unroll
    for (int o = 0; o < NP; ++o)
      Y[(2 * I[o] + ts) * ldy + col] = double2{fma(sc[o], r[o].x, yo[o].x), fma(sc[o], r[o].y, yo[o].y)};
  }
}

// qd[e][q] = w_q J (V, Bx, By, Bz), in FP64 and FP32
__global__ void mf_qdata_kernel(const double* __restrict__ V, const double* __restrict__ B,
                                const double* __restrict__ w1, double J, int nq, int64_t n_points,
                                double4* __restrict__ qd, float4* __restrict__ qd32) {
  const int nq3 = nq * nq * nq;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_points;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(p % nq3);
    const double wj = J * w1[q % nq] * w1[(q / nq) % nq] * w1[q / (nq * nq)];
    const double4 v = double4{wj * V[p], wj * B[3 * p], wj * B[3 * p + 1], wj * B[3 * p + 2]};
    qd[p] = v;
    qd32[p] = float4{(float)v.x, (float)v.y, (float)v.z, (float)v.w};
  }
}

template <class T, int NP, bool KT>
void launch_mf_t(chfsi_ctx* c, const KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw, int n_vec,
                 double alpha, const double* alpha_d) {
  typedef typename MfT<T>::C2 C2;
  typedef typename MfT<T>::Q4 Q4;
  constexpr int CW = mf_cw<T>(NP);
  const size_t sh = 2 * (size_t)CW * 2 * NP * NP * NP * sizeof(C2);
  const int n_chunks = cdiv(n_vec, CW);
  T a[3], b[3];
  for (int d = 0; d < 3; ++d) {
    const double sd = 2.0 / c->h[d];
    a[d] = (T)(0.5 * sd * sd);
    b[d] = (T)(kp.k[d] * sd);
  }
  const T half_k2 = (T)(0.5 * (kp.k[0] * kp.k[0] + kp.k[1] * kp.k[1] + kp.k[2] * kp.k[2]));
  const T* tab = nullptr;
  const Q4* qd = nullptr;
  const T* kin = nullptr;    // FP32 only (FP64 forms the weights in the kernel)
  if constexpr (sizeof(T) == 8) {
    tab = c->mf_tab.ptr;
    qd = reinterpret_cast<const Q4*>(c->mf_qd.ptr);
    kin = tab;
  } else {
    tab = c->mf_tab32.ptr;
    qd = reinterpret_cast<const Q4*>(c->mf_qd32.ptr);
    kin = c->mf_kin32.ptr;
  }
  const double np3 = (double)NP * NP * NP;
  for (int k = 0; k < c->n_colours; ++k) {
    const int n_in = c->colour_off[k + 1] - c->colour_off[k];
    if (n_in == 0) continue;
    const int64_t total = (int64_t)n_in * n_chunks;
    CHFSI_CHECK(total < (int64_t)1 << 30, CHFSI_EINVAL, "matrix-free apply: too many work items");
    // algorithmic flops of the dense cell product (the filter's count), flops of
    // 12 dense line contractions per spin (the even-odd form issues about half of
    // those multiply-adds), and the rows moved
    const double n2 = 2.0 * c->nloc;
    const double flops = 8.0 * n2 * n2 * n_vec * n_in;
    const double exec = 96.0 * np3 * NP * (double)n_vec * n_in;
    const double bytes = (double)n_in * 3.0 * c->nloc * 2.0 * n_vec * sizeof(double2);
    StageTimer tm(c, sizeof(T) == 8 ? CHFSI_STAGE_CELL_FP64 : CHFSI_STAGE_CELL_FP32, flops, exec, bytes);
    const int grid = (int)(8 * ((total + 7) / 8));
    hipLaunchKernelGGL((mf_apply_kernel<T, NP, KT>), dim3(grid), dim3(MfT<T>::NT), sh, c->stream, tab, qd,
                       c->cell_nodes.ptr, c->colour_cells.ptr + c->colour_off[k], (int)total, n_chunks,
                       c->minv_sqrt.ptr, X, ldx, W, ldw, n_vec, alpha, (T)c->J, half_k2, a[0], a[1], a[2], b[0],
                       b[1], b[2], kin, alpha_d);
    LAUNCH_CHECK();
  }
}

template <int NP>
void launch_mf_np(chfsi_ctx* c, const KPoint& kp, bool fp64, const double2* X, int64_t ldx, double2* W, int64_t ldw,
                  int n_vec, double alpha, const double* alpha_d) {
  if (fp64) {
    if (kp.gamma) launch_mf_t<double, NP, false>(c, kp, X, ldx, W, ldw, n_vec, alpha, alpha_d);
    else launch_mf_t<double, NP, true>(c, kp, X, ldx, W, ldw, n_vec, alpha, alpha_d);
  } else {
    if (kp.gamma) launch_mf_t<float, NP, false>(c, kp, X, ldx, W, ldw, n_vec, alpha, alpha_d);
    else launch_mf_t<float, NP, true>(c, kp, X, ldx, W, ldw, n_vec, alpha, alpha_d);
  }
}

}  // namespace

bool mf_supported(const chfsi_ctx* c) { return c->nq == c->np1 && c->np1 >= 2 && c->np1 <= 9; }

void mf_prepare(chfsi_ctx* c) {
  CHFSI_CHECK(mf_supported(c), CHFSI_EINVAL, "matrix-free apply needs n_q = p + 1 and 1 <= p <= 8");
  const int n = c->np1;
  std::vector<double> Bq, Dlag;
  lagrange_on(c->ref.xq, c->ref.xq, Bq, Dlag);   // Dlag[r][q] = l~_r'(x_q)
  std::vector<double> tab(2 * n * n + n);
  for (int a = 0; a < n; ++a)
    for (int q = 0; q < n; ++q) tab[a * n + q] = c->ref.B[(size_t)a * c->nq + q];
  for (int q = 0; q < n; ++q)
    for (int r = 0; r < n; ++r) tab[n * n + q * n + r] = Dlag[(size_t)r * n + q];
  for (int q = 0; q < n; ++q) tab[2 * n * n + q] = c->ref.wq[q];
  // even-odd tables of B (nodes -> points), B^T, Dq (G = Dq U) and Dq^T, each as
  // out[o] = sum_i M[i][o] in[i]
  const int h = n / 2, es = 2 * h * h + 2 * h + 1;
  auto Bm = [&](int i, int o) { return tab[i * n + o]; };
  auto Dm = [&](int q, int r) { return tab[n * n + q * n + r]; };
  auto eo = [&](const std::function<double(int, int)>& M, bool skew) {
    double big = 0.0, dev = 0.0;
    for (int i = 0; i < n; ++i)
      for (int o = 0; o < n; ++o) {
        big = std::max(big, std::fabs(M(i, o)));
        dev = std::max(dev, std::fabs(M(n - 1 - i, n - 1 - o) - (skew ? -1.0 : 1.0) * M(i, o)));
      }
    CHFSI_CHECK(dev <= 1e-12 * std::max(1.0, big), CHFSI_EINVAL, "quadrature rule is not symmetric");
    std::vector<double> t(es, 0.0);
    for (int i = 0; i < h; ++i)
      for (int o = 0; o < h; ++o) {
        t[i * h + o] = 0.5 * (M(i, o) + M(i, n - 1 - o));
        t[h * h + i * h + o] = 0.5 * (M(i, o) - M(i, n - 1 - o));
      }
    if (n % 2) {
      for (int o = 0; o < h; ++o) t[2 * h * h + o] = M(h, o);
      for (int i = 0; i < h; ++i) t[2 * h * h + h + i] = M(i, h);
      t[2 * h * h + 2 * h] = M(h, h);
    }
    tab.insert(tab.end(), t.begin(), t.end());
  };
  eo([&](int i, int o) { return Bm(i, o); }, false);
  eo([&](int i, int o) { return Bm(o, i); }, false);
  eo([&](int i, int o) { return Dm(o, i); }, true);
  eo([&](int i, int o) { return Dm(i, o); }, true);
  std::vector<float> tab32(tab.begin(), tab.end());
  // The FP32 tables keep identities of the exact ones, so that rounding them does
  // not perturb every cell the same way: the interpolation reproduces constants
  // and linear functions (sum_a l_a = 1, sum_a xi_a l_a(x) = x) and the
  // collocation derivative maps them to 0 and 1.  In each sum the closing entry
  // is re-formed in FP64 from the rounded others.  The tables of the transposed
  // contractions are then taken from the rounded forward ones (for a
  // centrosymmetric M the even-odd blocks of M^T are those of M transposed; for a
  // skew one the two blocks also swap), so that the FP32 operator keeps the exact
  // adjoint structure of the FP64 one.
  {
    const int b0 = 2 * n * n + n, bb0 = b0 + es, d0 = b0 + 2 * es, db0 = b0 + 3 * es;
    const std::vector<double>& xi = c->ref.xi;   // GLL nodes (input of B)
    const std::vector<double>& xq = c->ref.xq;   // quadrature points (output of B, input of Dq)
    auto Af = [&](int t0, int i, int o) -> float& { return tab32[t0 + i * h + o]; };
    auto Cf = [&](int t0, int i, int o) -> float& { return tab32[t0 + h * h + i * h + o]; };
    for (int o = 0; o < h; ++o) {
      // B: constants (sum of the A column and the middle row) and linear functions (C column)
      double sa = 0.0, sc = 0.0, da = 0.0, dc = 0.0;
      for (int i = 0; i < h; ++i) {
        if (!(n % 2 == 0 && i == h - 1)) sa += Af(b0, i, o);
        if (i > 0) sc += Cf(b0, i, o) * xi[i];
        if (i > 0) da += Af(d0, i, o) * xq[i];
        if (!(n % 2 == 0 && i == h - 1)) dc += Cf(d0, i, o);
      }
      if (n % 2) {
        tab32[b0 + 2 * h * h + o] = (float)(1.0 - 2.0 * sa);
        tab32[d0 + 2 * h * h + o] = (float)(-2.0 * dc);
      } else {
        Af(b0, h - 1, o) = (float)(0.5 - sa);
        Cf(d0, h - 1, o) = (float)(-dc);
      }
      Cf(b0, 0, o) = (float)((0.5 * xq[o] - sc) / xi[0]);
      Af(d0, 0, o) = (float)((0.5 - da) / xq[0]);
    }
    if (n % 2) {
      double sm = 0.0, dm = 0.0;
      for (int i = 0; i < h; ++i) sm += tab32[b0 + 2 * h * h + h + i];
      tab32[b0 + 2 * h * h + 2 * h] = (float)(1.0 - 2.0 * sm);
      for (int i = 1; i < h; ++i) dm += tab32[d0 + 2 * h * h + h + i] * xq[i];
      tab32[d0 + 2 * h * h + h] = (float)((0.5 - dm) / xq[0]);
      tab32[d0 + 2 * h * h + 2 * h] = 0.0f;
    }
    for (int i = 0; i < h; ++i)
      for (int o = 0; o < h; ++o) {
        Af(bb0, i, o) = Af(b0, o, i);
        Cf(bb0, i, o) = Cf(b0, o, i);
        Af(db0, i, o) = Cf(d0, o, i);
        Cf(db0, i, o) = Af(d0, o, i);
      }
    if (n % 2) {
      for (int k = 0; k < h; ++k) {
        tab32[bb0 + 2 * h * h + k] = tab32[b0 + 2 * h * h + h + k];
        tab32[bb0 + 2 * h * h + h + k] = tab32[b0 + 2 * h * h + k];
        tab32[db0 + 2 * h * h + k] = tab32[d0 + 2 * h * h + h + k];
        tab32[db0 + 2 * h * h + h + k] = tab32[d0 + 2 * h * h + k];
      }
      tab32[bb0 + 2 * h * h + 2 * h] = tab32[b0 + 2 * h * h + 2 * h];
      tab32[db0 + 2 * h * h + 2 * h] = 0.0f;
    }
  }
  // FP32 kinetic weights per point and direction: (2/h_d)^2 / 2 * J w_x w_y w_z
  const int n3 = n * n * n;
  std::vector<float> kin32(3 * (size_t)n3);
  for (int d = 0; d < 3; ++d) {
    const double sd = 2.0 / c->h[d];
    for (int q = 0; q < n3; ++q)
      kin32[(size_t)d * n3 + q] =
          (float)(0.5 * sd * sd * c->J * c->ref.wq[q % n] * c->ref.wq[(q / n) % n] * c->ref.wq[q / (n * n)]);
  }
  c->mf_tab.upload(tab.data(), tab.size(), c->stream);
  c->mf_tab32.upload(tab32.data(), tab32.size(), c->stream);
  c->mf_kin32.upload(kin32.data(), kin32.size(), c->stream);
  CHFSI_HIP(hipStreamSynchronize(c->stream));   // the host tables go out of scope
}

void mf_set_local(chfsi_ctx* c, const double* V, const double* B) {
  if (c->mf_tab.n == 0) mf_prepare(c);
  const int64_t n_points = (int64_t)c->n_cells * c->nq3;
  c->mf_qd.alloc((size_t)n_points * 4);
  c->mf_qd32.alloc((size_t)n_points * 4);
  DevBuf<double> w1;
  w1.upload(c->ref.wq.data(), c->ref.wq.size(), c->stream);
  hipLaunchKernelGGL(mf_qdata_kernel, dim3((unsigned)std::min<int64_t>(cdiv(n_points, 256), 8192)), dim3(256), 0,
                     c->stream, V, B, w1.ptr, c->J, c->nq, n_points, reinterpret_cast<double4*>(c->mf_qd.ptr),
                     reinterpret_cast<float4*>(c->mf_qd32.ptr));
  LAUNCH_CHECK();
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  c->mf_gen = c->gen;
}

void launch_mf_products(chfsi_ctx* c, const KPoint& kp, int prec, const double2* X, int64_t ldx, double2* W,
                        int64_t ldw, int n_vec, double alpha, const double* alpha_d) {
  const bool fp64 = prec != CHFSI_PREC_MIXED;
  switch (c->np1) {
    case 2: launch_mf_np<2>(c, kp, fp64, X, ldx, W, ldw, n_vec, alpha, alpha_d); break;
    case 3: launch_mf_np<3>(c, kp, fp64, X, ldx, W, ldw, n_vec, alpha, alpha_d); break;
    case 4: launch_mf_np<4>(c, kp, fp64, X, ldx, W, ldw, n_vec, alpha, alpha_d); break;
    case 5: launch_mf_np<5>(c, kp, fp64, X, ldx, W, ldw, n_vec, alpha, alpha_d); break;
    case 6: launch_mf_np<6>(c, kp, fp64, X, ldx, W, ldw, n_vec, alpha, alpha_d); break;
    case 7: launch_mf_np<7>(c, kp, fp64, X, ldx, W, ldw, n_vec, alpha, alpha_d); break;
    case 8: launch_mf_np<8>(c, kp, fp64, X, ldx, W, ldw, n_vec, alpha, alpha_d); break;
    case 9: launch_mf_np<9>(c, kp, fp64, X, ldx, W, ldw, n_vec, alpha, alpha_d); break;
    default: throw Error{CHFSI_EINVAL, "matrix-free apply: unsupported p"};
  }
}

}  // namespace chfsi
