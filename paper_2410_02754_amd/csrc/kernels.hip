// Device kernels and their launchers for gfx950 (CDNA4, wave64).
//
// Operator action (Sec. IV.B, "FE discretized matrix multivector product"):
// extraction X_e = R_e X, cell products H_e X_e, nonlocal projector terms,
// assembly Y = sum_e R_e^T Y_e.  The four steps run as
//   1. an element-wise pass that initialises the output with the recurrence
//      terms (beta W + gamma X),
//   2. the projector contraction C_a = P_a^H X, the coupling C'_a = Delta_a C_a
//      and the node-centric back-product W += P_a C'_a (eqn:FEHnloc),
//   3. one launch per cell colour of the fused gather / MFMA cell product /
//      scatter-add kernel; cells of one colour share no node, so the
//      read-add-write of the epilogue needs no atomics and the result is
//      bitwise reproducible.
//
// The cell products (step 3) live in cell.hip; this file holds the element-wise,
// nonlocal, adjoint and dense-block kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "mfma.h"
#include "sumfact.h"

namespace chfsi {

// ============================================================================
// Element-wise passes
// ============================================================================
__global__ void axpby_rows_kernel(double2* __restrict__ W, int64_t ldw, const double2* __restrict__ X,
                                  int64_t ldx, int64_t rows, int n_vec, double beta, double gamma) {
  const int64_t total = rows * n_vec;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n_vec;
    const int n = (int)(t - r * n_vec);
    double2 w = {0.0, 0.0};
    if (beta != 0.0) {
      w = W[r * ldw + n];
      w.x *= beta;
      w.y *= beta;
    }
    if (gamma != 0.0) {
      const double2 x = X[r * ldx + n];
      w.x += gamma * x.x;
      w.y += gamma * x.y;
    }
    W[r * ldw + n] = w;
  }
}

void launch_axpby_rows(chfsi_ctx* c, double2* W, int64_t ldw, const double2* X, int64_t ldx,
                       int64_t rows, int n_vec, double beta, double gamma) {
  const int64_t total = rows * n_vec;
  StageTimer tm(c, CHFSI_STAGE_AXPY, 0.0, 0.0,
                (double)total * sizeof(double2) * (1.0 + (beta != 0.0) + (gamma != 0.0)));
  const int blocks = (int)std::min<int64_t>(cdiv(total, 256), 8192);
  hipLaunchKernelGGL(axpby_rows_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, c->stream, W, ldw, X,
                     ldx, rows, n_vec, beta, gamma);
  LAUNCH_CHECK();
}

__global__ void copy_rows_kernel(double2* __restrict__ D, int64_t ldd, const double2* __restrict__ S,
                                 int64_t lds, int64_t rows, int n_vec) {
  const int64_t total = rows * n_vec;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n_vec;
    const int n = (int)(t - r * n_vec);
    D[r * ldd + n] = S[r * lds + n];
  }
}

void launch_copy_rows(chfsi_ctx* c, double2* dst, int64_t ldd, const double2* src, int64_t lds,
                      int64_t rows, int n_vec) {
  const int64_t total = rows * n_vec;
  const int blocks = (int)std::min<int64_t>(cdiv(total, 256), 8192);
  hipLaunchKernelGGL(copy_rows_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, c->stream, dst, ldd, src,
                     lds, rows, n_vec);
  LAUNCH_CHECK();
}

// ============================================================================
// Nonlocal projector terms (eqn:FEHnloc in the cell form of Sec. IV.B)
// ============================================================================
template <class T> struct C2;
template <> struct C2<double> { typedef double2 type; };
template <> struct C2<float> { typedef float2 type; };

constexpr int kMaxPj = 9;

// 16-column blocks per wave of the contraction and initialisation kernels: one
// in FP64 (fewer registers, more resident waves to cover the row loads), two in FP32.
template <class T>
constexpr int nl_col_blocks() { return sizeof(T) == 8 ? 1 : 2; }

// Contraction partials, one wave per (chunk of an atom's support, 16- or
// 32-column tile): partial[chunk][2 chi + s][n] = sum_j conj(P[j][chi]) X[2 node_j + s][n].
// Done as 16x16x4 MFMAs: row = projector index chi (n_pj <= 9 of the 16 rows
// used), k = four support entries per step, column = 16 of the tile's columns;
// sixteen entries' operands are loaded before their MFMAs are issued.
// REALP: the projector values are real (Gamma point), two real MFMAs per step.
// PACK (complex values, n_pj <= 8): rows 0-7 carry the real parts and rows
// 8-15 the imaginary parts of the projectors, so one MFMA against Re x and one
// against Im x replace the four of the plain complex step, and
//   Re c = (p_r x_r)[chi] + (p_i x_i)[chi + 8],  Im c = (p_r x_i)[chi] - (p_i x_r)[chi + 8];
// row chi + 8 is accumulator register j + 2 of the same lane (FP64) or register
// j of the lane 32 above (FP32).
template <class T, bool REALP, bool PACK = false>
__global__ __launch_bounds__(256) void nl_contract_kernel(
    const typename C2<T>::type* __restrict__ proj, const int32_t* __restrict__ sup_node,
    const int32_t* __restrict__ chunk_atom, const int32_t* __restrict__ chunk_begin,
    const int32_t* __restrict__ chunk_end, const int32_t* __restrict__ chunk_order,
    const int32_t* __restrict__ atom_npj, int max_pj, int n_work, int n_coltiles,
    const double2* __restrict__ X, int64_t ldx, int n_vec, typename C2<T>::type* __restrict__ partial) {
  typedef typename C2<T>::type CT;
  typedef typename Vec4<T>::type V4;
  static_assert(!PACK || !REALP, "packed rows: complex projector values only");
  constexpr int U = 4;                    // k-steps per batch
  constexpr int NCB = nl_col_blocks<T>();
  // each XCD takes a contiguous range of the (window, atom)-ordered chunks, so the
  // chunks of different atoms over the same rows meet in that XCD's L2
  const int per_xcd = (int)((gridDim.x + 7) / 8);
  const int bid = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  const int wid = __builtin_amdgcn_readfirstlane(bid * 4 + (int)(threadIdx.x >> 6));
  if (wid >= n_work) return;              // no barrier in this kernel
  const int lane = threadIdx.x & 63;
  const int kl = lane >> 4, il = lane & 15;
  const int oi = wid / n_coltiles, ct = wid - oi * n_coltiles;
  const int ch = chunk_order[oi];
  const int a = chunk_atom[ch], b = chunk_begin[ch], e = chunk_end[ch];
  const int npj = atom_npj[a];
  const int chi = PACK ? (il & 7) : il;   // projector of this lane's A row
  const bool rv = chi < npj;              // ... and whether it is in use
  int col[NCB];
  bool cv[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    col[cb] = ct * 16 * NCB + cb * 16 + il;
    cv[cb] = col[cb] < n_vec;
    if (!cv[cb]) col[cb] = n_vec - 1;     // clamped: loads stay in bounds
  }
  V4 cr[2][NCB], ci[2][NCB];              // [spin][16-column block]
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) cr[sp][cb] = ci[sp][cb] = V4{0, 0, 0, 0};
  for (int j0 = b; j0 < e; j0 += 4 * U) {
    CT pv[U];
    double2 xv[U][2][NCB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + 4 * u + kl;      // entry of this lane's k index
      const bool jv = j < e;
      const int64_t nd = sup_node[jv ? j : b];
      pv[u] = (jv && rv) ? proj[(size_t)j * max_pj + chi] : CT{(T)0, (T)0};
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const double2 v = X[(2 * nd + sp) * ldx + col[cb]];
          xv[u][sp][cb] = (jv && cv[cb]) ? v : double2{0.0, 0.0};
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (PACK) {
        const T av = il < 8 ? pv[u].x : pv[u].y;
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            cr[sp][cb] = mfma(av, (T)xv[u][sp][cb].x, cr[sp][cb]);   // [p_r; p_i] x_r
            ci[sp][cb] = mfma(av, (T)xv[u][sp][cb].y, ci[sp][cb]);   // [p_r; p_i] x_i
          }
      } else {
        const T pr = pv[u].x, pi = pv[u].y, npi = -pv[u].y;
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            const T xr = (T)xv[u][sp][cb].x, xi = (T)xv[u][sp][cb].y;
            cr[sp][cb] = mfma(pr, xr, cr[sp][cb]);      // conj(p) x
            if (!REALP) cr[sp][cb] = mfma(pi, xi, cr[sp][cb]);
            ci[sp][cb] = mfma(pr, xi, ci[sp][cb]);
            if (!REALP) ci[sp][cb] = mfma(npi, xr, ci[sp][cb]);
          }
      }
    }
  }
  CT* out = partial + (size_t)ch * 2 * max_pj * n_vec;
  if constexpr (PACK) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (sizeof(T) == 8 && j >= 2) break;                       // FP64: rows 8-15
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
          // row x + 8: same lane (FP64) or the lane 32 above (FP32; every lane shuffles)
          T hr, hi;
          if constexpr (sizeof(T) == 8) {
            hr = cr[sp][cb][j + 2];
            hi = ci[sp][cb][j + 2];
          } else {
            hr = __shfl_down(cr[sp][cb][j], 32);
            hi = __shfl_down(ci[sp][cb][j], 32);
          }
          const int x = acc_row<T>(lane, j);
          if (x >= 8 || x >= npj || !cv[cb]) continue;             // FP32: lanes 32-63 hold rows 8-15
          CT v;
          v.x = cr[sp][cb][j] + hi;
          v.y = ci[sp][cb][j] - hr;
          out[(size_t)(2 * x + sp) * n_vec + col[cb]] = v;
        }
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = acc_row<T>(lane, j);
      if (x >= npj) continue;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        if (!cv[cb]) continue;
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
          CT v;
          v.x = cr[sp][cb][j];
          v.y = ci[sp][cb][j];
          out[(size_t)(2 * x + sp) * n_vec + col[cb]] = v;
        }
      }
    }
  }
}

// Csum[a][r][n] = sum over the chunks of atom a of partial[chunk][r][n] (chunk order fixed)
// (a column group: partial holds n_vec columns, written to Csum columns col0.. of
// its ldc-wide rows)
template <class T>
__global__ __launch_bounds__(64) void nl_reduce_kernel(const typename C2<T>::type* __restrict__ partial,
                                                       const int32_t* __restrict__ atom_chunk0,
                                                       const int32_t* __restrict__ atom_npj, int max_pj,
                                                       int n_vec, int ldc, int col0,
                                                       typename C2<T>::type* __restrict__ Csum) {
  typedef typename C2<T>::type CT;
  const int a = blockIdx.x, r = blockIdx.y;
  const int col = blockIdx.z * 64 + threadIdx.x;
  const int mr = 2 * max_pj;
  if (r >= 2 * atom_npj[a] || col >= n_vec) return;
  T sr = 0, si = 0;
  const int c0 = atom_chunk0[a], c1 = atom_chunk0[a + 1];
  int ch = c0;
  for (; ch + 3 < c1; ch += 4) {
    CT v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = partial[((size_t)(ch + u) * mr + r) * n_vec + col];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sr += v[u].x;
      si += v[u].y;
    }
  }
  for (; ch < c1; ++ch) {
    const CT v = partial[((size_t)ch * mr + r) * n_vec + col];
    sr += v.x;
    si += v.y;
  }
  CT o;
  o.x = sr;
  o.y = si;
  Csum[((size_t)a * mr + r) * ldc + col0 + col] = o;
}

// C'[a][r][n] = alpha sum_r' Delta_a[r][r'] Csum[a][r'][n]; alpha_d (device, or
// null) overrides alpha at run time (graph replays with new filter bounds)
template <class T>
__global__ __launch_bounds__(64) void nl_delta_kernel(const typename C2<T>::type* __restrict__ Csum,
                                                      const int32_t* __restrict__ atom_npj,
                                                      const double2* __restrict__ delta, int max_pj, int n_vec,
                                                      double alpha, const double* __restrict__ alpha_d,
                                                      typename C2<T>::type* __restrict__ Cp) {
  typedef typename C2<T>::type CT;
  if (alpha_d) alpha = *alpha_d;
  const int a = blockIdx.x;
  const int col = blockIdx.y * 64 + threadIdx.x;
  if (col >= n_vec) return;
  const int nr = 2 * atom_npj[a];
  const int mr = 2 * max_pj;
  T cr[2 * kMaxPj], cim[2 * kMaxPj];
#pragma unroll
  for (int q = 0; q < 2 * kMaxPj; ++q) {
    cr[q] = cim[q] = (T)0;
    if (q < nr) {
      const CT v = Csum[((size_t)a * mr + q) * n_vec + col];
      cr[q] = v.x;
      cim[q] = v.y;
    }
  }
  for (int r = 0; r < nr; ++r) {
    T sr = 0, si = 0;
#pragma unroll
    for (int q = 0; q < 2 * kMaxPj; ++q)
      if (q < nr) {
        const double2 d = delta[((size_t)a * mr + r) * mr + q];
        sr += (T)d.x * cr[q] - (T)d.y * cim[q];
        si += (T)d.x * cim[q] + (T)d.y * cr[q];
      }
    CT o;
    o.x = (T)alpha * sr;
    o.y = (T)alpha * si;
    Cp[((size_t)a * mr + r) * n_vec + col] = o;
  }
}

// Recurrence initialisation fused with the nonlocal back-product, one wave per
// (run of kNlRun = 16 consecutive global nodes, 16- or 32-column tile):
//   W[2I+s][n] = beta Wold[2I+s][n] + gamma X[2I+s][n] + rscale[n] Rs[2I+s][n]
//               + sum_{atoms a at I} sum_chi P[entry(a, I)][chi] C'[a][2 chi + s][n]
// For each atom meeting the run, the back-product is the complex product of the
// run's 16 x n_pj projector block with the n_pj x (16 | 32) coefficient tile, done as
// 16x16x4 MFMAs (k = projector index, padded to a multiple of 4; nodes of the run
// outside the atom's support contribute zero rows).  All operands of an atom are
// loaded before its MFMAs; each coefficient row is read once per run.  W and
// Wold are not read without the beta term, X without the gamma term, Rs without
// the residual term (FL: which terms are present).  REALP: real projector values
// (Gamma point), two real MFMAs per step instead of four.  bg_d (device, or null)
// overrides (beta, gamma) at run time; FL still selects which terms are read.
constexpr int kInitBeta = 1, kInitGamma = 2, kInitRs = 4;

template <class T, int FL, bool REALP>
__global__ __launch_bounds__(256) void init_nl_kernel(
    const typename C2<T>::type* __restrict__ proj, const int32_t* __restrict__ run_off,
    const int32_t* __restrict__ pair_atom, const int32_t* __restrict__ pair_ent,
    const int32_t* __restrict__ atom_npj, int max_pj, const typename C2<T>::type* __restrict__ Cp,
    int has_nl, const double2* __restrict__ X, int64_t ldx, double2* W, int64_t ldw,
    const double2* Wold, int64_t ldo, const double2* __restrict__ Rs, int64_t ldr,
    const double* __restrict__ rscale, int64_t n_nodes, int n_work, int n_coltiles, int n_vec, double beta,
    double gamma, const double* __restrict__ bg_d) {
  typedef typename C2<T>::type CT;
  typedef typename Vec4<T>::type V4;
  static_assert(kNlRun == 16, "one MFMA row block per run");
  if (bg_d) {
    beta = bg_d[0];
    gamma = bg_d[1];
  }
  constexpr int KS = (kMaxPj + 3) / 4;    // k-steps per atom
  constexpr int NCB = nl_col_blocks<T>();
  const int wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  if (wid >= n_work) return;              // no barrier in this kernel
  const int run = wid / n_coltiles, ct = wid - run * n_coltiles;
  const int lane = threadIdx.x & 63;
  const int kl = lane >> 4, il = lane & 15;
  int col[NCB];
  bool cv[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    col[cb] = ct * 16 * NCB + cb * 16 + il;
    cv[cb] = col[cb] < n_vec;
    if (!cv[cb]) col[cb] = n_vec - 1;     // clamped: loads stay in bounds
  }
  V4 dr[2][NCB], di[2][NCB];              // [spin][16-column block]
  // FP64: the recurrence terms start the accumulators, so that their loads are in
  // flight while the projector back-product runs (lane element j of an
  // accumulator is node acc_row(lane, j) of the run, column col[cb])
  constexpr bool kPre = sizeof(T) == 8;
  const int64_t node0 = (int64_t)run * kNlRun;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      dr[sp][cb] = di[sp][cb] = V4{0, 0, 0, 0};
      if constexpr (kPre) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t node = node0 + acc_row<T>(lane, j);
          const int64_t row = 2 * (node < n_nodes ? node : n_nodes - 1) + sp;
          const int c = col[cb];
          double tr = 0.0, ti = 0.0;
          if (FL & kInitBeta) {
            const double2 o = Wold[row * ldo + c];
            tr += beta * o.x;
            ti += beta * o.y;
          }
          if (FL & kInitGamma) {
            const double2 xv = X[row * ldx + c];
            tr += gamma * xv.x;
            ti += gamma * xv.y;
          }
          if (FL & kInitRs) {
            const double2 rv = Rs[row * ldr + c];
            const double sc = rscale[c];
            tr += sc * rv.x;
            ti += sc * rv.y;
          }
          dr[sp][cb][j] = (T)tr;
          di[sp][cb][j] = (T)ti;
        }
      }
    }
  if (has_nl) {
    const int p0 = run_off[run], p1 = run_off[run + 1];
    for (int pr = p0; pr < p1; ++pr) {
      const int a = pair_atom[pr];
      const int npj = atom_npj[a];
      const int ent = pair_ent[(size_t)pr * kNlRun + il];      // A row = node il of the run
      const CT* cpa = Cp + (size_t)a * 2 * max_pj * n_vec;
      CT pa[KS];
      CT bv[KS][2][NCB];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int x = 4 * ks + kl;                               // projector index of this lane
        const bool xv = x < npj;
        pa[ks] = (xv && ent >= 0) ? proj[(size_t)ent * max_pj + x] : CT{(T)0, (T)0};
        const int xr = xv ? x : 0;
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            const CT v = cpa[(size_t)(2 * xr + sp) * n_vec + col[cb]];
            bv[ks][sp][cb] = (xv && cv[cb]) ? v : CT{(T)0, (T)0};
          }
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (4 * ks >= npj) break;                                // wave-uniform
        const T nai = -pa[ks].y;
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            dr[sp][cb] = mfma(pa[ks].x, bv[ks][sp][cb].x, dr[sp][cb]);
            if (!REALP) dr[sp][cb] = mfma(nai, bv[ks][sp][cb].y, dr[sp][cb]);
            di[sp][cb] = mfma(pa[ks].x, bv[ks][sp][cb].y, di[sp][cb]);
            if (!REALP) di[sp][cb] = mfma(pa[ks].y, bv[ks][sp][cb].x, di[sp][cb]);
          }
      }
    }
  }
  // lane holds nodes acc_row(lane, j) of the run, columns col[cb]; every load of
  // the epilogue is issued unconditionally (clamped rows) and only the stores
  // are predicated
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t node = node0 + acc_row<T>(lane, j);
    const bool nv = node < n_nodes;
    const int64_t nodec = nv ? node : n_nodes - 1;
    double2 v[NCB][2];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
        const int64_t row = 2 * nodec + sp;
        const int c = col[cb];
        double2 t = {(double)dr[sp][cb][j], (double)di[sp][cb][j]};
        if constexpr (kPre) {
          v[cb][sp] = t;
          continue;
        }
        if (FL & kInitBeta) {
          const double2 o = Wold[row * ldo + c];
          t.x += beta * o.x;
          t.y += beta * o.y;
        }
        if (FL & kInitGamma) {
          const double2 xv = X[row * ldx + c];
          t.x += gamma * xv.x;
          t.y += gamma * xv.y;
        }
        if (FL & kInitRs) {
          const double2 rv = Rs[row * ldr + c];
          const double sc = rscale[c];
          t.x += sc * rv.x;
          t.y += sc * rv.y;
        }
        v[cb][sp] = t;
      }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
        if (nv && cv[cb]) W[(2 * node + sp) * ldw + col[cb]] = v[cb][sp];
  }
}

// Nonlocal coefficients C' = alpha Delta P^H X for every atom; returns the
// device array [n_atoms][2 max_pj][n_vec] (in the scratch buffer), or null.
// Scratch: the caller's buffer (scratch, at least nonlocal_scratch_bytes(nl,
// n_vec) bytes) or the context's growable buffer.  alpha_d as in nl_delta_kernel.
// the packed complex contraction applies (at most 8 projectors per atom)
static bool pack_rows(const NonlocalK& nl) { return nl.max_pj <= 8; }

template <class T>
static const typename C2<T>::type* nonlocal_coeffs(chfsi_ctx* c, NonlocalK& nl,
                                                   const typename C2<T>::type* proj, const double2* X,
                                                   int64_t ldx, int n_vec, double alpha,
                                                   const double* alpha_d = nullptr, void* scratch = nullptr) {
  typedef typename C2<T>::type CT;
  if (nl.n_atoms == 0 || nl.n_entries == 0) return nullptr;
  const int mr = 2 * nl.max_pj;
  const size_t n_part = (size_t)nl.n_chunks * mr * n_vec;
  const size_t n_cp = (size_t)nl.n_atoms * mr * n_vec;
  const size_t bytes = (n_part + 2 * n_cp) * sizeof(CT);
  int group = n_vec;                      // columns per contraction launch
  if (!scratch && c->nl_fixed) {
    // fixed buffer: whole coefficient arrays, then as many columns of
    // partials per contraction launch as fit (the caller checked that one does)
    const size_t per_col = (size_t)nl.n_chunks * mr * sizeof(CT);
    const size_t head = 2 * n_cp * sizeof(CT);
    CHFSI_CHECK(c->nl_fixed_bytes >= head + per_col, CHFSI_EINVAL, "fixed nonlocal scratch too small");
    group = (int)std::min<size_t>(n_vec, (c->nl_fixed_bytes - head) / per_col);
    scratch = c->nl_fixed;
  } else if (!scratch) {
    c->scratch.alloc((bytes + sizeof(double) - 1) / sizeof(double));
    scratch = c->scratch.ptr;
  }
  CT* Csum = reinterpret_cast<CT*>(scratch);
  CT* Cp = Csum + n_cp;
  CT* partial = Cp + n_cp;
  double nl_flops = 0.0;
  for (const auto& at : nl.atoms)
    nl_flops += 2.0 * 8.0 * at.n_sup * at.n_pj * 2.0 * n_vec + 8.0 * 4.0 * at.n_pj * at.n_pj * n_vec;
  const double nl_bytes = (double)nl.n_entries * (2.0 * n_vec * sizeof(double2) + nl.max_pj * sizeof(CT));
  StageTimer tm(c, CHFSI_STAGE_NONLOCAL, nl_flops, nl_flops, nl_bytes);
  const int nct = cdiv(n_vec, 64);
  for (int c0 = 0; c0 < n_vec; c0 += group) {
    const int g = std::min(group, n_vec - c0);
    const int nct32 = cdiv(g, 16 * nl_col_blocks<T>());
    const int n_work = nl.n_chunks * nct32;
    const dim3 cgrid(8 * cdiv(cdiv(n_work, 4), 8));
    if (nl.real_proj)
      hipLaunchKernelGGL((nl_contract_kernel<T, true>), cgrid, dim3(256), 0, c->stream, proj, nl.sup_node.ptr,
                         nl.chunk_atom.ptr, nl.chunk_begin.ptr, nl.chunk_end.ptr, nl.chunk_order.ptr,
                         nl.atom_npj.ptr, nl.max_pj, n_work, nct32, X + c0, ldx, g, partial);
    else if (pack_rows(nl))
      hipLaunchKernelGGL((nl_contract_kernel<T, false, true>), cgrid, dim3(256), 0, c->stream, proj,
                         nl.sup_node.ptr, nl.chunk_atom.ptr, nl.chunk_begin.ptr, nl.chunk_end.ptr,
                         nl.chunk_order.ptr, nl.atom_npj.ptr, nl.max_pj, n_work, nct32, X + c0, ldx, g, partial);
    else
      hipLaunchKernelGGL((nl_contract_kernel<T, false>), cgrid, dim3(256), 0, c->stream, proj, nl.sup_node.ptr,
                         nl.chunk_atom.ptr, nl.chunk_begin.ptr, nl.chunk_end.ptr, nl.chunk_order.ptr,
                         nl.atom_npj.ptr, nl.max_pj, n_work, nct32, X + c0, ldx, g, partial);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(nl_reduce_kernel<T>, dim3(nl.n_atoms, mr, cdiv(g, 64)), dim3(64), 0, c->stream, partial,
                       nl.atom_chunk0.ptr, nl.atom_npj.ptr, nl.max_pj, g, n_vec, c0, Csum);
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(nl_delta_kernel<T>, dim3(nl.n_atoms, nct), dim3(64), 0, c->stream, Csum,
                     nl.atom_npj.ptr, nl.delta.ptr, nl.max_pj, n_vec, alpha, alpha_d, Cp);
  LAUNCH_CHECK();
  return Cp;
}

template <class T>
static void init_and_backproduct(chfsi_ctx* c, NonlocalK& nl, const typename C2<T>::type* proj,
                                 const typename C2<T>::type* Cp, const double2* X, int64_t ldx,
                                 double2* W, int64_t ldw, const double2* Wold, int64_t ldo, int n_vec,
                                 double beta, double gamma, const double2* Rs = nullptr, int64_t ldr = 0,
                                 const double* rscale = nullptr, const double* bg_d = nullptr) {
  const int64_t rows = 2 * c->n_nodes;
  StageTimer tm(c, CHFSI_STAGE_AXPY, Cp ? 8.0 * 2.0 * nl.n_entries * nl.max_pj * n_vec : 0.0, 0.0,
                (double)rows * n_vec * sizeof(double2) * (1.0 + (beta != 0.0) + (gamma != 0.0)));
  const int has = Cp != nullptr;
  const int64_t n_runs = (c->n_nodes + kNlRun - 1) / kNlRun;
  const int nct = cdiv(n_vec, 16 * nl_col_blocks<T>());
  const int n_work = (int)(n_runs * nct);
  const int fl = (beta != 0.0 ? kInitBeta : 0) | (gamma != 0.0 ? kInitGamma : 0) | (Rs ? kInitRs : 0);
  const dim3 grid(cdiv(n_work, 4)), blk(256);
#define INIT_NL_ARGS                                                                                      \
  proj, has ? nl.run_off.ptr : nullptr, has ? nl.pair_atom.ptr : nullptr, has ? nl.pair_ent.ptr : nullptr, \
      has ? nl.atom_npj.ptr : nullptr, nl.max_pj, Cp, has, X, ldx, W, ldw, Wold, ldo, Rs, ldr, rscale,    \
      c->n_nodes, n_work, nct, n_vec, beta, gamma, bg_d
#define INIT_NL_CASE(F)                                                                        \
  case F:                                                                                      \
    if (has && nl.real_proj)                                                                   \
      hipLaunchKernelGGL((init_nl_kernel<T, F, true>), grid, blk, 0, c->stream, INIT_NL_ARGS);  \
    else                                                                                       \
      hipLaunchKernelGGL((init_nl_kernel<T, F, false>), grid, blk, 0, c->stream, INIT_NL_ARGS); \
    break;
  switch (fl) {
    INIT_NL_CASE(0)
    INIT_NL_CASE(1)
    INIT_NL_CASE(2)
    INIT_NL_CASE(3)
    INIT_NL_CASE(4)
    INIT_NL_CASE(5)
    INIT_NL_CASE(6)
    default:
    INIT_NL_CASE(7)
  }
#undef INIT_NL_CASE
#undef INIT_NL_ARGS
  LAUNCH_CHECK();
}

void apply_H3(chfsi_ctx* c, KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw,
              const double2* Wold, int64_t ldo, int n_vec, int prec, double alpha, double beta, double gamma,
              const double2* Rs, int64_t ldr, const double* rscale) {
  if (prec == CHFSI_PREC_MIXED) {
    const float2* Cp = nonlocal_coeffs<float>(c, kp.nl, kp.nl.proj32.ptr, X, ldx, n_vec, alpha);
    init_and_backproduct<float>(c, kp.nl, kp.nl.proj32.ptr, Cp, X, ldx, W, ldw, Wold, ldo, n_vec, beta, gamma,
                                Rs, ldr, rscale);
  } else {
    const double2* Cp = nonlocal_coeffs<double>(c, kp.nl, kp.nl.proj.ptr, X, ldx, n_vec, alpha);
    init_and_backproduct<double>(c, kp.nl, kp.nl.proj.ptr, Cp, X, ldx, W, ldw, Wold, ldo, n_vec, beta, gamma,
                                 Rs, ldr, rscale);
  }
  if (c->form == CHFSI_FORM_MATRIX_FREE) {
    launch_mf_products(c, kp, prec, X, ldx, W, ldw, n_vec, alpha);
  } else {
    launch_cell_products(c, kp, prec, X, ldx, W, ldw, n_vec, alpha);
  }
}

void apply_H2(chfsi_ctx* c, KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw,
              const double2* Wold, int64_t ldo, int n_vec, int prec, double alpha, double beta,
              double gamma) {
  apply_H3(c, kp, X, ldx, W, ldw, Wold, ldo, n_vec, prec, alpha, beta, gamma, nullptr, 0, nullptr);
}

// Y[r][n] = a[n] Y[r][n] + b[n] X[r][n]   (per-column scalars on the device)
__global__ void cols_axpby_kernel(double2* __restrict__ Y, int64_t ldy, const double2* __restrict__ X, int64_t ldx,
                                  int64_t rows, int n_vec, const double* __restrict__ a, const double* __restrict__ b) {
  const int64_t total = rows * n_vec;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n_vec;
    const int n = (int)(t - r * n_vec);
    const double2 y = Y[r * ldy + n], x = X[r * ldx + n];
    Y[r * ldy + n] = double2{a[n] * y.x + b[n] * x.x, a[n] * y.y + b[n] * x.y};
  }
}

void launch_cols_axpby(chfsi_ctx* c, double2* Y, int64_t ldy, const double2* X, int64_t ldx, int64_t rows,
                       int n_vec, const double* a_d, const double* b_d) {
  const int64_t total = rows * n_vec;
  const int blocks = (int)std::min<int64_t>(cdiv(total, 256), 8192);
  StageTimer tm(c, CHFSI_STAGE_AXPY, 0.0, 0.0, 3.0 * (double)total * sizeof(double2));
  hipLaunchKernelGGL(cols_axpby_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, c->stream, Y, ldy, X, ldx, rows,
                     n_vec, a_d, b_d);
  LAUNCH_CHECK();
}

void apply_H(chfsi_ctx* c, KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw,
             int n_vec, int prec, double alpha, double beta, double gamma) {
  apply_H2(c, kp, X, ldx, W, ldw, W, ldw, n_vec, prec, alpha, beta, gamma);
}

// ---------------------------------------------------------------- batched support
void apply_nonlocal_init(chfsi_ctx* c, KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw,
                         int n_vec, int prec, double alpha, double beta, double gamma, const double* alpha_d,
                         const double* bg_d, void* scratch) {
  if (prec == CHFSI_PREC_MIXED) {
    const float2* Cp = nonlocal_coeffs<float>(c, kp.nl, kp.nl.proj32.ptr, X, ldx, n_vec, alpha, alpha_d, scratch);
    init_and_backproduct<float>(c, kp.nl, kp.nl.proj32.ptr, Cp, X, ldx, W, ldw, W, ldw, n_vec, beta, gamma,
                                nullptr, 0, nullptr, bg_d);
  } else {
    const double2* Cp = nonlocal_coeffs<double>(c, kp.nl, kp.nl.proj.ptr, X, ldx, n_vec, alpha, alpha_d, scratch);
    init_and_backproduct<double>(c, kp.nl, kp.nl.proj.ptr, Cp, X, ldx, W, ldw, W, ldw, n_vec, beta, gamma,
                                 nullptr, 0, nullptr, bg_d);
  }
}

size_t nonlocal_scratch_bytes_min(const KPoint& kp, int n_vec) {
  const NonlocalK& nl = kp.nl;
  if (nl.n_atoms == 0 || nl.n_entries == 0) return 0;
  const size_t mr = 2 * nl.max_pj;
  return ((size_t)nl.n_chunks * mr + 2 * (size_t)nl.n_atoms * mr * n_vec) * sizeof(double2);
}

size_t nonlocal_scratch_bytes(const KPoint& kp, int n_vec) {
  const NonlocalK& nl = kp.nl;
  if (nl.n_atoms == 0 || nl.n_entries == 0) return 0;
  const size_t mr = 2 * nl.max_pj;
  const size_t n = (size_t)nl.n_chunks * mr * n_vec + 2 * (size_t)nl.n_atoms * mr * n_vec;
  return n * sizeof(double2);  // the larger of the two precisions
}

// ============================================================================
// Adjoint: fields at the quadrature points and their cross densities
// ============================================================================
// One block per (cell, group of columns).  For CC columns at a time, the
// M^{-1/2}-scaled cell rows of L and Y (both spins) are gathered into LDS and
// interpolated to the quadrature points by sum factorisation over x, y, z
// (N_i = l_ax l_ay l_az); each thread then owns up to four points and
// accumulates, over the group's columns,
//   Re l^H y,  Re l^H sigma_x y,  Re l^H sigma_y y,  Re l^H sigma_z y,
// written (times w_q J) to partial[group][cell][point][4]; a second kernel adds
// the groups in a fixed order into dV, dB.
constexpr int kCdMaxQ = 4;   // points per thread: nq^3 <= 1024
// NS = 4 streams (L up, L down, Y up, Y down), or NS = 2 when L = Y (densities:
// the block is gathered and interpolated once).  colw: per-column weights (the
// occupations) or null; wJ: multiply by w_q J (the adjoint pairing) or not (the
// densities themselves).
template <int NS>
__global__ __launch_bounds__(256) void cross_density_kernel(
    const double2* __restrict__ L, int64_t ldl, const double2* __restrict__ Y, int64_t ldy, int n_vec,
    const int32_t* __restrict__ cell_nodes, const double* __restrict__ minv_sqrt,
    const double* __restrict__ B1, const double* __restrict__ wq1, double J, int np1, int nq, int nloc,
    int maxsz, int CC, int cols_per_group, const double* __restrict__ colw, int wJ,
    double* __restrict__ partial) {
  extern __shared__ double2 sm[];
  double2* bufA = sm;                               // [CC*NS][maxsz]
  double2* bufB = sm + (size_t)CC * NS * maxsz;     // [CC*NS][maxsz]
  double* sBt = reinterpret_cast<double*>(bufB + (size_t)CC * NS * maxsz);   // [np1][nq]
  const int e = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
  const int nq3 = nq * nq * nq;
  const int c_begin = g * cols_per_group, c_end = min(n_vec, c_begin + cols_per_group);
  for (int t = tid; t < np1 * nq; t += 256) sBt[t] = B1[t];
  double acc[kCdMaxQ][4];
#pragma unroll
  for (int i = 0; i < kCdMaxQ; ++i) acc[i][0] = acc[i][1] = acc[i][2] = acc[i][3] = 0.0;
  const int32_t* nodes = cell_nodes + (size_t)e * nloc;
  for (int n0 = c_begin; n0 < c_end; n0 += CC) {
    // gather: stream s = 2 * operand + spin
    for (int t = tid; t < CC * NS * nloc; t += 256) {
      const int i = t % nloc, s = (t / nloc) % NS, cc = t / (NS * nloc);
      const int col = n0 + cc;
      double2 v = {0.0, 0.0};
      if (col < c_end) {
        const int64_t I = nodes[i];
        const int64_t r = 2 * I + (s & 1);
        const double sc = minv_sqrt[I];
        const double2 z = (s < 2) ? L[r * ldl + col] : Y[r * ldy + col];
        v.x = sc * z.x;
        v.y = sc * z.y;
      }
      bufA[(size_t)(cc * NS + s) * maxsz + i] = v;
    }
    __syncthreads();
    // x: T1[qx + nq (ay + np az)] = sum_ax l_ax(qx) Z[ax + np (ay + np az)]
    for (int t = tid; t < CC * NS * nq * np1 * np1; t += 256) {
      const int o = t % (nq * np1 * np1), st = t / (nq * np1 * np1);
      const int qx = o % nq, rest = o / nq;
      const double2* in = bufA + (size_t)st * maxsz + rest * np1;
      double2 v = {0.0, 0.0};
      for (int ax = 0; ax < np1; ++ax) {
        const double b = sBt[ax * nq + qx];
        v.x += b * in[ax].x;
        v.y += b * in[ax].y;
      }
      bufB[(size_t)st * maxsz + o] = v;
    }
    __syncthreads();
    // y: T2[qx + nq (qy + nq az)] = sum_ay l_ay(qy) T1[qx + nq (ay + np az)]
    for (int t = tid; t < CC * NS * nq * nq * np1; t += 256) {
      const int o = t % (nq * nq * np1), st = t / (nq * nq * np1);
      const int qx = o % nq, qy = (o / nq) % nq, az = o / (nq * nq);
      const double2* in = bufB + (size_t)st * maxsz;
      double2 v = {0.0, 0.0};
      for (int ay = 0; ay < np1; ++ay) {
        const double b = sBt[ay * nq + qy];
        const double2 z = in[qx + nq * (ay + np1 * az)];
        v.x += b * z.x;
        v.y += b * z.y;
      }
      bufA[(size_t)st * maxsz + o] = v;
    }
    __syncthreads();
    // z: Zq[qx + nq (qy + nq qz)] = sum_az l_az(qz) T2[qx + nq (qy + nq az)]
    for (int t = tid; t < CC * NS * nq3; t += 256) {
      const int o = t % nq3, st = t / nq3;
      const int qxy = o % (nq * nq), qz = o / (nq * nq);
      const double2* in = bufA + (size_t)st * maxsz;
      double2 v = {0.0, 0.0};
      for (int az = 0; az < np1; ++az) {
        const double b = sBt[az * nq + qz];
        const double2 z = in[qxy + nq * nq * az];
        v.x += b * z.x;
        v.y += b * z.y;
      }
      bufB[(size_t)st * maxsz + o] = v;
    }
    __syncthreads();
#pragma unroll
    for (int qi = 0; qi < kCdMaxQ; ++qi) {
      const int q = tid + 256 * qi;
      if (q >= nq3) continue;
      for (int cc = 0; cc < CC; ++cc) {
        if (n0 + cc >= c_end) break;
        const double cw = colw ? colw[n0 + cc] : 1.0;
        const double2 l0 = bufB[(size_t)(cc * NS + 0) * maxsz + q], l1 = bufB[(size_t)(cc * NS + 1) * maxsz + q];
        const double2 y0 = bufB[(size_t)(cc * NS + NS - 2) * maxsz + q];
        const double2 y1 = bufB[(size_t)(cc * NS + NS - 1) * maxsz + q];
        // conj(l_a) y_b = (lr - i li)(yr + i yi)
        const double r00 = l0.x * y0.x + l0.y * y0.y, i00 = l0.x * y0.y - l0.y * y0.x;
        const double r11 = l1.x * y1.x + l1.y * y1.y, i11 = l1.x * y1.y - l1.y * y1.x;
        const double r01 = l0.x * y1.x + l0.y * y1.y, i01 = l0.x * y1.y - l0.y * y1.x;
        const double r10 = l1.x * y0.x + l1.y * y0.y, i10 = l1.x * y0.y - l1.y * y0.x;
        (void)i00;
        (void)i11;
        acc[qi][0] += cw * (r00 + r11);   // 1
        acc[qi][1] += cw * (r01 + r10);   // sigma_x
        acc[qi][2] += cw * (i01 - i10);   // sigma_y: Re(conj(l0)(-i y1) + conj(l1)(i y0))
        acc[qi][3] += cw * (r00 - r11);   // sigma_z
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int qi = 0; qi < kCdMaxQ; ++qi) {
    const int q = tid + 256 * qi;
    if (q >= nq3) continue;
    const int qx = q % nq, qy = (q / nq) % nq, qz = q / (nq * nq);
    const double w = wJ ? wq1[qx] * wq1[qy] * wq1[qz] * J : 1.0;
    double* out = partial + (((size_t)g * gridDim.x + e) * nq3 + q) * 4;
#pragma unroll
    for (int d = 0; d < 4; ++d) out[d] = w * acc[qi][d];
  }
}

// dV[e][q] += alpha sum_g partial[g][e][q][0], dB[e][q][d] += alpha sum_g partial[g][e][q][1 + d]
__global__ void cross_density_reduce_kernel(const double* __restrict__ partial, int64_t n_points, int n_groups,
                                            double alpha, double* __restrict__ dV, double* __restrict__ dB) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_points;
       p += (int64_t)gridDim.x * blockDim.x) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < n_groups; ++g)
#pragma unroll
      for (int d = 0; d < 4; ++d) s[d] += partial[((size_t)g * n_points + p) * 4 + d];
    dV[p] += alpha * s[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) dB[p * 3 + d] += alpha * s[1 + d];
  }
}

// The same sums with n_q = n_p by sum factorisation.  A workgroup of 512
// threads owns one cell and a group of columns, and walks the group in chunks of
// CW columns of NS streams (NF = NS CW = 8 fields, one LDS buffer of n_p^3
// complex values per field: 44 KB at n_p = 7, two workgroups per CU).  Per chunk
// each thread loads the z-lines of its (column, stream, line) tasks straight into
// registers (column fastest, so neighbouring lanes read one row), interpolates
// along z there, and the y and x passes run in place in LDS; the next chunk's
// z-lines are loaded while the current chunk runs its LDS phases (LDS-only
// barriers).  tab = the matrix-free tables [B][Dq][w][even-odd tables].
// The n_groups column groups are interleaved (group g takes the chunks g,
// g + n_groups, ...) and n_groups is a multiple of the chunks that share a
// 128-byte row line, so the groups of one cell, neighbouring work items on one
// XCD, read the pieces of each line at the same time.  Work item bid -> column
// group bid % n_groups, cell order[bid / n_groups] (the densities' tiled order).
constexpr int kQfThreads = 512;
constexpr int qf_fields(int) { return 8; }

template <int NP, int NS>
__global__ __launch_bounds__(kQfThreads) void qfield_sf_kernel(
    const double2* __restrict__ L, int64_t ldl, const double2* __restrict__ Y, int64_t ldy, int n_vec,
    const int32_t* __restrict__ cell_nodes, const double* __restrict__ minv_sqrt, const double* __restrict__ tab,
    double J, int n_cells, int n_groups, const int32_t* __restrict__ order, const double* __restrict__ colw,
    int wJ, double* __restrict__ partial) {
  constexpr int NT = kQfThreads;
  constexpr int NF = qf_fields(NP), CW = NF / NS;
  constexpr int N2 = NP * NP, N3 = N2 * NP;
  constexpr int NTASK = NF * N2, TPT = (NTASK + NT - 1) / NT;
  constexpr int QPT = (N3 + NT - 1) / NT;
  extern __shared__ double2 qf_sm[];
  double2* buf = qf_sm;                 // [CW][NS][N3]
  const double* w1 = tab + 2 * N2;
  const double* eoBf = tab + 2 * N2 + NP;    // even-odd table of B (sf_eo)
  const int total = n_cells * n_groups;
  const int per_xcd = (total + 7) / 8;
  const int bid = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (bid >= total) return;
  const int g = bid % n_groups, e = order[bid / n_groups], tid = threadIdx.x;
  const int c_end = n_vec, c_step = CW * n_groups;
  const int32_t* nodes = cell_nodes + (size_t)e * N3;

  // the thread's tasks: (column offset c, stream s = 2 operand + spin, z-line l);
  // row pointers and M^{-1/2} factors are fixed over the chunks
  const double2* row[TPT][NP];
  double sc[TPT][NP];
  int tcol[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int t = min(tid + NT * k, NTASK - 1);
    const int c = t % CW, s = (t / CW) % NS, l = t / (CW * NS);
    tcol[k] = c;
#pragma unroll
    for (int z = 0; z < NP; ++z) {
      const int64_t I = nodes[l + z * N2];
      const int64_t r = 2 * I + (s & 1);
      row[k][z] = (s < 2) ? L + r * ldl : Y + r * ldy;
      sc[k][z] = minv_sqrt[I];
    }
  }
  double2 zv[TPT][NP];
#pragma unroll
  for (int k = 0; k < TPT; ++k)
#pragma unroll
    for (int z = 0; z < NP; ++z) zv[k][z] = row[k][z][min(g * CW + tcol[k], c_end - 1)];

  double acc[QPT][4];
#pragma unroll
  for (int j = 0; j < QPT; ++j) acc[j][0] = acc[j][1] = acc[j][2] = acc[j][3] = 0.0;
  for (int n0 = g * CW; n0 < c_end; n0 += c_step) {
    double cwv[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) cwv[c] = (n0 + c < c_end) ? (colw ? colw[n0 + c] : 1.0) : 0.0;
    // interpolation along z in registers (zero past the last column)
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      const int t = tid + NT * k;
      if (t >= NTASK) break;
      const int c = t % CW, s = (t / CW) % NS, l = t / (CW * NS);
      const bool ok = n0 + c < c_end;
      double2 u[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const double f = ok ? sc[k][i] : 0.0;
        u[i] = double2{f * zv[k][i].x, f * zv[k][i].y};
      }
      double2* out = buf + (c * NS + s) * N3 + l;
      double2 r[NP];
      sf_eo<double, NP, false>(eoBf, u, r);
#pragma unroll
      for (int o = 0; o < NP; ++o) out[o * N2] = r[o];
    }
    if (n0 + c_step < c_end) {
#pragma unroll
      for (int k = 0; k < TPT; ++k)
#pragma unroll
        for (int z = 0; z < NP; ++z) zv[k][z] = row[k][z][min(n0 + c_step + tcol[k], c_end - 1)];
    }
    lds_barrier();
    sf_line_pass<NP, NF, 1, NT>(eoBf, buf, buf);
    lds_barrier();
    sf_line_pass<NP, NF, 0, NT>(eoBf, buf, buf);
    lds_barrier();
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
      const int q = tid + NT * j;
      if (q >= N3) continue;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const double cw = cwv[c];
        const double2 l0 = buf[(c * NS + 0) * N3 + q], l1 = buf[(c * NS + 1) * N3 + q];
        const double2 y0 = buf[(c * NS + NS - 2) * N3 + q], y1 = buf[(c * NS + NS - 1) * N3 + q];
        const double r00 = l0.x * y0.x + l0.y * y0.y;
        const double r11 = l1.x * y1.x + l1.y * y1.y;
        const double r01 = l0.x * y1.x + l0.y * y1.y, i01 = l0.x * y1.y - l0.y * y1.x;
        const double r10 = l1.x * y0.x + l1.y * y0.y, i10 = l1.x * y0.y - l1.y * y0.x;
        acc[j][0] += cw * (r00 + r11);
        acc[j][1] += cw * (r01 + r10);
        acc[j][2] += cw * (i01 - i10);
        acc[j][3] += cw * (r00 - r11);
      }
    }
    lds_barrier();   // the next chunk overwrites the buffer
  }
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int q = tid + NT * j;
    if (q >= N3) continue;
    const double w = wJ ? J * w1[q % NP] * w1[(q / NP) % NP] * w1[q / N2] : 1.0;
    double* out = partial + (((size_t)g * n_cells + e) * N3 + q) * 4;
#pragma unroll
    for (int d = 0; d < 4; ++d) out[d] = w * acc[j][d];
  }
}

// Densities (one operand, two spins) with n_q = n_p: a workgroup of 512 threads
// owns one cell and one of n_groups interleaved column groups (group g takes the
// chunks of DC = 4 columns g, g + n_groups, ...) and walks it chunk by chunk,
// both spins at once (8 LDS fields of n_p^3 values, 44 KB at n_p = 7).  A
// chunk's z-line loads cover 4 consecutive columns of a row, half a 128-byte
// line: the group holding the other half is the neighbouring work item, which
// runs at the same time on the same XCD, so each line is fetched once.
// M^{-1/2} at the cell's nodes sits in LDS, so the kernel stays within 128
// VGPRs at n_p <= 7 and two workgroups share a CU.  The LDS fields are padded
// (den_px, den_fp: x extent and field gap per n_p) so that the eight lanes of
// a 128-bit LDS access hit distinct banks in the line passes (at n_p = 7 the
// compact layout puts two lanes of every eight on one bank in the y pass).  The next chunk's z-lines are
// loaded while the current one runs its LDS phases (LDS-only barriers).  Work
// item bid -> column group bid % n_groups, cell order[bid / n_groups] (4x4x4
// tiles of cells, tile after tile; each XCD takes a contiguous range, so the
// workgroups resident on an XCD hold a compact block of cells and their shared
// face nodes meet in its L2).  Output as qfield_sf_kernel (no quadrature weights).
constexpr int kDenCols = 4;
constexpr int kDenTile = 4;
constexpr int den_px(int NP) { return NP <= 3 ? NP : NP <= 6 ? 7 : 9; }
constexpr int den_fp(int NP) {
  return NP == 2 ? 1 : NP == 4 ? 1 : NP == 5 ? 6 : NP == 6 ? 11 : NP == 8 ? 1 : NP == 9 ? 6 : 0;
}
constexpr int den_field(int NP) { return den_px(NP) * NP * NP + den_fp(NP); }

template <int NP>
__global__ __launch_bounds__(kQfThreads) void density_sf_kernel(
    const double2* __restrict__ X, int64_t ldx, int n_vec, const int32_t* __restrict__ cell_nodes,
    const int32_t* __restrict__ order, const double* __restrict__ minv_sqrt, const double* __restrict__ tab,
    int n_cells, int n_groups, const double* __restrict__ colw, double* __restrict__ partial) {
  constexpr int NT = kQfThreads, DC = kDenCols, NF = 2 * DC;
  constexpr int N2 = NP * NP, N3 = N2 * NP;
  constexpr int NTASK = NF * N2, TPT = (NTASK + NT - 1) / NT;
  constexpr int QPT = (N3 + NT - 1) / NT;
  constexpr int SY = den_px(NP), SZ = SY * NP, SF = den_field(NP);
  static_assert(SY >= NP && (NP - 1) * (1 + SY + SZ) < SF, "padded field layout overlaps");
  extern __shared__ double2 den_sm[];
  double2* buf = den_sm;                                    // [DC][2 spins][SF]
  double* ssc = reinterpret_cast<double*>(buf + NF * SF);   // [N3] M^{-1/2} at the cell's nodes
  const double* eoBf = tab + 2 * N2 + NP;
  const int total = n_cells * n_groups;
  const int per_xcd = (total + 7) / 8;
  const int bid = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (bid >= total) return;
  const int g = bid % n_groups, e = order[bid / n_groups], tid = threadIdx.x;
  const int c_end = n_vec, c_step = DC * n_groups;
  const int32_t* nodes = cell_nodes + (size_t)e * N3;
  for (int i = tid; i < N3; i += NT) ssc[i] = minv_sqrt[nodes[i]];

  // the thread's z-line tasks: column offset c fastest, then the spin, then the line
  int32_t nd[TPT][NP];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int t = min(tid + NT * k, NTASK - 1);
    const int l = t / NF;
#pragma unroll
    for (int z = 0; z < NP; ++z) nd[k][z] = nodes[l + z * N2];
  }
  auto zload = [&](int n0, double2 (&zv)[TPT][NP]) {
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      const int t = min(tid + NT * k, NTASK - 1);
      const int col = min(n0 + t % DC, c_end - 1);
      const int sp = (t / DC) & 1;
#pragma unroll
      for (int z = 0; z < NP; ++z) zv[k][z] = X[(2 * (int64_t)nd[k][z] + sp) * ldx + col];
    }
  };
  double2 zv[TPT][NP];
  zload(g * DC, zv);
  double acc[QPT][4];
#pragma unroll
  for (int j = 0; j < QPT; ++j) acc[j][0] = acc[j][1] = acc[j][2] = acc[j][3] = 0.0;
  lds_barrier();                          // ssc is written
  for (int n0 = g * DC; n0 < c_end; n0 += c_step) {
    // z interpolation in registers (zero past the last column) into LDS
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      const int t = tid + NT * k;
      if (t >= NTASK) break;
      const int c = t % DC, sp = (t / DC) & 1, l = t / NF;
      const bool ok = n0 + c < c_end;
      double2 u[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const double f = ok ? ssc[l + i * N2] : 0.0;
        u[i] = double2{f * zv[k][i].x, f * zv[k][i].y};
      }
      double2* out = buf + (2 * c + sp) * SF + (l % NP) + (l / NP) * SY;
      double2 r[NP];
      sf_eo<double, NP, false>(eoBf, u, r);
#pragma unroll
      for (int o = 0; o < NP; ++o) out[o * SZ] = r[o];
    }
    if (n0 + c_step < c_end) zload(n0 + c_step, zv);
    lds_barrier();
    sf_line_pass<NP, NF, 1, NT, double, SY, SZ, SF>(eoBf, buf, buf);
    lds_barrier();
    sf_line_pass<NP, NF, 0, NT, double, SY, SZ, SF>(eoBf, buf, buf);
    lds_barrier();
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
      const int q = tid + NT * j;
      if (q >= N3) continue;
      const int pq = (q % NP) + ((q / NP) % NP) * SY + (q / N2) * SZ;
#pragma unroll
      for (int c = 0; c < DC; ++c) {
        const double cw = (n0 + c < c_end) ? (colw ? colw[n0 + c] : 1.0) : 0.0;
        const double2 u0 = buf[(2 * c) * SF + pq], u1 = buf[(2 * c + 1) * SF + pq];
        const double r00 = u0.x * u0.x + u0.y * u0.y;
        const double r11 = u1.x * u1.x + u1.y * u1.y;
        const double r01 = u0.x * u1.x + u0.y * u1.y, i01 = u0.x * u1.y - u0.y * u1.x;
        acc[j][0] += cw * (r00 + r11);
        acc[j][1] += cw * (2.0 * r01);       // u^H sigma_x u
        acc[j][2] += cw * (2.0 * i01);       // u^H sigma_y u
        acc[j][3] += cw * (r00 - r11);       // u^H sigma_z u
      }
    }
    lds_barrier();   // the next round overwrites the buffer
  }
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int q = tid + NT * j;
    if (q >= N3) continue;
    double* out = partial + (((size_t)g * n_cells + e) * N3 + q) * 4;
#pragma unroll
    for (int d = 0; d < 4; ++d) out[d] = acc[j][d];
  }
}

// The cell order of density_sf_kernel: tiles of kDenTile^3 cells (ragged at
// the edges), tile after tile, cells within a tile x fastest.
static void den_order_prepare(chfsi_ctx* c) {
  if (c->den_order.ptr && c->den_order.n == (size_t)c->n_cells) return;
  constexpr int T = kDenTile;
  std::vector<int32_t> ord;
  ord.reserve(c->n_cells);
  const int nx = c->nc[0], ny = c->nc[1], nz = c->nc[2];
  for (int tz = 0; tz < nz; tz += T)
    for (int ty = 0; ty < ny; ty += T)
      for (int tx = 0; tx < nx; tx += T)
        for (int z = tz; z < std::min(nz, tz + T); ++z)
          for (int y = ty; y < std::min(ny, ty + T); ++y)
            for (int x = tx; x < std::min(nx, tx + T); ++x) ord.push_back(x + nx * (y + ny * z));
  CHFSI_CHECK((int64_t)ord.size() == c->n_cells, CHFSI_EINVAL, "densities: cell order does not cover the mesh");
  c->den_order.release();
  c->den_order.upload(ord.data(), ord.size(), c->stream);
  CHFSI_HIP(hipStreamSynchronize(c->stream));   // the host vector ends here
}

template <int NP>
static void launch_density_sf(chfsi_ctx* c, const double2* X, int64_t ldx, int n_vec, const double* colw,
                              double* rho, double* mag) {
  constexpr int DC = kDenCols;
  constexpr int N3 = NP * NP * NP;
  const size_t sh = (size_t)2 * DC * den_field(NP) * sizeof(double2) + (size_t)N3 * sizeof(double);
  if (c->mf_tab.n == 0) mf_prepare(c);
  den_order_prepare(c);
  // at least two groups (the two halves of each 128-byte row line), more on
  // small meshes to fill the GPU; every group holds at least one chunk
  const int n_chunks = cdiv(n_vec, DC);
  const int want = std::max(2, cdiv(4096, std::max(1, c->n_cells)));
  const int groups = std::max(1, std::min(n_chunks, want));
  const int64_t n_points = (int64_t)c->n_cells * c->nq3;
  c->cd_partial.alloc((size_t)groups * n_points * 4);
  const int64_t total = (int64_t)c->n_cells * groups;
  CHFSI_CHECK(total < (int64_t)1 << 30, CHFSI_EINVAL, "densities: too many work items");
  StageTimer tm(c, CHFSI_STAGE_AXPY, 0.0, 0.0, (double)c->n_cells * c->nloc * 2.0 * n_vec * sizeof(double2));
  hipLaunchKernelGGL((density_sf_kernel<NP>), dim3((unsigned)(8 * ((total + 7) / 8))), dim3(kQfThreads), sh,
                     c->stream, X, ldx, n_vec, c->cell_nodes.ptr, c->den_order.ptr, c->minv_sqrt.ptr,
                     c->mf_tab.ptr, c->n_cells, groups, colw, c->cd_partial.ptr);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(cross_density_reduce_kernel, dim3((unsigned)std::min<int64_t>(cdiv(n_points, 256), 4096)),
                     dim3(256), 0, c->stream, c->cd_partial.ptr, n_points, groups, 1.0, rho, mag);
  LAUNCH_CHECK();
}

template <int NP, int NS>
static void launch_qfield_sf(chfsi_ctx* c, const double2* L, int64_t ldl, const double2* Y, int64_t ldy,
                             int n_vec, const double* colw, int wJ, double alpha, double* dV, double* dB) {
  constexpr int CW = qf_fields(NP) / NS;
  const size_t sh = (size_t)qf_fields(NP) * NP * NP * NP * sizeof(double2);
  if (c->mf_tab.n == 0) mf_prepare(c);
  den_order_prepare(c);
  // a multiple of the chunks that share a 128-byte row line (8 complex values),
  // at least 4096 work items where the columns allow; each group holds a chunk
  constexpr int LQ = 8 / CW > 1 ? 8 / CW : 1;
  const int n_chunks = cdiv(n_vec, CW);
  const int want = LQ * cdiv(std::max(1, cdiv(4096, std::max(1, c->n_cells))), LQ);
  const int groups = std::max(1, std::min(n_chunks, want));
  const int64_t n_points = (int64_t)c->n_cells * c->nq3;
  c->cd_partial.alloc((size_t)groups * n_points * 4);
  const int64_t total = (int64_t)c->n_cells * groups;
  CHFSI_CHECK(total < (int64_t)1 << 30, CHFSI_EINVAL, "quadrature-point fields: too many work items");
  StageTimer tm(c, CHFSI_STAGE_AXPY, 0.0, 0.0, (double)NS / 2 * c->n_cells * c->nloc * 2.0 * n_vec * sizeof(double2));
  hipLaunchKernelGGL((qfield_sf_kernel<NP, NS>), dim3((unsigned)(8 * ((total + 7) / 8))), dim3(kQfThreads), sh,
                     c->stream, L, ldl, Y, ldy, n_vec, c->cell_nodes.ptr, c->minv_sqrt.ptr, c->mf_tab.ptr, c->J,
                     c->n_cells, groups, c->den_order.ptr, colw, wJ, c->cd_partial.ptr);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(cross_density_reduce_kernel, dim3((unsigned)std::min<int64_t>(cdiv(n_points, 256), 4096)),
                     dim3(256), 0, c->stream, c->cd_partial.ptr, n_points, groups, alpha, dV, dB);
  LAUNCH_CHECK();
}

// n_q = n_p: sum-factorised line passes; otherwise the general kernel below.
template <int NS>
static bool qfield_fast(chfsi_ctx* c, const double2* L, int64_t ldl, const double2* Y, int64_t ldy, int n_vec,
                        const double* colw, int wJ, double alpha, double* dV, double* dB) {
  if (c->nq != c->np1) return false;
  switch (c->np1) {
    case 2: launch_qfield_sf<2, NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB); return true;
    case 3: launch_qfield_sf<3, NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB); return true;
    case 4: launch_qfield_sf<4, NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB); return true;
    case 5: launch_qfield_sf<5, NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB); return true;
    case 6: launch_qfield_sf<6, NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB); return true;
    case 7: launch_qfield_sf<7, NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB); return true;
    case 8: launch_qfield_sf<8, NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB); return true;
    case 9: launch_qfield_sf<9, NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB); return true;
    default: return false;
  }
}

// Shared launcher: partial sums per (cell, column group), then the fixed-order
// group reduction adding alpha * (sums) into (dV, dB).
template <int NS>
static void launch_cross_density(chfsi_ctx* c, const double2* L, int64_t ldl, const double2* Y, int64_t ldy,
                                 int n_vec, const double* colw, int wJ, double alpha, double* dV, double* dB) {
  if (qfield_fast<NS>(c, L, ldl, Y, ldy, n_vec, colw, wJ, alpha, dV, dB)) return;
  const int np1 = c->np1, nq = c->nq;
  const int maxsz = std::max(std::max(c->nloc, nq * np1 * np1), std::max(nq * nq * np1, c->nq3));
  CHFSI_CHECK(c->nq3 <= 256 * kCdMaxQ, CHFSI_EINVAL, "quadrature-point fields support n_q <= 10");
  const size_t per_cc = 2 * NS * (size_t)maxsz * sizeof(double2);
  const size_t budget = 128 * 1024;
  const int CC = (int)std::max<size_t>(1, std::min<size_t>(4, budget / per_cc));
  const size_t sh = CC * per_cc + np1 * nq * sizeof(double);
  CHFSI_CHECK(sh <= 160 * 1024, CHFSI_EINVAL, "quadrature-point fields: cell too large for LDS");
  if (c->ref_b1.n == 0) {
    c->ref_b1.upload(c->ref.B.data(), c->ref.B.size(), c->stream);
    c->ref_wq.upload(c->ref.wq.data(), c->ref.wq.size(), c->stream);
  }
  // column groups: enough (cell, group) blocks to fill the GPU, whole CC chunks each
  const int max_groups = std::max(1, cdiv(n_vec, CC));
  const int want = std::max(1, cdiv(4096, std::max(1, c->n_cells)));
  int groups = std::min(max_groups, want);
  const int cpg = CC * cdiv(cdiv(n_vec, groups), CC);
  groups = cdiv(n_vec, cpg);
  const int64_t n_points = (int64_t)c->n_cells * c->nq3;
  c->cd_partial.alloc((size_t)groups * n_points * 4);
  StageTimer tm(c, CHFSI_STAGE_AXPY, 0.0, 0.0, (double)NS / 2 * c->n_cells * c->nloc * 2.0 * n_vec * sizeof(double2));
  hipLaunchKernelGGL(cross_density_kernel<NS>, dim3(c->n_cells, groups), dim3(256), sh, c->stream, L, ldl, Y,
                     ldy, n_vec, c->cell_nodes.ptr, c->minv_sqrt.ptr, c->ref_b1.ptr, c->ref_wq.ptr, c->J, np1, nq,
                     c->nloc, maxsz, CC, cpg, colw, wJ, c->cd_partial.ptr);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(cross_density_reduce_kernel, dim3((unsigned)std::min<int64_t>(cdiv(n_points, 256), 4096)),
                     dim3(256), 0, c->stream, c->cd_partial.ptr, n_points, groups, alpha, dV, dB);
  LAUNCH_CHECK();
}

void cross_density(chfsi_ctx* c, const double2* L, int64_t ldl, const double2* Y, int64_t ldy, int n_vec,
                   double alpha, double* dV, double* dB) {
  launch_cross_density<4>(c, L, ldl, Y, ldy, n_vec, nullptr, 1, alpha, dV, dB);
}

void densities(chfsi_ctx* c, const double2* X, int64_t ldx, int n_vec, const double* occ_d, double* rho,
               double* mag) {
  if (c->nq == c->np1) {
    switch (c->np1) {
      case 2: launch_density_sf<2>(c, X, ldx, n_vec, occ_d, rho, mag); return;
      case 3: launch_density_sf<3>(c, X, ldx, n_vec, occ_d, rho, mag); return;
      case 4: launch_density_sf<4>(c, X, ldx, n_vec, occ_d, rho, mag); return;
      case 5: launch_density_sf<5>(c, X, ldx, n_vec, occ_d, rho, mag); return;
      case 6: launch_density_sf<6>(c, X, ldx, n_vec, occ_d, rho, mag); return;
      case 7: launch_density_sf<7>(c, X, ldx, n_vec, occ_d, rho, mag); return;
      case 8: launch_density_sf<8>(c, X, ldx, n_vec, occ_d, rho, mag); return;
      case 9: launch_density_sf<9>(c, X, ldx, n_vec, occ_d, rho, mag); return;
      default: break;
    }
  }
  launch_cross_density<2>(c, X, ldx, X, ldx, n_vec, occ_d, 0, 1.0, rho, mag);
}

// ============================================================================
// Dense tall-skinny products (FP64 MFMA) for CholGS and Rayleigh-Ritz
// ============================================================================
// Both products run on one LDS-staged tile engine: workgroup tile 128 x 64
// complex outputs, 4 waves of 64 x 32 (4 x 2 blocks of 16 x 16, 4 real MFMAs
// per complex block and k-step of 4), k staged through LDS in double-buffered
// stages of 8, k-major ([k][m] and [k][n]) so that every fragment read is 16
// consecutive complex values.  The next stage's global loads are issued before
// the current stage's MFMAs.
constexpr int kGM = 128, kGN = 64, kGK = 8, kGPad = 2;   // pad: k rows 4 apart on other banks

struct GemmSmem {
  double2 a[2][kGK][kGM + kGPad];
  double2 b[2][kGK][kGN + kGPad];
};

// acc[mb][nb] (re, im) += op(A) B over one LDS stage; CONJ: op(A) = conj(A)
template <bool CONJ>
__device__ __forceinline__ void gemm_stage(const GemmSmem& sm, int buf, int wm, int wn, int lane, d4 (&cr)[4][2],
                                           d4 (&ci)[4][2]) {
  const int kl = lane >> 4, il = lane & 15;
#pragma unroll
  for (int ks = 0; ks < kGK / 4; ++ks) {
    double2 fa[4], fb[2];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) fa[mb] = sm.a[buf][ks * 4 + kl][wm * 64 + mb * 16 + il];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) fb[nb] = sm.b[buf][ks * 4 + kl][wn * 32 + nb * 16 + il];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const double ar = fa[mb].x, ai = CONJ ? -fa[mb].y : fa[mb].y, nai = -ai;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        cr[mb][nb] = mfma(ar, fb[nb].x, cr[mb][nb]);
        cr[mb][nb] = mfma(nai, fb[nb].y, cr[mb][nb]);
        ci[mb][nb] = mfma(ar, fb[nb].y, ci[mb][nb]);
        ci[mb][nb] = mfma(ai, fb[nb].x, ci[mb][nb]);
      }
    }
  }
}

// Partial S = X^H Y over chunks of rows, lower-triangle tiles only when asked.
// Work item = (tile, chunk group g); group g walks the row chunks g, g + G, ...
// and the items of one group are consecutive on one XCD, so the tiles reading
// the same rows share that XCD's L2.  partial[g] holds the group's n x n sum.
__global__ __launch_bounds__(256) void gram_kernel(const double2* __restrict__ X, int64_t ldx,
                                                   const double2* __restrict__ Y, int64_t ldy,
                                                   int64_t rows, int n, int64_t chunk_rows, int n_groups,
                                                   const int2* __restrict__ tiles, int n_tiles,
                                                   double2* __restrict__ partial) {
  __shared__ GemmSmem sm;
  const int n_work = n_tiles * n_groups;
  const int per_xcd = (int)((gridDim.x + 7) / 8);
  const int bid = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (bid >= n_work) return;              // uniform over the block, before any barrier
  const int g = bid / n_tiles;
  const int2 tl = tiles[bid - g * n_tiles];
  const int i0 = tl.x * kGM, j0 = tl.y * kGN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave & 1, wn = wave >> 1;
  // staging map: A 8 rows x 128 cols (4 per thread), B 8 rows x 64 cols (2 per thread);
  // slot u of a thread is column (tid & 31) + 32 u, so each LDS store writes 32
  // consecutive elements of a row (no bank conflicts) and each load reads 512 B
  const int ak = tid >> 5, am = tid & 31;
  const int bk = tid >> 5, bn = tid & 31;
  d4 cr[4][2], ci[4][2];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) cr[mb][nb] = ci[mb][nb] = d4{0, 0, 0, 0};
  const int64_t n_chunks = (rows + chunk_rows - 1) / chunk_rows;
  double2 pa[4], pb[2];
  auto gload = [&](int64_t r0, int64_t r_end) {
    const int64_t r = r0 + ak;
    const bool rv = r < r_end;
    const double2* xp = X + (rv ? r : 0) * ldx;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = i0 + am + 32 * u;
      pa[u] = (rv && c < n) ? xp[c] : double2{0.0, 0.0};
    }
    const int64_t rb = r0 + bk;
    const bool rbv = rb < r_end;
    const double2* yp = Y + (rbv ? rb : 0) * ldy;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int c = j0 + bn + 32 * u;
      pb[u] = (rbv && c < n) ? yp[c] : double2{0.0, 0.0};
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) sm.a[buf][ak][am + 32 * u] = pa[u];
#pragma unroll
    for (int u = 0; u < 2; ++u) sm.b[buf][bk][bn + 32 * u] = pb[u];
  };
  for (int64_t ch = g; ch < n_chunks; ch += n_groups) {
    const int64_t r_begin = ch * chunk_rows;
    const int64_t r_end = std::min<int64_t>(rows, r_begin + chunk_rows);
    const int nst = (int)((r_end - r_begin + kGK - 1) / kGK);
    __syncthreads();                      // previous chunk's last stage is read
    gload(r_begin, r_end);
    lstore(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
      const int buf = st & 1;
      const bool more = st + 1 < nst;
      if (more) gload(r_begin + (int64_t)(st + 1) * kGK, r_end);
      gemm_stage<true>(sm, buf, wm, wn, lane, cr, ci);
      if (more) lstore(buf ^ 1);          // that buffer was last read before the previous barrier
      __syncthreads();
    }
  }
  double2* out = partial + (size_t)g * n * n;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ri = i0 + wm * 64 + mb * 16 + acc_row<double>(lane, j);
        const int cj = j0 + wn * 32 + nb * 16 + (lane & 15);
        if (ri < n && cj < n) out[(size_t)ri * n + cj] = double2{cr[mb][nb][j], ci[mb][nb][j]};
      }
}

// S[i][j] = sum over groups of partial[g][i][j] for the (i, j) of the listed tiles
__global__ void gram_reduce_kernel(const double2* __restrict__ partial, int n_groups, int n,
                                   const int2* __restrict__ tiles, double2* __restrict__ S) {
  const int2 tl = tiles[blockIdx.x];
  for (int t = threadIdx.x; t < kGM * kGN; t += blockDim.x) {
    const int i = tl.x * kGM + t / kGN, j = tl.y * kGN + t % kGN;
    if (i >= n || j >= n) continue;
    double2 s = {0.0, 0.0};
    for (int g = 0; g < n_groups; ++g) {
      const double2 v = partial[((size_t)g * n + i) * n + j];
      s.x += v.x;
      s.y += v.y;
    }
    S[(size_t)i * n + j] = s;
  }
}

void gram(chfsi_ctx* c, const double2* X, int64_t ldx, const double2* Y, int64_t ldy, int64_t rows,
          int n, std::vector<cplx>& S, bool lower_only) {
  const int nti = cdiv(n, kGM), ntj = cdiv(n, kGN);
  std::vector<int2> tiles;
  for (int i = 0; i < nti; ++i)
    for (int j = 0; j < ntj; ++j)
      if (!lower_only || j * kGN < (i + 1) * kGM) tiles.push_back(int2{i, j});
  const int ntl = (int)tiles.size();
  // one resident round of work items (two 256-thread workgroups per CU at this
  // kernel's register use); row chunks of 256
  const int64_t chunk_rows = 256;
  const int64_t n_chunks = std::max<int64_t>(1, (rows + chunk_rows - 1) / chunk_rows);
  const int n_groups = (int)std::max<int64_t>(1, std::min<int64_t>(n_chunks, 512 / ntl));
  const size_t need = (size_t)n_groups * n * n + (size_t)n * n;   // double2 units
  c->scratch.alloc(2 * need + ntl);                               // + tiles (int2 = 1 double)
  double2* partial = reinterpret_cast<double2*>(c->scratch.ptr);
  double2* Sd = partial + (size_t)n_groups * n * n;
  int2* td = reinterpret_cast<int2*>(Sd + (size_t)n * n);
  CHFSI_HIP(hipMemcpyAsync(td, tiles.data(), ntl * sizeof(int2), hipMemcpyHostToDevice, c->stream));
  StageTimer tm(c, CHFSI_STAGE_GRAM, 8.0 * (double)rows * n * n * (lower_only ? 0.5 : 1.0),
                8.0 * (double)rows * kGM * kGN * ntl, 2.0 * (double)rows * n * sizeof(double2));
  const int n_work = ntl * n_groups;
  hipLaunchKernelGGL(gram_kernel, dim3(8 * cdiv(n_work, 8)), dim3(256), 0, c->stream, X, ldx, Y, ldy, rows, n,
                     chunk_rows, n_groups, td, ntl, partial);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(ntl), dim3(256), 0, c->stream, partial, n_groups, n, td, Sd);
  LAUNCH_CHECK();
  std::vector<double2> h((size_t)n * n);
  CHFSI_HIP(hipMemcpyAsync(h.data(), Sd, (size_t)n * n * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  S.resize((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (lower_only && j > i)
        S[(size_t)i * n + j] = std::conj(cplx(h[(size_t)j * n + i].x, h[(size_t)j * n + i].y));
      else
        S[(size_t)i * n + j] = cplx(h[(size_t)i * n + j].x, h[(size_t)i * n + j].y);
    }
}

// X[r0 + r][:] = P[r][:] Q over a row panel P (a copy of those rows).  upper:
// Q[k][j] = 0 for k > j, so the k range of a column tile ends at its last column;
// a workgroup then takes column tiles ct and n_ct - 1 - ct of its row tile in turn
// (equal work per workgroup: the k ranges of the pair add up to n + kGN).
// Work item = (row tile, column tile or pair), consecutive on one XCD, so the
// column tiles of one row tile read its panel rows through one L2.
__global__ __launch_bounds__(256) void rotate_kernel(const double2* __restrict__ P, int n,
                                                     int64_t prow, const double2* __restrict__ Q,
                                                     double2* __restrict__ X, int64_t ldx, int upper,
                                                     int n_rt, int n_ct) {
  __shared__ GemmSmem sm;
  const int n_cw = upper ? (n_ct + 1) / 2 : n_ct;    // column work items per row tile
  const int n_work = n_rt * n_cw;
  const int per_xcd = (int)((gridDim.x + 7) / 8);
  const int bid = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (bid >= n_work) return;              // uniform over the block, before any barrier
  const int rt = bid / n_cw, cw = bid - rt * n_cw;
  const int64_t r0 = (int64_t)rt * kGM;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave & 1, wn = wave >> 1;
  // staging map: A 128 panel rows x 8 k (4 consecutive k per thread, stored
  // k-major), B 8 rows of Q x 64 columns (columns (tid & 31) + 32 u)
  const int am = tid >> 1, ak = (tid & 1) * 4;
  const int bk = tid >> 5, bn = tid & 31;
  const int64_t ra = r0 + am;
  const bool rav = ra < prow;
  const double2* prow_p = P + (rav ? ra : 0) * (int64_t)n;
  const int n_pass = (upper && n_ct - 1 - cw != cw) ? 2 : 1;
  for (int pass = 0; pass < n_pass; ++pass) {
    const int ct = pass == 0 ? cw : n_ct - 1 - cw;
    const int j0 = ct * kGN;
    const int kend = upper ? std::min(n, j0 + kGN) : n;
    d4 cr[4][2], ci[4][2];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) cr[mb][nb] = ci[mb][nb] = d4{0, 0, 0, 0};
    double2 pa[4], pb[2];
    auto gload = [&](int k0) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + ak + u;
        pa[u] = (rav && k < kend) ? prow_p[k] : double2{0.0, 0.0};
      }
      const int kb = k0 + bk;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int cj = j0 + bn + 32 * u;
        pb[u] = (kb < kend && cj < n) ? Q[(size_t)kb * n + cj] : double2{0.0, 0.0};
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int u = 0; u < 4; ++u) sm.a[buf][ak + u][am] = pa[u];
#pragma unroll
      for (int u = 0; u < 2; ++u) sm.b[buf][bk][bn + 32 * u] = pb[u];
    };
    const int nst = (kend + kGK - 1) / kGK;
    if (pass > 0) __syncthreads();          // the previous tile's last stage has read sm
    gload(0);
    lstore(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
      const int buf = st & 1;
      const bool more = st + 1 < nst;
      if (more) gload((st + 1) * kGK);
      gemm_stage<false>(sm, buf, wm, wn, lane, cr, ci);
      if (more) lstore(buf ^ 1);
      __syncthreads();
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t r = r0 + wm * 64 + mb * 16 + acc_row<double>(lane, j);
          const int cj = j0 + wn * 32 + nb * 16 + (lane & 15);
          if (r < prow && cj < n) X[r * ldx + cj] = double2{cr[mb][nb][j], ci[mb][nb][j]};
        }
  }
}

void rotate_inplace(chfsi_ctx* c, double2* X, int64_t ldx, int64_t rows, int n, const std::vector<cplx>& Q,
                    bool upper) {
  // panel of rows copied to scratch, then multiplied back into place
  int64_t prow = std::max<int64_t>(kGM, ((int64_t)1 << 27) / ((int64_t)n * 16));   // <= 128 MiB
  prow = std::min<int64_t>(prow, rows);
  prow = (prow + kGM - 1) / kGM * kGM;
  c->panel.alloc((size_t)prow * n * 2 + (size_t)n * n * 2);
  double2* P = reinterpret_cast<double2*>(c->panel.ptr);
  double2* Qd = P + (size_t)prow * n;
  std::vector<double2> qh((size_t)n * n);
  for (size_t i = 0; i < qh.size(); ++i) qh[i] = double2{Q[i].real(), Q[i].imag()};
  CHFSI_HIP(hipMemcpyAsync(Qd, qh.data(), qh.size() * sizeof(double2), hipMemcpyHostToDevice, c->stream));
  StageTimer tm(c, CHFSI_STAGE_ROTATE, 8.0 * (double)rows * n * n * (upper ? 0.5 : 1.0),
                8.0 * (double)rows * n * n, 4.0 * (double)rows * n * sizeof(double2));
  for (int64_t r0 = 0; r0 < rows; r0 += prow) {
    const int64_t pr = std::min(prow, rows - r0);
    launch_copy_rows(c, P, n, X + r0 * ldx, ldx, pr, n);
    const int n_rt = cdiv(pr, kGM), n_ct = cdiv(n, kGN);
    const int n_cw = upper ? (n_ct + 1) / 2 : n_ct;
    const int grid = 8 * cdiv((int64_t)n_rt * n_cw, 8);
    hipLaunchKernelGGL(rotate_kernel, dim3(grid), dim3(256), 0, c->stream, P, n, pr, Qd, X + r0 * ldx, ldx,
                       upper ? 1 : 0, n_rt, n_ct);
    LAUNCH_CHECK();
  }
  CHFSI_HIP(hipStreamSynchronize(c->stream));   // qh leaves scope
}

// ============================================================================
// Reductions with a fixed grid (deterministic order)
// ============================================================================
constexpr int kRedGroups = 256;

__global__ __launch_bounds__(256) void resid_kernel(const double2* __restrict__ W, int64_t ldw,
                                                    const double2* __restrict__ X, int64_t ldx,
                                                    int64_t rows, int n, const double* __restrict__ theta,
                                                    double* __restrict__ partial) {
  __shared__ double red[256];
  const int g = blockIdx.x;
  const int col = blockIdx.y * 64 + (threadIdx.x & 63);
  const int lr = threadIdx.x >> 6;
  double s = 0.0;
  if (col < n) {
    const double th = theta[col];
    for (int64_t r = (int64_t)g * 4 + lr; r < rows; r += (int64_t)kRedGroups * 4) {
      const double2 w = W[r * ldw + col], x = X[r * ldx + col];
      const double dr = w.x - th * x.x, di = w.y - th * x.y;
      s += dr * dr + di * di;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 64 && col < n)
    partial[(size_t)g * n + col] = ((red[threadIdx.x] + red[threadIdx.x + 64]) + red[threadIdx.x + 128]) +
                                   red[threadIdx.x + 192];
}

void column_resid_norms(chfsi_ctx* c, const double2* W, int64_t ldw, const double2* X, int64_t ldx,
                        int64_t rows, int n, const double* theta, double* out) {
  c->scratch.alloc((size_t)kRedGroups * n + n);
  double* part = c->scratch.ptr;
  double* th = part + (size_t)kRedGroups * n;
  CHFSI_HIP(hipMemcpyAsync(th, theta, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(resid_kernel, dim3(kRedGroups, cdiv(n, 64)), dim3(256), 0, c->stream, W, ldw, X, ldx,
                     rows, n, th, part);
  LAUNCH_CHECK();
  std::vector<double> h((size_t)kRedGroups * n);
  CHFSI_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int g = 0; g < kRedGroups; ++g) s += h[(size_t)g * n + j];
    out[j] = std::sqrt(s);
  }
}

__global__ __launch_bounds__(256) void dot_kernel(const double2* __restrict__ x, const double2* __restrict__ y,
                                                  int64_t rows, double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t r = blockIdx.x * 256 + threadIdx.x; r < rows; r += (int64_t)kRedGroups * 256)
    s += x[r].x * y[r].x + x[r].y * y[r].y;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

double dot_re(chfsi_ctx* c, const double2* x, const double2* y, int64_t rows) {
  c->scratch.alloc(kRedGroups);
  hipLaunchKernelGGL(dot_kernel, dim3(kRedGroups), dim3(256), 0, c->stream, x, y, rows, c->scratch.ptr);
  LAUNCH_CHECK();
  double h[kRedGroups];
  CHFSI_HIP(hipMemcpyAsync(h, c->scratch.ptr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (int g = 0; g < kRedGroups; ++g) s += h[g];
  return s;
}

// ============================================================================
// Seeded fill (SplitMix64, counter form) and finiteness check
// ============================================================================
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void fill_random_kernel(double2* __restrict__ X, int64_t n_rows, int n_vec, int64_t ld,
                                   uint64_t seed, int64_t row0, int col0, int64_t ntc) {
  const int64_t total = n_rows * n_vec;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / n_vec;
    const int n = (int)(t - r * n_vec);
    const uint64_t j = (uint64_t)(row0 + r) * (uint64_t)ntc + (uint64_t)(col0 + n);
    const double ur = (double)(splitmix64_at(seed, 2 * j) >> 11) * (1.0 / 9007199254740992.0);
    const double ui = (double)(splitmix64_at(seed, 2 * j + 1) >> 11) * (1.0 / 9007199254740992.0);
    X[r * ld + n] = double2{2.0 * ur - 1.0, 2.0 * ui - 1.0};
  }
}

void launch_fill_random(chfsi_ctx* c, double2* X, int64_t n_rows, int n_vec, int64_t ld, uint64_t seed,
                        int64_t row0, int col0, int64_t ntc) {
  const int64_t total = n_rows * n_vec;
  const int blocks = (int)std::min<int64_t>(cdiv(total, 256), 8192);
  hipLaunchKernelGGL(fill_random_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, c->stream, X, n_rows,
                     n_vec, ld, seed, row0, col0, ntc);
  LAUNCH_CHECK();
}

__global__ void zero_int_kernel(int* __restrict__ f) { f[0] = 0; }

__global__ void nonfinite_kernel(const double* __restrict__ p, int64_t n, int* __restrict__ flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(p[i])) flag[0] = 1;
}

int check_finite(chfsi_ctx* c, const double* p, int64_t n) {
  c->scratch.alloc(1);
  int* flag = reinterpret_cast<int*>(c->scratch.ptr);
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, c->stream, flag);
  LAUNCH_CHECK();
  const int blocks = (int)std::min<int64_t>(cdiv(n, 256), 4096);
  hipLaunchKernelGGL(nonfinite_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, c->stream, p, n, flag);
  LAUNCH_CHECK();
  int h = 0;
  CHFSI_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  return h ? 0 : 1;
}

}  // namespace chfsi
