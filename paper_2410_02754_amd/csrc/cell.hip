// Cell-level operator: setup of the Pauli-form cell matrices and the fused
// gather / MFMA cell product / scatter-add kernels (Sec. IV.B, the
// cell-level dense products of the FE matrix-multivector product), per
// colour for one operator or as a persistent grid over a batch.
//
// Cell operator storage ("Pauli form"): the spinor cell matrix of
// eqn:FEHlocEl with the k-terms of eqn:FEHloc is, with every term scaled by
// M_D^{-1/2} on both sides,
//   [[A + Bz + iS, Bx - iBy], [Bx + iBy, A - Bz + iS]]
// with A = kinetic + |k|^2/2 mass + V-weighted mass and B_d the B_d-weighted
// masses (real symmetric) and S the skew-symmetrised k-gradient term (real
// antisymmetric, zero at Gamma).  Each cell stores the real matrices
// Hp = A + Bz, Hm = A - Bz, Bx, By (and S when k != 0) instead of the complex
// 2n x 2n matrix: half the bytes, and 12 instead of 16 real MFMAs per complex
// multiply-add block at Gamma.  Matrices are stored pre-tiled in MFMA
// A-operand order: [cell][row block of 16][k-step of 4][matrix][64 lanes].
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "mfma.h"

namespace chfsi {

// ============================================================================
// Cell operator setup
// ============================================================================
// One block per (cell, row block of 16).  Weighted masses by quadrature,
//   M_f[i][j] = sum_q w_q J f(r_q) N_i(r_q) N_j(r_q),  N_i = l_ax l_ay l_az,
// for f in {V, Bx, By, Bz}; then the scaled Pauli-form matrices.
__global__ __launch_bounds__(256) void cell_setup_kernel(
    const double* __restrict__ V, const double* __restrict__ B, const double* __restrict__ U0,
    const double* __restrict__ Sk, const double* __restrict__ minv_sqrt,
    const int32_t* __restrict__ cell_nodes, const double* __restrict__ B1,
    const double* __restrict__ wq1, double J, int np1, int nq, int nloc, int nrb, int nkb, int nmat,
    double* __restrict__ out) {
  extern __shared__ double smem[];
  const int nq3 = nq * nq * nq;
  double* sW = smem;                 // [4][nq3]
  double* sB1 = sW + 4 * nq3;        // [np1][nq]
  double* sS = sB1 + np1 * nq;       // [nloc] M^{-1/2} at the cell's nodes
  const int e = blockIdx.x, rb = blockIdx.y;
  for (int q = threadIdx.x; q < nq3; q += blockDim.x) {
    const int qx = q % nq, qy = (q / nq) % nq, qz = q / (nq * nq);
    const double wJ = wq1[qx] * wq1[qy] * wq1[qz] * J;
    sW[q] = wJ * V[(size_t)e * nq3 + q];
    for (int d = 0; d < 3; ++d) sW[(d + 1) * nq3 + q] = wJ * B[((size_t)e * nq3 + q) * 3 + d];
  }
  for (int t = threadIdx.x; t < np1 * nq; t += blockDim.x) sB1[t] = B1[t];
  for (int a = threadIdx.x; a < nloc; a += blockDim.x)
    sS[a] = minv_sqrt[cell_nodes[(size_t)e * nloc + a]];
  __syncthreads();
  const int npad = nkb * 4;
  for (int t = threadIdx.x; t < 16 * npad; t += blockDim.x) {
    const int il = t % 16, j = t / 16;
    const int i = rb * 16 + il;
    double mv = 0.0, mbx = 0.0, mby = 0.0, mbz = 0.0;
    const bool valid = (i < nloc) && (j < nloc);
    if (valid) {
      const int ax = i % np1, ay = (i / np1) % np1, az = i / (np1 * np1);
      const int bx = j % np1, by = (j / np1) % np1, bz = j / (np1 * np1);
      for (int qz = 0; qz < nq; ++qz) {
        const double ez = sB1[az * nq + qz] * sB1[bz * nq + qz];
        for (int qy = 0; qy < nq; ++qy) {
          const double eyz = ez * sB1[ay * nq + qy] * sB1[by * nq + qy];
          const int qb = nq * (qy + nq * qz);
          for (int qx = 0; qx < nq; ++qx) {
            const double ev = eyz * sB1[ax * nq + qx] * sB1[bx * nq + qx];
            const int q = qb + qx;
            mv += ev * sW[q];
            mbx += ev * sW[nq3 + q];
            mby += ev * sW[2 * nq3 + q];
            mbz += ev * sW[3 * nq3 + q];
          }
        }
      }
    }
    double vals[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (valid) {
      const double s = sS[i] * sS[j];
      const double a0 = U0[(size_t)i * nloc + j] + mv;
      vals[0] = s * (a0 + mbz);
      vals[1] = s * (a0 - mbz);
      vals[2] = s * mbx;
      vals[3] = s * mby;
      vals[4] = (nmat > 4) ? s * Sk[(size_t)i * nloc + j] : 0.0;
    }
    const int kb = j / 4, lane = (j % 4) * 16 + il;
    double* dst = out + (((size_t)e * nrb + rb) * nkb + kb) * nmat * 64 + lane;
    for (int m = 0; m < nmat; ++m) dst[m * 64] = vals[m];
  }
}

__global__ void f64_to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

void launch_cell_setup(chfsi_ctx* c, KPoint& kp, const double* V, const double* B, const double* U0,
                       const double* S) {
  const size_t per_cell = (size_t)c->nrb * c->nkb * kp.nmat * 64;
  kp.cell64.alloc(per_cell * c->n_cells);
  DevBuf<double> b1, wq;
  b1.upload(c->ref.B.data(), c->ref.B.size(), c->stream);
  wq.upload(c->ref.wq.data(), c->ref.wq.size(), c->stream);
  const size_t sh = (4 * (size_t)c->nq3 + c->np1 * c->nq + c->nloc) * sizeof(double);
  dim3 grid(c->n_cells, c->nrb);
  hipLaunchKernelGGL(cell_setup_kernel, grid, dim3(256), sh, c->stream, V, B, U0, S, c->minv_sqrt.ptr,
                     c->cell_nodes.ptr, b1.ptr, wq.ptr, c->J, c->np1, c->nq, c->nloc, c->nrb, c->nkb,
                     kp.nmat, kp.cell64.ptr);
  LAUNCH_CHECK();
  CHFSI_HIP(hipStreamSynchronize(c->stream));
}

void launch_cell_to_f32(chfsi_ctx* c, KPoint& kp) {
  const size_t n = kp.cell64.n;
  kp.cell32.alloc(n);
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(4096), dim3(256), 0, c->stream, kp.cell64.ptr, kp.cell32.ptr, n);
  LAUNCH_CHECK();
}

// ============================================================================
// Fused gather / cell product / scatter-add, one launch per colour
// ============================================================================
// Block = 4 waves as 2 (row blocks) x 2 (column halves).  Block tile: 32 local
// rows x BN = 32*CB columns of one cell.  K loop over the cell's local nodes in
// stages of 8 nodes: the gathered spinor rows (X_up = a + ib, X_dn = c + id)
// are staged in LDS as four planar real arrays, double-buffered, with the
// next stage's global loads issued before the current stage's MFMAs.  Each
// wave reads its A fragments (Hp, Hm, Bx, By, S) straight from the pre-tiled
// cell operator.  Per 4-node k-step and 16-column block the products are
//   Yup_r += Hp a + Bx c + By d - S b      Yup_i += Hp b + Bx d - By c + S a
//   Ydn_r += Hm c + Bx a - By b - S d      Ydn_i += Hm d + Bx b + By a + S c
template <class T, int CB>
struct CellSmem {
  static constexpr int BN = 32 * CB;
  static constexpr int BK = 8;
  static constexpr int PAD = 16;          // row pad: 4 k-rows of a fragment hit disjoint banks
  T sB[2][4][BK][BN + PAD];
  int32_t sNode[(kMaxP + 1) * (kMaxP + 1) * (kMaxP + 1)];
};

// One block tile of the fused gather / cell product / scatter-add for cell e,
// row tile rt (two 16-row blocks) and column tile ct.  Starts and ends with
// the block synchronised, so it can be called repeatedly by a persistent block.
template <class T, int CB, bool HAS_S>
__device__ __forceinline__ void cell_tile(CellSmem<T, CB>& sm, const T* __restrict__ cm,
                                          const int32_t* __restrict__ cell_nodes, int e, int rt, int ct,
                                          int nloc, int nrb, int nkb, int nmat,
                                          const double2* __restrict__ X, int64_t ldx,
                                          double2* __restrict__ W, int64_t ldw, int n_vec, double alpha) {
  typedef typename Vec4<T>::type V4;
  constexpr int BN = 32 * CB;
  constexpr int BK = 8;
  constexpr int NPRE = (BK * 2 * BN) / 256;
  constexpr int NM = HAS_S ? 5 : 4;
  auto& sB = sm.sB;
  auto& sNode = sm.sNode;
  __syncthreads();                        // previous tile's LDS reads are done

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 1, wc = wave >> 1;
  const int rb = rt * 2 + wr;
  const bool row_active = rb < nrb;
  // an inactive row block (odd nrb) computes on the last valid block and skips the epilogue,
  // so the stage loop below has no branches and loads overlap the MFMAs
  const int rb_eff = row_active ? rb : nrb - 1;
  const int col0 = ct * BN;

  for (int i = tid; i < nloc; i += 256) sNode[i] = cell_nodes[(size_t)e * nloc + i];
  __syncthreads();

  V4 acc[CB][4];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[cb][k] = V4{0, 0, 0, 0};

  const T* Abase = cm + ((size_t)(e * nrb + rb_eff) * nkb) * nmat * 64 + lane;
  const int nstage = nkb / 2;
  double2 pre[NPRE];
  T aC[2][NM], aN[2][NM];

  // per-thread constants of the gather: (k node, spin, column) of each prefetch slot
  int g_kk[NPRE], g_sp[NPRE], g_col[NPRE];
  bool g_cv[NPRE];
#pragma unroll
  for (int j = 0; j < NPRE; ++j) {
    const int idx = tid + 256 * j;
    g_col[j] = idx % BN;
    g_sp[j] = (idx / BN) & 1;
    g_kk[j] = idx / (2 * BN);
    g_cv[j] = col0 + g_col[j] < n_vec;
  }
  const int gcol_max = n_vec - 1;

  auto gload = [&](int s) {
#pragma unroll
    for (int j = 0; j < NPRE; ++j) {
      const int knode = s * BK + g_kk[j];
      const bool valid = g_cv[j] && knode < nloc;
      const int kn = knode < nloc ? knode : 0;                    // in-bounds address always
      const int gcol = min(col0 + g_col[j], gcol_max);
      const double2 v = X[(2 * (int64_t)sNode[kn] + g_sp[j]) * ldx + gcol];
      pre[j] = valid ? v : double2{0.0, 0.0};
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int j = 0; j < NPRE; ++j) {
      sB[buf][2 * g_sp[j]][g_kk[j]][g_col[j]] = (T)pre[j].x;
      sB[buf][2 * g_sp[j] + 1][g_kk[j]][g_col[j]] = (T)pre[j].y;
    }
  };
  auto aload = [&](int s, T (&dst)[2][NM]) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const T* Ap = Abase + (size_t)(s * 2 + kk) * nmat * 64;
#pragma unroll
      for (int m = 0; m < NM; ++m) dst[kk][m] = Ap[m * 64];
    }
  };

  aload(0, aC);
  gload(0);
  lstore(0);
  __syncthreads();
  for (int s = 0; s < nstage; ++s) {
    const int buf = s & 1;
    const int sn = s + 1 < nstage ? s + 1 : s;      // the last stage reloads itself (unused)
    gload(sn);
    aload(sn, aN);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const T hp = aC[kk][0], hm = aC[kk][1], bx = aC[kk][2], by = aC[kk][3];
      const T sv = HAS_S ? aC[kk][NM - 1] : (T)0;
      const T nby = -by, nsv = -sv;
      const int krow = kk * 4 + (lane >> 4);
      T ba[CB], bb[CB], bc[CB], bd[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int col = wc * (CB * 16) + cb * 16 + (lane & 15);
        ba[cb] = sB[buf][0][krow][col];
        bb[cb] = sB[buf][1][krow][col];
        bc[cb] = sB[buf][2][krow][col];
        bd[cb] = sB[buf][3][krow][col];
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        acc[cb][0] = mfma(hp, ba[cb], acc[cb][0]);
        acc[cb][1] = mfma(hp, bb[cb], acc[cb][1]);
        acc[cb][2] = mfma(hm, bc[cb], acc[cb][2]);
        acc[cb][3] = mfma(hm, bd[cb], acc[cb][3]);
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        acc[cb][0] = mfma(bx, bc[cb], acc[cb][0]);
        acc[cb][1] = mfma(bx, bd[cb], acc[cb][1]);
        acc[cb][2] = mfma(bx, ba[cb], acc[cb][2]);
        acc[cb][3] = mfma(bx, bb[cb], acc[cb][3]);
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        acc[cb][0] = mfma(by, bd[cb], acc[cb][0]);
        acc[cb][1] = mfma(nby, bc[cb], acc[cb][1]);
        acc[cb][2] = mfma(nby, bb[cb], acc[cb][2]);
        acc[cb][3] = mfma(by, ba[cb], acc[cb][3]);
      }
      if (HAS_S) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          acc[cb][0] = mfma(nsv, bb[cb], acc[cb][0]);
          acc[cb][1] = mfma(sv, ba[cb], acc[cb][1]);
          acc[cb][2] = mfma(nsv, bd[cb], acc[cb][2]);
          acc[cb][3] = mfma(sv, bc[cb], acc[cb][3]);
        }
      }
    }
    lstore(buf ^ 1);       // the other buffer was last read before the previous barrier
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int m = 0; m < NM; ++m) aC[kk][m] = aN[kk][m];
  }

  if (!row_active) return;                // (no barrier follows inside the tile)
  // epilogue: lane holds rows acc_row(lane, j), column lane%16 of each 16x16 tile
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int rl = rb * 16 + acc_row<T>(lane, j);
    if (rl >= nloc) continue;
    const int64_t node = sNode[rl];
    double2* w0 = W + (2 * node) * ldw;
    double2* w1 = W + (2 * node + 1) * ldw;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int gcol = col0 + wc * (CB * 16) + cb * 16 + (lane & 15);
      if (gcol >= n_vec) continue;
      double2 o0 = w0[gcol], o1 = w1[gcol];
      o0.x += alpha * (double)acc[cb][0][j];
      o0.y += alpha * (double)acc[cb][1][j];
      o1.x += alpha * (double)acc[cb][2][j];
      o1.y += alpha * (double)acc[cb][3][j];
      w0[gcol] = o0;
      w1[gcol] = o1;
    }
  }
}

template <class T, int CB, bool HAS_S>
__global__ __launch_bounds__(256) void cell_apply_kernel(
    const T* __restrict__ cm, const int32_t* __restrict__ cell_nodes,
    const int32_t* __restrict__ cells, int nloc, int nrb, int nkb, int nmat, int n_rowtiles,
    int n_coltiles, int n_work, const double2* __restrict__ X, int64_t ldx, double2* __restrict__ W,
    int64_t ldw, int n_vec, double alpha) {
  __shared__ CellSmem<T, CB> sm;
  // Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
  // XCD gets a contiguous range of (cell, row tile, column tile) work and the
  // row tiles of one cell share that XCD's L2 for the gathered rows.
  const int per_xcd = (n_work + 7) / 8;
  const int bid = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (bid >= n_work) return;              // uniform over the block, before any barrier
  const int ct = bid % n_coltiles;
  const int rt = (bid / n_coltiles) % n_rowtiles;
  const int ci = bid / (n_coltiles * n_rowtiles);
  cell_tile<T, CB, HAS_S>(sm, cm, cell_nodes, cells[ci], rt, ct, nloc, nrb, nkb, nmat, X, ldx, W, ldw, n_vec,
                          alpha);
}

// Batched form: one persistent grid walks a static list of (task, cell, row
// tile, column tile) items of one colour phase across many independent
// operators (k-points, systems).  Items were ordered on the host so that item
// i runs on XCD i % 8 and the row tiles of a cell share an XCD.

// Resident workgroups per CU the persistent form is compiled for: what the
// per-colour kernel reaches, so the item walk costs no occupancy.
template <int CB>
constexpr int cell_min_blocks() { return CB == 4 ? 1 : CB == 2 ? 3 : 4; }

template <class T, int CB, bool HAS_S>
__global__ __launch_bounds__(256, cell_min_blocks<CB>()) void cell_batch_kernel(const BatchTaskArgs tasks,
                                                         const int4* __restrict__ items, int n_items,
                                                         const double* __restrict__ alpha, int src) {
  __shared__ CellSmem<T, CB> sm;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    if (w.x < 0) continue;                // padding item (uniform over the block)
    const BatchTaskDev& t = tasks.t[w.x];
    const T* cm = sizeof(T) == 8 ? (const T*)t.cm64 : (const T*)t.cm32;
    cell_tile<T, CB, HAS_S>(sm, cm, t.cell_nodes, w.y, w.z, w.w, t.nloc, t.nrb, t.nkb, t.nmat, t.buf[src],
                            t.ld[src], t.buf[src ^ 1], t.ld[src ^ 1], t.n_vec, alpha[w.x]);
  }
}

template <class T, int CB, bool HAS_S>
static void launch_cells(chfsi_ctx* c, const T* cm, int nmat, const double2* X, int64_t ldx,
                         double2* W, int64_t ldw, int n_vec, double alpha) {
  const int BN = 32 * CB;
  const int n_rowtiles = cdiv(c->nrb, 2);
  const int n_coltiles = cdiv(n_vec, BN);
  for (int k = 0; k < c->n_colours; ++k) {
    const int n_in = c->colour_off[k + 1] - c->colour_off[k];
    if (n_in == 0) continue;
    const int nblk = n_in * n_rowtiles * n_coltiles;
    const double n2 = 2.0 * c->nloc;
    const double flops = 8.0 * n2 * n2 * n_vec * n_in;
    // issued MFMA flops: per cell nrb row blocks x 2 column waves per column tile,
    // each nkb k-steps of CB x (12 | 16) MFMAs of 16x16x4 (2048 flops)
    const double exec = (double)n_in * c->nrb * 2.0 * n_coltiles * c->nkb * CB * (HAS_S ? 16 : 12) * 2048.0;
    const double bytes = (double)n_in * ((double)nmat * c->nloc * c->nloc * sizeof(T) +
                                         3.0 * c->nloc * 2.0 * n_vec * sizeof(double2));
    StageTimer tm(c, sizeof(T) == 8 ? CHFSI_STAGE_CELL_FP64 : CHFSI_STAGE_CELL_FP32, flops, exec, bytes);
    const int grid = 8 * ((nblk + 7) / 8);
    hipLaunchKernelGGL((cell_apply_kernel<T, CB, HAS_S>), dim3(grid), dim3(256), 0, c->stream, cm,
                       c->cell_nodes.ptr, c->colour_cells.ptr + c->colour_off[k], c->nloc, c->nrb,
                       c->nkb, nmat, n_rowtiles, n_coltiles, nblk, X, ldx, W, ldw, n_vec, alpha);
    LAUNCH_CHECK();
  }
}

template <class T, bool HAS_S>
static void launch_cells_cb(chfsi_ctx* c, const T* cm, int nmat, const double2* X, int64_t ldx,
                            double2* W, int64_t ldw, int n_vec, double alpha) {
  // 64-column tiles for every block wider than 32: at p = 5..6 they run 1-4 %
  // faster than 128-column tiles in both precisions (three workgroups per CU
  // instead of one hide the epilogue and barrier latencies; the two column tiles
  // of a cell read its operator through the same L2).  The per-column arithmetic
  // does not depend on the tile width, so results are bitwise the same.
  if (n_vec > 32)
    launch_cells<T, 2, HAS_S>(c, cm, nmat, X, ldx, W, ldw, n_vec, alpha);
  else
    launch_cells<T, 1, HAS_S>(c, cm, nmat, X, ldx, W, ldw, n_vec, alpha);
}

// Local (cell) part of H_hat for all colours: W += alpha * sum_e R_e^T H_e R_e X.
void launch_cell_products(chfsi_ctx* c, KPoint& kp, int prec, const double2* X, int64_t ldx, double2* W,
                          int64_t ldw, int n_vec, double alpha) {
  if (prec == CHFSI_PREC_MIXED) {
    if (kp.gamma) launch_cells_cb<float, false>(c, kp.cell32.ptr, kp.nmat, X, ldx, W, ldw, n_vec, alpha);
    else launch_cells_cb<float, true>(c, kp.cell32.ptr, kp.nmat, X, ldx, W, ldw, n_vec, alpha);
  } else {
    if (kp.gamma) launch_cells_cb<double, false>(c, kp.cell64.ptr, kp.nmat, X, ldx, W, ldw, n_vec, alpha);
    else launch_cells_cb<double, true>(c, kp.cell64.ptr, kp.nmat, X, ldx, W, ldw, n_vec, alpha);
  }
}

// ---------------------------------------------------------------- batched form
template <class T, int CB, bool HAS_S>
static void launch_batch_t(hipStream_t s, const BatchTaskArgs& tasks, const int4* items, int n_items,
                           const double* alpha, int src, int grid) {
  hipLaunchKernelGGL((cell_batch_kernel<T, CB, HAS_S>), dim3(grid), dim3(256), 0, s, tasks, items, n_items, alpha,
                     src);
  LAUNCH_CHECK();
}

template <class T, bool HAS_S>
static void launch_batch_cb(hipStream_t s, int CB, const BatchTaskArgs& tasks, const int4* items, int n_items,
                            const double* alpha, int src, int grid) {
  if (CB == 4)
    launch_batch_t<T, 4, HAS_S>(s, tasks, items, n_items, alpha, src, grid);
  else if (CB == 2)
    launch_batch_t<T, 2, HAS_S>(s, tasks, items, n_items, alpha, src, grid);
  else
    launch_batch_t<T, 1, HAS_S>(s, tasks, items, n_items, alpha, src, grid);
}

void launch_cell_batch(hipStream_t s, bool fp64, int CB, bool has_s, const BatchTaskArgs& tasks, const int4* items,
                       int n_items, const double* alpha, int src, int grid) {
  if (fp64) {
    if (has_s) launch_batch_cb<double, true>(s, CB, tasks, items, n_items, alpha, src, grid);
    else launch_batch_cb<double, false>(s, CB, tasks, items, n_items, alpha, src, grid);
  } else {
    if (has_s) launch_batch_cb<float, true>(s, CB, tasks, items, n_items, alpha, src, grid);
    else launch_batch_cb<float, false>(s, CB, tasks, items, n_items, alpha, src, grid);
  }
}

template <class T, int CB, bool HAS_S>
static int occ_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cell_batch_kernel<T, CB, HAS_S>, 256, 0) != hipSuccess) n = 1;
  return std::max(1, n);
}

int cell_batch_blocks_per_cu(bool fp64, int CB, bool has_s) {
  if (fp64) {
    if (has_s) return CB == 4 ? occ_t<double, 4, true>() : CB == 2 ? occ_t<double, 2, true>() : occ_t<double, 1, true>();
    return CB == 4 ? occ_t<double, 4, false>() : CB == 2 ? occ_t<double, 2, false>() : occ_t<double, 1, false>();
  }
  if (has_s) return CB == 4 ? occ_t<float, 4, true>() : CB == 2 ? occ_t<float, 2, true>() : occ_t<float, 1, true>();
  return CB == 4 ? occ_t<float, 4, false>() : CB == 2 ? occ_t<float, 2, false>() : occ_t<float, 1, false>();
}

template <class T, bool HAS_S>
static void cells_with_cb(chfsi_ctx* c, int CB, const T* cm, int nmat, const double2* X, int64_t ldx, double2* W,
                          int64_t ldw, int n_vec) {
  if (CB == 4) launch_cells<T, 4, HAS_S>(c, cm, nmat, X, ldx, W, ldw, n_vec, 1.0);
  else if (CB == 2) launch_cells<T, 2, HAS_S>(c, cm, nmat, X, ldx, W, ldw, n_vec, 1.0);
  else launch_cells<T, 1, HAS_S>(c, cm, nmat, X, ldx, W, ldw, n_vec, 1.0);
}

// Mean time (ms) of the cell stage of one apply with column tiles of 32*CB.
double time_cell_stage(chfsi_ctx* c, KPoint& kp, int CB, int prec, const double2* X, int64_t ldx, double2* W,
                       int64_t ldw, int n_vec, int reps) {
  const bool was = c->stats_on;
  c->stats_on = false;
  hipEvent_t e0, e1;
  CHFSI_HIP(hipEventCreate(&e0));
  CHFSI_HIP(hipEventCreate(&e1));
  auto run = [&]() {
    if (prec == CHFSI_PREC_MIXED) {
      if (kp.gamma) cells_with_cb<float, false>(c, CB, kp.cell32.ptr, kp.nmat, X, ldx, W, ldw, n_vec);
      else cells_with_cb<float, true>(c, CB, kp.cell32.ptr, kp.nmat, X, ldx, W, ldw, n_vec);
    } else {
      if (kp.gamma) cells_with_cb<double, false>(c, CB, kp.cell64.ptr, kp.nmat, X, ldx, W, ldw, n_vec);
      else cells_with_cb<double, true>(c, CB, kp.cell64.ptr, kp.nmat, X, ldx, W, ldw, n_vec);
    }
  };
  run();                                   // warm
  CHFSI_HIP(hipEventRecord(e0, c->stream));
  for (int r = 0; r < reps; ++r) run();
  CHFSI_HIP(hipEventRecord(e1, c->stream));
  CHFSI_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  CHFSI_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->stats_on = was;
  return ms / reps;
}

}  // namespace chfsi
