// Sum-factorised contractions of cell fields along one direction, shared by
// the matrix-free operator and the quadrature-point field kernels.
//
// A cell field holds n_p^3 complex values at the points x + n_p (y + n_p z)
// (nodes or quadrature points, n_q = n_p).  A workgroup of NT threads holds NF
// such fields in LDS; a pass along direction DIM gives each thread one line
// (n_p values along DIM, the other two coordinates fixed) of one field, so every
// value read from LDS feeds n_p multiply-adds.
#pragma once

#include <hip/hip_runtime.h>

namespace chfsi {

// columns per workgroup of the matrix-free operator (2 fields per column: the
// spins) for two LDS buffers of about 44 KB, so that three workgroups share a CU
constexpr int sf_cols(int NP) { return NP <= 4 ? 8 : NP == 5 ? 4 : NP <= 7 ? 2 : 1; }

// Workgroup barrier for LDS hand-offs: waits for this wave's LDS operations
// only, so global loads issued before it (a prefetch of the next work item) stay
// in flight; __syncthreads() would wait for them as well.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// First point of line l along DIM.
template <int NP, int DIM>
__device__ __forceinline__ int sf_line_base(int l) {
  if constexpr (DIM == 0) return l * NP;                                // l = y + NP z
  else if constexpr (DIM == 1) return (l % NP) + (l / NP) * NP * NP;    // l = x + NP z
  else return l;                                                        // l = x + NP y
}

// Complex pair of the arithmetic type.
template <class T> struct SfC2;
template <> struct SfC2<double> { typedef double2 type; };
template <> struct SfC2<float> { typedef float2 type; };

// Even-odd form of a 1-D contraction out[o] = sum_i M[i][o] in[i] (n = NP).
// The GLL nodes and the quadrature points are symmetric about the cell centre,
// so the interpolation matrix B and its transpose are centrosymmetric
// (M[n-1-i][n-1-o] = M[i][o]) and the collocation derivative and its transpose
// skew-centrosymmetric (M[n-1-i][n-1-o] = -M[i][o], SK).  With h = n/2,
// e_i = in_i + in_{n-1-i}, d_i = in_i - in_{n-1-i} (i < h) and the middle value m,
//   out_o = S_o + D_o, out_{n-1-o} = S_o - D_o (o < h),
//   S_o = sum_i A[i][o] (e_i | d_i) [+ M[h][o] m],  D_o = sum_i C[i][o] (d_i | e_i) [+ M[h][o] m],
//   A = (M[i][o] + M[i][n-1-o]) / 2,  C = (M[i][o] - M[i][n-1-o]) / 2,
// (centrosymmetric | skew; the middle term goes to S, resp. D) and the middle
// output sum_i M[i][h] (e_i | d_i) [+ M[h][h] m]: 2h^2 + 2h + 1 multiply-adds
// instead of n^2 (25 instead of 49 at n = 7).  Table: [A: h*h][C: h*h][M[h][o]:
// h][M[i][h]: h][M[h][h]].
constexpr int sf_eo_size(int NP) { return 2 * (NP / 2) * (NP / 2) + 2 * (NP / 2) + 1; }

template <class T, int N, bool SK>
__device__ __forceinline__ void sf_eo(const T* __restrict__ tb, const typename SfC2<T>::type* in,
                                      typename SfC2<T>::type* out) {
  typedef typename SfC2<T>::type C2;
  constexpr int h = N / 2;
  constexpr bool odd = (N % 2) != 0;
  const T* A = tb;
  const T* Cm = tb + h * h;
  const T* mrow = tb + 2 * h * h;
  const T* mcol = mrow + h;
  C2 e[h], d[h];
#pragma unroll
  for (int i = 0; i < h; ++i) {
    e[i] = C2{in[i].x + in[N - 1 - i].x, in[i].y + in[N - 1 - i].y};
    d[i] = C2{in[i].x - in[N - 1 - i].x, in[i].y - in[N - 1 - i].y};
  }
#pragma unroll
  for (int o = 0; o < h; ++o) {
    T sr = 0, si = 0, dr = 0, di = 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const C2 a = SK ? d[i] : e[i];
      const C2 b = SK ? e[i] : d[i];
      sr = fma(A[i * h + o], a.x, sr);
      si = fma(A[i * h + o], a.y, si);
      dr = fma(Cm[i * h + o], b.x, dr);
      di = fma(Cm[i * h + o], b.y, di);
    }
    if constexpr (odd) {
      if constexpr (SK) {
        dr = fma(mrow[o], in[h].x, dr);
        di = fma(mrow[o], in[h].y, di);
      } else {
        sr = fma(mrow[o], in[h].x, sr);
        si = fma(mrow[o], in[h].y, si);
      }
    }
    out[o] = C2{sr + dr, si + di};
    out[N - 1 - o] = C2{sr - dr, si - di};
  }
  if constexpr (odd) {
    T r = 0, im = 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const C2 a = SK ? d[i] : e[i];
      r = fma(mcol[i], a.x, r);
      im = fma(mcol[i], a.y, im);
    }
    if constexpr (!SK) {
      r = fma(mcol[h], in[h].x, r);
      im = fma(mcol[h], in[h].y, im);
    }
    out[h] = C2{r, im};
  }
}

// First point of line l along DIM in a padded field (point (x, y, z) at
// x + SY y + SZ z).
template <int NP, int DIM, int SY, int SZ>
__device__ __forceinline__ int sf_line_base_padded(int l) {
  if constexpr (DIM == 0) return (l % NP) * SY + (l / NP) * SZ;    // l = y + NP z
  else if constexpr (DIM == 1) return (l % NP) + (l / NP) * SZ;    // l = x + NP z
  else return (l % NP) + (l / NP) * SY;                             // l = x + NP y
}

// out = contraction of fields 0..NF-1 along DIM with a centrosymmetric n_p x n_p
// matrix given by its even-odd table (sf_eo):
//   B (nodes -> points):  out[.. o ..] = sum_i B[i][o] in[.. i ..]
//   B^T (points -> nodes): out[.. o ..] = sum_i B[o][i] in[.. i ..]
// in and out may be the same buffer: a thread reads its whole line before it
// writes it, and the lines of one pass are disjoint.  Fields are compact
// (point (x, y, z) at x + NP y + NP^2 z, fields NP^3 apart) unless SY, SZ, SF
// give a padded layout: point at x + SY y + SZ z, fields SF apart.
template <int NP, int NF, int DIM, int NT = 256, class T = double, int SY = NP, int SZ = NP * NP,
          int SF = NP * NP * NP>
__device__ __forceinline__ void sf_line_pass(const T* __restrict__ eo, const typename SfC2<T>::type* in,
                                             typename SfC2<T>::type* out) {
  typedef typename SfC2<T>::type C2;
  constexpr int N2 = NP * NP;
  constexpr bool compact = SY == NP && SZ == N2;
  constexpr int S = DIM == 0 ? 1 : DIM == 1 ? SY : SZ;
  for (int t = threadIdx.x; t < N2 * NF; t += NT) {
    const int l = t % N2, f = t / N2;
    int base;
    if constexpr (compact) base = f * SF + sf_line_base<NP, DIM>(l);
    else base = f * SF + sf_line_base_padded<NP, DIM, SY, SZ>(l);
    C2 v[NP], r[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) v[j] = in[base + j * S];
    sf_eo<T, NP, false>(eo, v, r);
#pragma unroll
    for (int o = 0; o < NP; ++o) out[base + o * S] = r[o];
  }
}

}  // namespace chfsi
