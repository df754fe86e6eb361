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
constexpr int sf_cols(int NP) { return NP <= 4 ? 8 : NP == 5 ? 4 : NP == 6 ? 3 : NP == 7 ? 2 : 1; }

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

// out = contraction of fields 0..NF-1 along DIM with the n_p x n_p table M:
//   FWD:  out[.. o ..] = sum_i M[i][o] in[.. i ..]   (nodes -> points with M = B)
//   !FWD: out[.. o ..] = sum_i M[o][i] in[.. i ..]   (points -> nodes)
// in and out may be the same buffer: a thread reads its whole line before it
// writes it, and the lines of one pass are disjoint.
template <int NP, int NF, int DIM, bool FWD, int NT = 256, class T = double>
__device__ __forceinline__ void sf_line_pass(const T* __restrict__ M, const typename SfC2<T>::type* in,
                                             typename SfC2<T>::type* out) {
  typedef typename SfC2<T>::type C2;
  constexpr int N2 = NP * NP, N3 = N2 * NP;
  constexpr int S = DIM == 0 ? 1 : DIM == 1 ? NP : N2;
  for (int t = threadIdx.x; t < N2 * NF; t += NT) {
    const int l = t % N2, f = t / N2;
    const int base = f * N3 + sf_line_base<NP, DIM>(l);
    C2 v[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) v[j] = in[base + j * S];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      T re = 0, im = 0;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        const T m = FWD ? M[i * NP + o] : M[o * NP + i];
        re = fma(m, v[i].x, re);
        im = fma(m, v[i].y, im);
      }
      out[base + o * S] = C2{re, im};
    }
  }
}

}  // namespace chfsi
