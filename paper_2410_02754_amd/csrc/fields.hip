// Scalar fields of the self-consistent loop (Sec. III.B: the fixed-point map
// and its density mixing; Sec. IV.A: the two-grid start).
//
// Fields live at the cell quadrature points ([E][nq^3], the order of
// chfsi_quad_points) or at the global nodes ([M]).  The FE scalar operator
// A = K_s + kappa^2 M_c (K_s = int grad N_I . grad N_J, M_c = int N_I N_J) has
// the same cell matrix in every cell of the uniform mesh, so its action is
// one shared dense cell matrix applied to the gathered nodal values, with a
// colour-ordered scatter-add (no atomics, bitwise reproducible).  Screened
// Poisson problems (kappa^2 - lap) u = g are solved in the FE space by
// conjugate gradients preconditioned with the assembled diagonal of A.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "mfma.h"

namespace chfsi {

namespace {
constexpr int kFieldRed = 256;      // fixed reduction grid (deterministic order)

// y[I(e, i)] += sum_j A[i][j] x[I(e, j)] for the cells of one colour
__global__ __launch_bounds__(256) void scal_cell_op_kernel(const double* __restrict__ A,
                                                           const int32_t* __restrict__ cell_nodes,
                                                           const int32_t* __restrict__ cells, int nloc,
                                                           const double* __restrict__ x, double* __restrict__ y) {
  extern __shared__ double xs[];
  const int e = cells[blockIdx.x];
  const int32_t* nd = cell_nodes + (size_t)e * nloc;
  for (int j = threadIdx.x; j < nloc; j += blockDim.x) xs[j] = x[nd[j]];
  __syncthreads();
  for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
    const double* Ai = A + (size_t)i * nloc;
    double s = 0.0;
    for (int j = 0; j < nloc; ++j) s += Ai[j] * xs[j];
    y[nd[i]] += s;
  }
}

// b[I(e, i)] += sum_q N[i][q] wJ[q] g[e][q] for the cells of one colour
__global__ __launch_bounds__(256) void scal_project_kernel(const double* __restrict__ Nt,
                                                           const double* __restrict__ wJ,
                                                           const int32_t* __restrict__ cell_nodes,
                                                           const int32_t* __restrict__ cells, int nloc, int nq3,
                                                           const double* __restrict__ g, double* __restrict__ b) {
  extern __shared__ double gs[];
  const int e = cells[blockIdx.x];
  for (int q = threadIdx.x; q < nq3; q += blockDim.x) gs[q] = wJ[q] * g[(size_t)e * nq3 + q];
  __syncthreads();
  const int32_t* nd = cell_nodes + (size_t)e * nloc;
  for (int i = threadIdx.x; i < nloc; i += blockDim.x) {
    const double* Ni = Nt + (size_t)i * nq3;
    double s = 0.0;
    for (int q = 0; q < nq3; ++q) s += Ni[q] * gs[q];
    b[nd[i]] += s;
  }
}

// out[e][q] = sum_i N[i][q] u[I(e, i)]
__global__ __launch_bounds__(256) void scal_interp_kernel(const double* __restrict__ Nt,
                                                          const int32_t* __restrict__ cell_nodes, int nloc, int nq3,
                                                          const double* __restrict__ u, double* __restrict__ out) {
  extern __shared__ double us[];
  const int e = blockIdx.x;
  const int32_t* nd = cell_nodes + (size_t)e * nloc;
  for (int i = threadIdx.x; i < nloc; i += blockDim.x) us[i] = u[nd[i]];
  __syncthreads();
  for (int q = threadIdx.x; q < nq3; q += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nloc; ++i) s += Nt[(size_t)i * nq3 + q] * us[i];
    out[(size_t)e * nq3 + q] = s;
  }
}

// partial[g] = sum over this group's strided range of x[i] * y[i] * (w ? w[i % nw] : 1)
__global__ __launch_bounds__(256) void wdot_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                   const double* __restrict__ w, int64_t nw, int64_t n,
                                                   double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kFieldRed * 256) {
    const double t = x[i] * (y ? y[i] : 1.0);
    s += w ? t * w[i % nw] : t;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// y = a x + b y (y may be null: y = a x written to out)
__global__ void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b, const double* y,
                             double* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ void mul_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ x,
                           double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] * x[i];
}

__global__ void fill_kernel(int64_t n, double v, double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = v;
}

// LSDA (Dirac) exchange under the locally collinear substitution
// rho_up,dn = (rho +- |m|)/2: v_s = -(6/pi)^(1/3) rho_s^(1/3),
// V = (v_up + v_dn)/2, B = (v_up - v_dn)/2 m/|m|  (B = 0 where m = 0)
__global__ void exchange_kernel(int64_t n, const double* __restrict__ rho, const double* __restrict__ m,
                                const double* __restrict__ vadd, const double* __restrict__ badd,
                                double* __restrict__ V, double* __restrict__ B) {
  const double cx = cbrt(6.0 / M_PI);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double mx = m[3 * i], my = m[3 * i + 1], mz = m[3 * i + 2];
    const double ma = sqrt(mx * mx + my * my + mz * mz);
    const double ru = fmax(0.5 * (rho[i] + ma), 0.0), rd = fmax(0.5 * (rho[i] - ma), 0.0);
    const double vu = -cx * cbrt(ru), vd = -cx * cbrt(rd);
    V[i] = 0.5 * (vu + vd) + (vadd ? vadd[i] : 0.0);
    const double f = ma > 0.0 ? 0.5 * (vu - vd) / ma : 0.0;
    B[3 * i] = f * mx + (badd ? badd[3 * i] : 0.0);
    B[3 * i + 1] = f * my + (badd ? badd[3 * i + 1] : 0.0);
    B[3 * i + 2] = f * mz + (badd ? badd[3 * i + 2] : 0.0);
  }
}

// two-grid transfer: every fine node takes the coarse field of its canonical cell
// (the cell where its local index is below p in each direction), through the
// coarse Lagrange basis at the fine GLL nodes: Yf = M_f^{1/2} T (M_c^{-1/2} Yc)
__global__ __launch_bounds__(256) void block_interp_kernel(
    const double2* __restrict__ Yc, int64_t ldc, double2* __restrict__ Yf, int64_t ldf, int n_vec,
    const double* __restrict__ T /*[npc][npf]*/, const int32_t* __restrict__ cnodes_c, const double* __restrict__ ms_c,
    const double* __restrict__ ms_f, int pf, int npc, int ncx, int ncy, int nfx, int nfy, int64_t n_fine) {
  const int64_t total = n_fine * n_vec;
  const int nlc = npc * npc * npc;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t I = t / n_vec;
    const int col = (int)(t - I * n_vec);
    const int ix = (int)(I % nfx), iy = (int)((I / nfx) % nfy), iz = (int)(I / ((int64_t)nfx * nfy));
    const int cx = ix / pf, cy = iy / pf, cz = iz / pf;
    const int ax = ix - cx * pf, ay = iy - cy * pf, az = iz - cz * pf;
    const int32_t* nd = cnodes_c + (size_t)(cx + ncx * (cy + ncy * cz)) * nlc;
    const int npf = pf + 1;
    double2 s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
    for (int k = 0; k < npc; ++k) {
      const double tz = T[k * npf + az];
      for (int j = 0; j < npc; ++j) {
        const double tyz = tz * T[j * npf + ay];
        for (int i = 0; i < npc; ++i) {
          const double w = tyz * T[i * npf + ax];
          const int64_t J = nd[i + npc * (j + npc * k)];
          const double sc = w * ms_c[J];
          const double2 u0 = Yc[(2 * J) * ldc + col], u1 = Yc[(2 * J + 1) * ldc + col];
          s0.x += sc * u0.x;
          s0.y += sc * u0.y;
          s1.x += sc * u1.x;
          s1.y += sc * u1.y;
        }
      }
    }
    const double f = 1.0 / ms_f[I];
    Yf[(2 * I) * ldf + col] = double2{f * s0.x, f * s0.y};
    Yf[(2 * I + 1) * ldf + col] = double2{f * s1.x, f * s1.y};
  }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 8192)); }
}  // namespace

// ---------------------------------------------------------------- host side
struct FieldOps {
  DevBuf<double> Nt;       // [nloc][nq3] 3-D interpolation table
  DevBuf<double> wJ;       // [nq3] w_q J
  DevBuf<double> wJ3;      // [3 nq3] w_q J repeated per vector component
  DevBuf<double> ones;     // [max(M, E nq3)] ones
  DevBuf<double> md;       // [M] lumped mass M_D
  DevBuf<double> gq;       // [E nq3] a field at the quadrature points
  DevBuf<double> A;        // [nloc][nloc] shared cell matrix of the last kappa^2
  DevBuf<double> dinv;     // [M] inverse assembled diagonal of A
  DevBuf<double> red;      // reduction partials
  DevBuf<double> v[5];     // CG vectors and a nodal right-hand side
  double md_sum = 0.0;
  double kappa2 = -1.0;
  bool ready = false;
};

static void fill(chfsi_ctx* c, int64_t n, double v, double* out);
static void axpby(chfsi_ctx* c, int64_t n, double a, const double* x, double b, const double* y, double* out);

static FieldOps& fops(chfsi_ctx* c) {
  if (!c->fields) c->fields = std::make_shared<FieldOps>();
  FieldOps& f = *c->fields;
  if (!f.ready) {
    const int n = c->np1, nq = c->nq, nloc = c->nloc, nq3 = c->nq3;
    std::vector<double> Nt((size_t)nloc * nq3), wJ(nq3);
    for (int i = 0; i < nloc; ++i) {
      const int ia[3] = {i % n, (i / n) % n, i / (n * n)};
      for (int q = 0; q < nq3; ++q) {
        const int qa[3] = {q % nq, (q / nq) % nq, q / (nq * nq)};
        Nt[(size_t)i * nq3 + q] =
            c->ref.B[ia[0] * nq + qa[0]] * c->ref.B[ia[1] * nq + qa[1]] * c->ref.B[ia[2] * nq + qa[2]];
      }
    }
    for (int q = 0; q < nq3; ++q)
      wJ[q] = c->ref.wq[q % nq] * c->ref.wq[(q / nq) % nq] * c->ref.wq[q / (nq * nq)] * c->J;
    std::vector<double> wJ3((size_t)3 * nq3), md(c->n_nodes);
    for (int q = 0; q < nq3; ++q) wJ3[3 * q] = wJ3[3 * q + 1] = wJ3[3 * q + 2] = wJ[q];
    f.md_sum = 0.0;
    for (int64_t i = 0; i < c->n_nodes; ++i) {
      md[i] = 1.0 / (c->minv_sqrt_h[i] * c->minv_sqrt_h[i]);
      f.md_sum += md[i];
    }
    const int64_t np = (int64_t)c->n_cells * nq3;
    f.Nt.upload(Nt.data(), Nt.size(), c->stream);
    f.wJ.upload(wJ.data(), wJ.size(), c->stream);
    f.wJ3.upload(wJ3.data(), wJ3.size(), c->stream);
    f.md.upload(md.data(), md.size(), c->stream);
    f.ones.alloc(std::max<int64_t>(c->n_nodes, np));
    fill(c, std::max<int64_t>(c->n_nodes, np), 1.0, f.ones.ptr);
    f.gq.alloc(np);
    f.red.alloc(kFieldRed);
    for (auto& b : f.v) b.alloc(c->n_nodes);
    CHFSI_HIP(hipStreamSynchronize(c->stream));
    f.ready = true;
  }
  return f;
}

static void set_kappa(chfsi_ctx* c, FieldOps& f, double kappa2) {
  if (f.kappa2 == kappa2) return;
  const size_t nloc = c->nloc;
  std::vector<double> A(nloc * nloc);
  for (size_t i = 0; i < A.size(); ++i) A[i] = 2.0 * c->Kin[i] + kappa2 * c->Mcons[i];
  std::vector<double> d(c->n_nodes, 0.0);
  for (int e = 0; e < c->n_cells; ++e)
    for (size_t a = 0; a < nloc; ++a) d[c->cell_nodes_h[(size_t)e * nloc + a]] += A[a * nloc + a];
  for (auto& x : d) x = 1.0 / x;
  f.A.upload(A.data(), A.size(), c->stream);
  f.dinv.upload(d.data(), d.size(), c->stream);
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  f.kappa2 = kappa2;
}

// sum_i x_i y_i (w_{i mod nw}); fixed grid, partials summed on the host in order
static double wdot(chfsi_ctx* c, FieldOps& f, const double* x, const double* y, const double* w, int64_t nw,
                   int64_t n) {
  hipLaunchKernelGGL(wdot_kernel, dim3(kFieldRed), dim3(256), 0, c->stream, x, y, w, nw, n, f.red.ptr);
  LAUNCH_CHECK();
  double h[kFieldRed];
  CHFSI_HIP(hipMemcpyAsync(h, f.red.ptr, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (int g = 0; g < kFieldRed; ++g) s += h[g];
  return s;
}

static void axpby(chfsi_ctx* c, int64_t n, double a, const double* x, double b, const double* y, double* out) {
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, c->stream, n, a, x, b, y, out);
  LAUNCH_CHECK();
}

static void fill(chfsi_ctx* c, int64_t n, double v, double* out) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, c->stream, n, v, out);
  LAUNCH_CHECK();
}

// y = A x (nodal)
static void scal_apply(chfsi_ctx* c, FieldOps& f, const double* x, double* y) {
  fill(c, c->n_nodes, 0.0, y);
  const size_t sh = c->nloc * sizeof(double);
  for (int k = 0; k < c->n_colours; ++k) {
    const int n_in = c->colour_off[k + 1] - c->colour_off[k];
    if (n_in == 0) continue;
    hipLaunchKernelGGL(scal_cell_op_kernel, dim3(n_in), dim3(256), sh, c->stream, f.A.ptr, c->cell_nodes.ptr,
                       c->colour_cells.ptr + c->colour_off[k], c->nloc, x, y);
    LAUNCH_CHECK();
  }
}

// b = int N_I g (nodal, overwritten)
static void scal_project(chfsi_ctx* c, FieldOps& f, const double* g, double* b) {
  fill(c, c->n_nodes, 0.0, b);
  const size_t sh = c->nq3 * sizeof(double);
  for (int k = 0; k < c->n_colours; ++k) {
    const int n_in = c->colour_off[k + 1] - c->colour_off[k];
    if (n_in == 0) continue;
    hipLaunchKernelGGL(scal_project_kernel, dim3(n_in), dim3(256), sh, c->stream, f.Nt.ptr, f.wJ.ptr,
                       c->cell_nodes.ptr, c->colour_cells.ptr + c->colour_off[k], c->nloc, c->nq3, g, b);
    LAUNCH_CHECK();
  }
}

static void scal_interp(chfsi_ctx* c, FieldOps& f, const double* u, double* out) {
  hipLaunchKernelGGL(scal_interp_kernel, dim3(c->n_cells), dim3(256), c->nloc * sizeof(double), c->stream,
                     f.Nt.ptr, c->cell_nodes.ptr, c->nloc, c->nq3, u, out);
  LAUNCH_CHECK();
}

// A u = b by CG preconditioned with diag(A)^{-1}; b is v[4]; u returned in v[0].
// Stops when ||r|| <= tol ||b||.  Returns the iteration count (negative if max_iter hit).
static int pcg(chfsi_ctx* c, FieldOps& f, double tol, int max_iter, double* rel_out) {
  const int64_t n = c->n_nodes;
  double *u = f.v[0].ptr, *r = f.v[1].ptr, *z = f.v[2].ptr, *pp = f.v[3].ptr, *b = f.v[4].ptr;
  double* Ap = z;   // z and A p are not live at the same time
  fill(c, n, 0.0, u);
  axpby(c, n, 1.0, b, 0.0, nullptr, r);
  const double bn = std::sqrt(wdot(c, f, b, b, nullptr, 1, n));
  if (bn == 0.0) {
    if (rel_out) *rel_out = 0.0;
    return 0;
  }
  hipLaunchKernelGGL(mul_kernel, dim3(grid_for(n)), dim3(256), 0, c->stream, n, f.dinv.ptr, r, pp);
  LAUNCH_CHECK();
  double rz = wdot(c, f, r, pp, nullptr, 1, n);
  double rel = 1.0;
  int it = 0;
  for (; it < max_iter; ++it) {
    scal_apply(c, f, pp, Ap);
    const double pAp = wdot(c, f, pp, Ap, nullptr, 1, n);
    const double al = rz / pAp;
    axpby(c, n, al, pp, 1.0, u, u);
    axpby(c, n, -al, Ap, 1.0, r, r);
    rel = std::sqrt(wdot(c, f, r, r, nullptr, 1, n)) / bn;
    if (rel <= tol) {
      ++it;
      break;
    }
    hipLaunchKernelGGL(mul_kernel, dim3(grid_for(n)), dim3(256), 0, c->stream, n, f.dinv.ptr, r, z);
    LAUNCH_CHECK();
    const double rz1 = wdot(c, f, r, z, nullptr, 1, n);
    axpby(c, n, 1.0, z, rz1 / rz, pp, pp);
    rz = rz1;
  }
  if (rel_out) *rel_out = rel;
  return rel <= tol ? it : -it;
}

double field_integral(chfsi_ctx* c, const double* g) {
  FieldOps& f = fops(c);
  return wdot(c, f, g, nullptr, f.wJ.ptr, c->nq3, (int64_t)c->n_cells * c->nq3);
}

double field_inner(chfsi_ctx* c, const double* r1, const double* m1, const double* r2, const double* m2) {
  FieldOps& f = fops(c);
  const int64_t np = (int64_t)c->n_cells * c->nq3;
  double s = wdot(c, f, r1, r2, f.wJ.ptr, c->nq3, np);
  if (m1 && m2) s += wdot(c, f, m1, m2, f.wJ3.ptr, 3 * c->nq3, 3 * np);
  return 0.5 * s;
}

// (kappa^2 - lap) u = scale g in the FE space, u at the quadrature points (u may
// alias g).  kappa2 == 0: the periodic problem with g - mean(g), u of zero
// lumped-mass mean.  Returns the CG iteration count (negative: not converged).
int screened_poisson(chfsi_ctx* c, double kappa2, double scale, const double* g, double* u_q, double tol,
                     int max_iter, double* rel) {
  FieldOps& f = fops(c);
  set_kappa(c, f, kappa2);
  const int64_t np = (int64_t)c->n_cells * c->nq3;
  const double vol = c->box[0] * c->box[1] * c->box[2];
  const double* src = g;
  if (kappa2 == 0.0) {
    const double gbar = field_integral(c, g) / vol;
    axpby(c, np, 1.0, g, -gbar, f.ones.ptr, f.gq.ptr);          // g - mean(g)
    src = f.gq.ptr;
  }
  scal_project(c, f, src, f.v[4].ptr);
  if (scale != 1.0) axpby(c, c->n_nodes, scale, f.v[4].ptr, 0.0, nullptr, f.v[4].ptr);
  if (kappa2 == 0.0) {
    // the right-hand side's roundoff component along the constants (the null space)
    const double bm = wdot(c, f, f.v[4].ptr, nullptr, nullptr, 1, c->n_nodes) / (double)c->n_nodes;
    axpby(c, c->n_nodes, 1.0, f.v[4].ptr, -bm, f.ones.ptr, f.v[4].ptr);
  }
  const int it = pcg(c, f, tol, max_iter, rel);
  if (kappa2 == 0.0) {
    const double mean = wdot(c, f, f.v[0].ptr, f.md.ptr, nullptr, 1, c->n_nodes) / f.md_sum;
    axpby(c, c->n_nodes, 1.0, f.v[0].ptr, -mean, f.ones.ptr, f.v[0].ptr);
  }
  scal_interp(c, f, f.v[0].ptr, u_q);
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  return it;
}

void launch_exchange(chfsi_ctx* c, int64_t n_points, const double* rho, const double* m, const double* vadd,
                     const double* badd, double* V, double* B) {
  hipLaunchKernelGGL(exchange_kernel, dim3(grid_for(n_points)), dim3(256), 0, c->stream, n_points, rho, m, vadd,
                     badd, V, B);
  LAUNCH_CHECK();
}

void field_axpby(chfsi_ctx* c, int64_t n, double a, const double* x, double b, const double* y, double* out) {
  axpby(c, n, a, x, b, y, out);
}

void field_fill(chfsi_ctx* c, int64_t n, double v, double* out) { fill(c, n, v, out); }

void interpolate_block(chfsi_ctx* cc, chfsi_ctx* cf, const double2* Yc, int64_t ldc, double2* Yf, int64_t ldf,
                       int n_vec) {
  std::vector<double> T, D;
  lagrange_on(cc->ref.xi, cf->ref.xi, T, D);      // T[i][a] = l_i^{p-1}(xi_a^p)
  DevBuf<double> Td;
  Td.upload(T.data(), T.size(), cf->stream);
  const int64_t total = cf->n_nodes * n_vec;
  hipLaunchKernelGGL(block_interp_kernel, dim3(grid_for(total)), dim3(256), 0, cf->stream, Yc, ldc, Yf, ldf, n_vec,
                     Td.ptr, cc->cell_nodes.ptr, cc->minv_sqrt.ptr, cf->minv_sqrt.ptr, cf->p, cc->np1, cc->nc[0],
                     cc->nc[1], cf->Nd[0], cf->Nd[1], cf->n_nodes);
  LAUNCH_CHECK();
  CHFSI_HIP(hipStreamSynchronize(cf->stream));
}

}  // namespace chfsi
