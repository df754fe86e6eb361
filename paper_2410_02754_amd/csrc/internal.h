// Private declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/chfsi.h"

namespace chfsi {

using cplx = std::complex<double>;

constexpr int kMaxP = 8;
constexpr int kMaxNq = 12;
constexpr int kRowBlk = 16;  // MFMA row granularity of the cell operator tiles
constexpr int kKStep = 4;    // MFMA reduction depth per fragment

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};

#define CHFSI_HIP(call)                                                               \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::chfsi::Error{CHFSI_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define CHFSI_CHECK(cond, code, msg)                                                  \
  do {                                                                                \
    if (!(cond)) throw ::chfsi::Error{(code), (msg)};                                 \
  } while (0)

// ---------------------------------------------------------------- device buffer
template <class T>
struct DevBuf {
  T* ptr = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count <= n && ptr) return;
    release();
    if (count == 0) return;
    hipError_t e = hipMalloc(&ptr, count * sizeof(T));
    if (e != hipSuccess) {
      ptr = nullptr;
      throw Error{CHFSI_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    n = count;
  }
  void upload(const T* h, size_t count, hipStream_t s) {
    alloc(count);
    CHFSI_HIP(hipMemcpyAsync(ptr, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

// ---------------------------------------------------------------- reference element (host)
struct RefElement {
  int p = 0, np1 = 0, nq = 0;
  std::vector<double> xi, wgll;   // GLL nodes/weights
  std::vector<double> xq, wq;     // quadrature points/weights (GL or GLL)
  std::vector<double> B, D;       // [np1][nq] l_a(x_q), l_a'(x_q)
};
void gll_rule(int p, std::vector<double>& x, std::vector<double>& w);
void gl_rule(int n, std::vector<double>& x, std::vector<double>& w);
void lagrange_on(const std::vector<double>& nodes, const std::vector<double>& pts,
                 std::vector<double>& B, std::vector<double>& D);
RefElement make_ref(int p, int quad, int nq);

// ---------------------------------------------------------------- nonlocal tables per k
struct AtomTables {
  int n_pj = 0;                 // orbitals (spinor columns = 2 n_pj)
  int n_sup = 0;                // support nodes
  int64_t node_off = 0;         // offset into the concatenated support arrays
  std::vector<cplx> delta;      // [2 n_pj][2 n_pj]
};

struct NonlocalK {
  int n_atoms = 0;
  int max_pj = 0;
  int64_t n_entries = 0;        // sum over atoms of n_sup
  std::vector<AtomTables> atoms;
  // device, concatenated over atoms (atom a occupies [node_off, node_off + n_sup))
  DevBuf<int32_t> sup_node;     // [n_entries] global node
  DevBuf<double2> proj;         // [n_entries][max_pj] M^{-1/2}-scaled P_hat (complex)
  DevBuf<float2> proj32;        // same, FP32
  DevBuf<double2> delta;        // [n_atoms][2 max_pj][2 max_pj]
  DevBuf<int32_t> atom_off;     // [n_atoms + 1] entry offsets
  DevBuf<int32_t> atom_npj;     // [n_atoms]
  bool real_proj = false;       // every projector value is real (Gamma point)
  // chunked reduction work list for C = P^H X: the entries of one atom inside one
  // window of kNlWindow consecutive global nodes (at most kNlChunk of them);
  // chunk ids are grouped by atom (the reduction order), chunk_order lists them
  // by (window, atom) so that chunks reading the same rows run together
  int n_chunks = 0;
  DevBuf<int32_t> chunk_atom;   // [n_chunks]
  DevBuf<int32_t> chunk_begin;  // [n_chunks]
  DevBuf<int32_t> chunk_end;    // [n_chunks]
  DevBuf<int32_t> chunk_order;  // [n_chunks] launch order
  DevBuf<int32_t> atom_chunk0;  // [n_atoms + 1]
  // back-product over runs of kNlRun consecutive global nodes: the atoms whose
  // support meets run r are pair_atom[run_off[r] .. run_off[r + 1]) (ascending),
  // and pair_ent[pair][i] is that atom's support entry of node kNlRun r + i (-1: none)
  int64_t n_pairs = 0;
  DevBuf<int32_t> run_off;      // [n_runs + 1]
  DevBuf<int32_t> pair_atom;    // [n_pairs]
  DevBuf<int32_t> pair_ent;     // [n_pairs][kNlRun]
};
constexpr int kNlChunk = 512;
constexpr int kNlWindow = 1024;
constexpr int kNlRun = 16;

// ---------------------------------------------------------------- context
struct KPoint {
  double k[3];
  bool gamma;
  int nmat;                     // 4 at Gamma (Hp, Hm, Bx, By), 5 with the k-term S
  DevBuf<double> cell64;        // tiled cell operators, FP64
  DevBuf<float> cell32;         // FP32 copy
  NonlocalK nl;
};

// Device descriptor of one task of a batched filter (see batch.cpp).
struct BatchTaskDev {
  const double* cm64;
  const float* cm32;
  const int32_t* cell_nodes;
  double2* buf[2];
  int64_t ld[2];
  int n_vec, nloc, nrb, nkb, nmat;
  int pad;
};
// Task descriptors of one persistent launch, passed by value in the kernel
// arguments (pointers read from the argument segment compile to global, not
// flat, accesses); larger batches launch in chunks of this many tasks.
constexpr int kBatchLaunchTasks = 32;
struct BatchTaskArgs {
  BatchTaskDev t[kBatchLaunchTasks];
};

struct FieldOps;   // SCF field solves (fields.hip)

struct StageRec {
  int stage;
  hipEvent_t start, stop;
  double flops, exec_flops, bytes;
};

}  // namespace chfsi

struct chfsi_ctx {
  int nc[3];
  double box[3];
  double h[3];
  double J;
  int p, np1, nloc, quad, nq, nq3;
  int Nd[3];
  int64_t n_nodes;
  int n_cells;
  hipStream_t stream;
  int device = 0;                             // HIP device current at chfsi_create
  chfsi::RefElement ref;
  // numbering and colouring
  std::vector<int32_t> cell_nodes_h;          // [E][nloc]
  chfsi::DevBuf<int32_t> cell_nodes;          // [E][nloc]
  int n_colours;
  std::vector<int> colour_off;                // [n_colours + 1]
  chfsi::DevBuf<int32_t> colour_cells;        // cells sorted by colour
  std::vector<double> minv_sqrt_h;            // [M] M_D^{-1/2}
  chfsi::DevBuf<double> minv_sqrt;
  // cell operator tiling
  int nrb;                                    // row blocks of 16 (padded)
  int nkb;                                    // k-steps of 4 (padded to nrb*4)
  // uniform reference matrices (host, real [nloc][nloc])
  std::vector<double> Kin, Mcons;
  std::vector<double> Cgrad[3];               // d-th component of the k-gradient matrix
  std::vector<chfsi::KPoint*> kp;
  bool have_local = false;
  // bumped by every call that rebuilds device operator data (set_local, set_atoms,
  // set_apply_form): objects holding its device pointers check it before use
  uint64_t gen = 0;
  uint64_t mf_gen = 0;                        // gen of the last matrix-free quadrature data (0: none)
  // internal scratch
  chfsi::DevBuf<double> scratch;              // reductions, small matrices
  // when set, the nonlocal coefficients of every apply use this fixed buffer
  // (nl_fixed_bytes long) instead of growing `scratch`, contracting as many
  // columns per launch as fit (the allocation-free filter entry point)
  void* nl_fixed = nullptr;
  size_t nl_fixed_bytes = 0;
  chfsi::DevBuf<double> panel;                // row panel for in-place rotations
  chfsi::DevBuf<double> cd_partial;           // adjoint cross densities per column group
  chfsi::DevBuf<int32_t> den_order;           // cell order of the density kernels (4x4x4 tiles)
  chfsi::DevBuf<double> ref_b1, ref_wq;       // 1-D interpolation table and weights (device copy)
  chfsi::DevBuf<double> occ;                  // occupations of the last density call (device copy)
  // form of the local operator: CHFSI_FORM_CELL_MATRIX (stored cell matrices)
  // or CHFSI_FORM_MATRIX_FREE (sum factorisation from the quadrature data)
  int form = 0;
  chfsi::DevBuf<double> mf_tab;               // [B: np1^2][Dq: np1^2][w: np1]
  chfsi::DevBuf<double> mf_qd;                // [E][nq^3][4]: w_q J (V, Bx, By, Bz)
  chfsi::DevBuf<float> mf_tab32, mf_qd32;     // FP32 copies for mixed precision
  chfsi::DevBuf<float> mf_kin32;              // [3][nq^3] FP32 kinetic weights per point
  // tables and work vectors of the SCF field solves (built on first use)
  std::shared_ptr<chfsi::FieldOps> fields;
  // stage timing
  bool stats_on = false;
  std::vector<chfsi::StageRec> pending;
  std::vector<hipEvent_t> event_pool;
  chfsi_stage_stats stats[CHFSI_N_STAGES] = {};
  std::string last_error;
};

namespace chfsi {
// Records HIP events around a stage's launches when timing is enabled.
class StageTimer {
 public:
  StageTimer(chfsi_ctx* c, int stage, double flops, double exec_flops, double bytes);
  ~StageTimer();
 private:
  chfsi_ctx* c_;
  StageRec rec_;
  bool on_;
};
void stats_resolve(chfsi_ctx* c);
void stats_add_host(chfsi_ctx* c, int stage, double ms);

// host setup (fe_host.cpp)
void build_mesh(chfsi_ctx* c);
void build_uniform_mats(chfsi_ctx* c);
void build_nonlocal(chfsi_ctx* c, KPoint& kp, int n_atoms, const chfsi_atom_desc* atoms);
void angular_momentum_real(int l, std::vector<cplx>& L);   // [3][2l+1][2l+1]

// dense host linear algebra (dense_host.cpp)
int cholesky_lower(std::vector<cplx>& S, int n);           // returns -1 ok, else bad column
void lower_inverse(const std::vector<cplx>& L, int n, std::vector<cplx>& Linv);
void hermitian_eig(const std::vector<cplx>& A, int n, std::vector<double>& w, std::vector<cplx>& V);

// device launchers (kernels.hip)
void launch_cell_setup(chfsi_ctx* c, KPoint& kp, const double* V, const double* B,
                       const double* U0, const double* S);
void launch_cell_to_f32(chfsi_ctx* c, KPoint& kp);
void launch_cell_products(chfsi_ctx* c, KPoint& kp, int prec, const double2* X, int64_t ldx, double2* W,
                          int64_t ldw, int n_vec, double alpha);
int check_finite(chfsi_ctx* c, const double* p, int64_t n);
// W <- alpha H_hat X + beta W + gamma X   (W is not read when beta == 0)
void apply_H(chfsi_ctx* c, KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw,
             int n_vec, int prec, double alpha, double beta, double gamma);
// W <- alpha H_hat X + beta Wold + gamma X   (Wold may equal W; not read when beta == 0)
void apply_H2(chfsi_ctx* c, KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw,
              const double2* Wold, int64_t ldo, int n_vec, int prec, double alpha, double beta,
              double gamma);
// ... + the column-scaled source sum_n rscale[n] Rs[:, n] (Rs may be null)
void apply_H3(chfsi_ctx* c, KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw,
              const double2* Wold, int64_t ldo, int n_vec, int prec, double alpha, double beta, double gamma,
              const double2* Rs, int64_t ldr, const double* rscale);
// Y[r][n] = a[n] Y[r][n] + b[n] X[r][n] with device per-column scalars
void launch_cols_axpby(chfsi_ctx* c, double2* Y, int64_t ldy, const double2* X, int64_t ldx, int64_t rows,
                       int n_vec, const double* a_d, const double* b_d);
// dV[e][q] += alpha w_q J Re sum_n l^H y, dB_d[e][q] += alpha w_q J Re sum_n l^H sigma_d y
void cross_density(chfsi_ctx* c, const double2* L, int64_t ldl, const double2* Y, int64_t ldy, int n_vec,
                   double alpha, double* dV, double* dB);
// rho += sum_n occ_d[n] u_n^H u_n, mag += sum_n occ_d[n] u_n^H sigma u_n at every quadrature point
// matrix-free local operator (matfree.hip)
bool mf_supported(const chfsi_ctx* c);
void mf_prepare(chfsi_ctx* c);
void mf_set_local(chfsi_ctx* c, const double* V, const double* B);
// W += alpha H_loc X with the matrix-free operator; alpha_d (device, or NULL)
// overrides alpha at run time (graph replays with new filter bounds)
void launch_mf_products(chfsi_ctx* c, const KPoint& kp, int prec, const double2* X, int64_t ldx, double2* W,
                        int64_t ldw, int n_vec, double alpha, const double* alpha_d = nullptr);
void densities(chfsi_ctx* c, const double2* X, int64_t ldx, int n_vec, const double* occ_d, double* rho,
               double* mag);
void launch_axpby_rows(chfsi_ctx* c, double2* W, int64_t ldw, const double2* X, int64_t ldx,
                       int64_t rows, int n_vec, double beta, double gamma);
void launch_copy_rows(chfsi_ctx* c, double2* dst, int64_t ldd, const double2* src, int64_t lds,
                      int64_t rows, int n_vec);
void gram(chfsi_ctx* c, const double2* X, int64_t ldx, const double2* Y, int64_t ldy, int64_t rows,
          int n, std::vector<cplx>& S, bool lower_only);
void rotate_inplace(chfsi_ctx* c, double2* X, int64_t ldx, int64_t rows, int n,
                    const std::vector<cplx>& Q, bool upper_triangular);
// Rayleigh-Ritz, first half: work = H X (FP64) and the projected matrix
// Hp = X^H work (n x n, host, lower half); the caller solves it (hermitian_eig)
// and rotates X by the eigenvectors (rotate_inplace), possibly later.
void rr_project(chfsi_ctx* c, int ik, const double2* X, int64_t ldx, double2* work, int64_t ldw, int n_vec,
                std::vector<cplx>& Hp);
void column_resid_norms(chfsi_ctx* c, const double2* W, int64_t ldw, const double2* X, int64_t ldx,
                        int64_t rows, int n, const double* theta, double* out);
double dot_re(chfsi_ctx* c, const double2* x, const double2* y, int64_t rows);
// batched filter support (kernels.hip)
void launch_cell_batch(hipStream_t s, bool fp64, int CB, bool has_s, const BatchTaskArgs& tasks, const int4* items,
                       int n_items, const double* alpha, int src, int grid);
int cell_batch_blocks_per_cu(bool fp64, int CB, bool has_s);
double time_cell_stage(chfsi_ctx* c, KPoint& kp, int CB, int prec, const double2* X, int64_t ldx, double2* W,
                       int64_t ldw, int n_vec, int reps);
// bytes of device scratch the nonlocal coefficients of one apply of this width need
size_t nonlocal_scratch_bytes(const KPoint& kp, int n_vec);
// the smallest fixed buffer that serves an apply of this width when the
// contraction runs one column per launch (the coefficient arrays are whole)
size_t nonlocal_scratch_bytes_min(const KPoint& kp, int n_vec);
// the scaled Chebyshev recurrence of chfsi_cheb_filter (arguments checked)
void check_filter_args(chfsi_ctx* c, void* X, int64_t ldx, void* work, int64_t ldw, int n_vec, int degree,
                       double a, double b, double a0, int prec_mode);
void cheb_filter_run(chfsi_ctx* c, KPoint& kp, void* X, int64_t ldx, void* work, int64_t ldw, int n_vec,
                     int degree, double a, double b, double a0, int prec_mode);
KPoint& kpoint_of(chfsi_ctx* c, int ik);
// SCF fields (fields.hip): integrals and the eqn:innerPdt product at the
// quadrature points, screened Poisson solves, exchange, the two-grid transfer
double field_integral(chfsi_ctx* c, const double* g);
double field_inner(chfsi_ctx* c, const double* r1, const double* m1, const double* r2, const double* m2);
int screened_poisson(chfsi_ctx* c, double kappa2, double scale, const double* g, double* u_q, double tol,
                     int max_iter, double* rel);
void launch_exchange(chfsi_ctx* c, int64_t n_points, const double* rho, const double* m, const double* vadd,
                     const double* badd, double* V, double* B);
// out = a x + b y (y may be null: out = a x; a NaN in y propagates even if b = 0)
void field_axpby(chfsi_ctx* c, int64_t n, double a, const double* x, double b, const double* y, double* out);
void field_fill(chfsi_ctx* c, int64_t n, double v, double* out);
void interpolate_block(chfsi_ctx* cc, chfsi_ctx* cf, const double2* Yc, int64_t ldc, double2* Yf, int64_t ldf,
                       int n_vec);
// looks up this device's copy of the allocation-free entry point's scratch
// array (once per device; the device must be current)
void noalloc_scratch_init();
// W <- beta W + gamma X + alpha H_nl X (nonlocal part and recurrence terms of one
// apply).  alpha_d, bg_d (device, or null): alpha and (beta, gamma) read at run
// time; the term flags still follow beta != 0, gamma != 0.  scratch: caller-owned,
// >= nonlocal_scratch_bytes(kp, n_vec), or null for the context's growable buffer.
void apply_nonlocal_init(chfsi_ctx* c, KPoint& kp, const double2* X, int64_t ldx, double2* W, int64_t ldw,
                         int n_vec, int prec, double alpha, double beta, double gamma, const double* alpha_d,
                         const double* bg_d, void* scratch);
void launch_fill_random(chfsi_ctx* c, double2* X, int64_t n_rows, int n_vec, int64_t ld,
                        uint64_t seed, int64_t row0, int col0, int64_t n_total_cols);
}  // namespace chfsi
