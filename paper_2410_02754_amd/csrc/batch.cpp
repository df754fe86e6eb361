// Batched Chebyshev filtering of many independent operators (the k-points of
// a Monkhorst-Pack grid and independent systems of uneven size; the
// eigenproblems of different k are independent, Sec. III.B).
//
// Per recurrence step the projector terms and the initialisation run per task;
// the cell products of all tasks run as one persistent launch per colour phase
// (and per tile shape / k-term variant) walking a static item list.  Column
// tile widths are chosen per task by timing the candidates on the task's own
// data.  The whole degree-m filter of all tasks is captured into a hipGraph once
// and replayed for any bounds: every recurrence coefficient is read from device
// tables that are refreshed before each replay.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <tuple>

#include "internal.h"

using namespace chfsi;

struct BatchGroup {
  int cb;
  bool has_s;
  int chunk;                                 // tasks [chunk * kBatchLaunchTasks, +kBatchLaunchTasks)
  BatchTaskArgs args;                        // their descriptors, by value for the launch
  std::vector<int> n_items;                  // per colour
  std::vector<DevBuf<int4>*> items;          // per colour
  int grid[2];                               // persistent grid: [0] FP32, [1] FP64
  ~BatchGroup() {
    for (auto* p : items) delete p;
  }
};

struct chfsi_batch {
  std::vector<chfsi_batch_task> tasks;
  std::vector<KPoint*> kps;
  int degree = 0, prec = 0, flags = 0;
  hipStream_t stream = nullptr;
  std::vector<int> cb;                       // chosen column blocks per task
  std::vector<double> tune_ms;               // [n_tasks][3] timings of CB = 1, 2, 4 (or -1)
  std::vector<BatchGroup*> groups;
  int max_colours = 0;
  DevBuf<double> coef_tab;                   // alpha [degree][n_tasks], then (beta, gamma) [degree][n_tasks][2]
  struct {
    double* ptr = nullptr;
  } alpha_tab, bg_tab;                       // views into coef_tab
  double* coef_h = nullptr;                  // pinned host copy of coef_tab
  hipEvent_t coef_done = nullptr;            // the last upload of coef_h has been read
  DevBuf<unsigned char> nl_scratch;          // nonlocal partial sums, shared by the tasks (one stream)
  std::vector<uint64_t> gen;                 // context generations at creation
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n_captures = 0, n_replays = 0;
  double capture_ms = 0.0, instantiate_ms = 0.0;
  std::string last_error;
  ~chfsi_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (coef_done) (void)hipEventDestroy(coef_done);
    if (coef_h) (void)hipHostFree(coef_h);
    for (auto* g : groups) delete g;
  }
};

static int cb_index(int cb) { return cb == 4 ? 2 : cb == 2 ? 1 : 0; }

// item lists of one (CB, k-term, task chunk) group, one list per colour, in XCD
// order; item task indices are local to the chunk
static void build_items(chfsi_batch* b, BatchGroup& g) {
  const int nt = (int)b->tasks.size();
  const int t0 = g.chunk * kBatchLaunchTasks, t1 = std::min(nt, t0 + kBatchLaunchTasks);
  g.n_items.assign(b->max_colours, 0);
  g.items.assign(b->max_colours, nullptr);
  for (int col = 0; col < b->max_colours; ++col) {
    std::vector<std::vector<int4>> per_xcd(8);
    int unit = 0;
    for (int t = t0; t < t1; ++t) {
      if (b->cb[t] != g.cb || (!b->kps[t]->gamma) != g.has_s) continue;
      chfsi_ctx* c = b->tasks[t].ctx;
      if (col >= c->n_colours) continue;
      std::vector<int32_t> cells(c->colour_off[col + 1] - c->colour_off[col]);
      if (!cells.empty())
        CHFSI_HIP(hipMemcpy(cells.data(), c->colour_cells.ptr + c->colour_off[col], cells.size() * sizeof(int32_t),
                            hipMemcpyDeviceToHost));
      const int nrt = (c->nrb + 1) / 2;
      const int nct = (b->tasks[t].n_vec + 32 * g.cb - 1) / (32 * g.cb);
      for (int e : cells)
        for (int ct = 0; ct < nct; ++ct, ++unit)
          for (int rt = 0; rt < nrt; ++rt) per_xcd[unit % 8].push_back(int4{t - t0, e, rt, ct});
    }
    size_t len = 0;
    for (auto& v : per_xcd) len = std::max(len, v.size());
    std::vector<int4> flat(8 * len, int4{-1, 0, 0, 0});
    for (int x = 0; x < 8; ++x)
      for (size_t j = 0; j < per_xcd[x].size(); ++j) flat[8 * j + x] = per_xcd[x][j];
    g.n_items[col] = (int)flat.size();
    g.items[col] = new DevBuf<int4>();
    if (!flat.empty()) g.items[col]->upload(flat.data(), flat.size(), b->stream);
  }
  for (int f = 0; f < 2; ++f) {
    int maxn = 0;
    for (int n : g.n_items) maxn = std::max(maxn, n);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
      int v = 0;
      if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    const int cap = cus * cell_batch_blocks_per_cu(f == 1, g.cb, g.has_s);
    g.grid[f] = std::max(8, 8 * ((std::min(maxn, cap) + 7) / 8));
  }
  CHFSI_HIP(hipStreamSynchronize(b->stream));
}

// the degree-m filter of every task, enqueued on the batch stream.  Every
// recurrence coefficient is read from the batch's device tables (alpha_tab,
// bg_tab), so the enqueued work does not depend on the bounds and one captured
// graph replays for any bounds.
static void run_filter(chfsi_batch* b) {
  const int nt = (int)b->tasks.size(), m = b->degree;
  for (int k = 1; k <= m; ++k) {
    const int src = (k - 1) & 1;
    const int prec = (b->prec == CHFSI_PREC_MIXED && k < m) ? CHFSI_PREC_MIXED : CHFSI_PREC_FP64;
    const double* al_k = b->alpha_tab.ptr + (size_t)(k - 1) * nt;
    const double* bg_k = b->bg_tab.ptr + (size_t)(k - 1) * nt * 2;
    for (int t = 0; t < nt; ++t) {
      const auto& tk = b->tasks[t];
      double2* buf[2] = {(double2*)tk.X_d, (double2*)tk.work_d};
      const int64_t ld[2] = {tk.ldx, tk.ldw};
      // the host values only select the terms present (k = 1 has no Y_{k-2} term);
      // the kernels read alpha, beta, gamma from the tables
      apply_nonlocal_init(tk.ctx, *b->kps[t], buf[src], ld[src], buf[src ^ 1], ld[src ^ 1], tk.n_vec, prec, 1.0,
                          k == 1 ? 0.0 : 1.0, 1.0, al_k + t, bg_k + 2 * t, b->nl_scratch.ptr);
    }
    for (int col = 0; col < b->max_colours; ++col)
      for (auto* g : b->groups) {
        if (g->n_items[col] == 0) continue;
        launch_cell_batch(b->stream, prec == CHFSI_PREC_FP64, g->cb, g->has_s, g->args, g->items[col]->ptr,
                          g->n_items[col], al_k + g->chunk * kBatchLaunchTasks, src,
                          g->grid[prec == CHFSI_PREC_FP64]);
      }
    // matrix-free tasks: their own colour launches, alpha read from the table
    for (int t = 0; t < nt; ++t) {
      if (b->cb[t] != 0) continue;
      const auto& tk = b->tasks[t];
      double2* buf[2] = {(double2*)tk.X_d, (double2*)tk.work_d};
      const int64_t ld[2] = {tk.ldx, tk.ldw};
      launch_mf_products(tk.ctx, *b->kps[t], prec, buf[src], ld[src], buf[src ^ 1], ld[src ^ 1], tk.n_vec, 0.0,
                         al_k + t);
    }
  }
  if (m & 1)
    for (int t = 0; t < nt; ++t) {
      const auto& tk = b->tasks[t];
      launch_copy_rows(tk.ctx, (double2*)tk.X_d, tk.ldx, (const double2*)tk.work_d, tk.ldw, 2 * tk.ctx->n_nodes,
                       tk.n_vec);
    }
}

// scaled-recurrence coefficients of every task: alpha_k, and (beta_k, gamma_k =
// -c alpha_k) with Y_k = alpha_k H Y_{k-1} + beta_k Y_{k-2} + gamma_k Y_{k-1}
static void upload_coeffs(chfsi_batch* b, const std::vector<double>& bounds) {
  const int nt = (int)b->tasks.size(), m = b->degree;
  for (int t = 0; t < nt; ++t) {
    const double a = bounds[3 * t], bb = bounds[3 * t + 1], a0 = bounds[3 * t + 2];
    const double e = 0.5 * (bb - a), c = 0.5 * (bb + a), s1 = e / (a0 - c);
    double sg = s1;
    double al = s1 / e;
    b->coef_h[t] = al;
    b->coef_h[(size_t)m * nt + 2 * t] = 0.0;
    b->coef_h[(size_t)m * nt + 2 * t + 1] = -c * al;
    for (int k = 2; k <= m; ++k) {
      const double sn = 1.0 / (2.0 / s1 - sg);
      al = 2.0 * sn / e;
      b->coef_h[(size_t)(k - 1) * nt + t] = al;
      b->coef_h[(size_t)m * nt + 2 * ((size_t)(k - 1) * nt + t)] = -sg * sn;
      b->coef_h[(size_t)m * nt + 2 * ((size_t)(k - 1) * nt + t) + 1] = -c * al;
      sg = sn;
    }
  }
  // the host table is pinned memory owned by the batch: the copy is ordered on
  // the stream before the filter's kernels, and the next upload waits for it
  CHFSI_HIP(hipEventSynchronize(b->coef_done));
  CHFSI_HIP(hipMemcpyAsync(b->alpha_tab.ptr, b->coef_h, (size_t)3 * m * nt * sizeof(double), hipMemcpyHostToDevice,
                           b->stream));
  CHFSI_HIP(hipEventRecord(b->coef_done, b->stream));
}

extern "C" {

int chfsi_batch_create(int n_tasks, const chfsi_batch_task* tasks, int degree, int prec_mode, int flags,
                       chfsi_batch** out) {
  chfsi_batch* b = nullptr;
  try {
    CHFSI_CHECK(n_tasks >= 1 && tasks && out, CHFSI_EINVAL, "need n_tasks >= 1, tasks and out");
    CHFSI_CHECK(degree >= 1, CHFSI_EINVAL, "degree must be >= 1");
    CHFSI_CHECK(prec_mode == CHFSI_PREC_FP64 || prec_mode == CHFSI_PREC_MIXED, CHFSI_EINVAL, "unknown precision");
    b = new chfsi_batch();
    b->degree = degree;
    b->prec = prec_mode;
    b->flags = flags;
    b->tasks.assign(tasks, tasks + n_tasks);
    b->stream = tasks[0].ctx ? tasks[0].ctx->stream : nullptr;
    CHFSI_CHECK(!(flags & CHFSI_BATCH_GRAPH) || b->stream != nullptr, CHFSI_EINVAL,
                "graph capture needs a non-default stream");
    for (int t = 0; t < n_tasks; ++t) {
      const auto& tk = tasks[t];
      CHFSI_CHECK(tk.ctx != nullptr, CHFSI_EINVAL, "task without a context");
      CHFSI_CHECK(tk.ctx->have_local, CHFSI_ESTATE, "chfsi_set_local has not been called for a task");
      CHFSI_CHECK(tk.ctx->stream == b->stream, CHFSI_EINVAL, "all tasks must share one stream");
      CHFSI_CHECK(tk.ik >= 0 && tk.ik < (int)tk.ctx->kp.size(), CHFSI_EINVAL, "k-point index out of range");
      CHFSI_CHECK(tk.X_d && tk.work_d && tk.X_d != tk.work_d && tk.n_vec >= 1 && tk.ldx >= tk.n_vec &&
                      tk.ldw >= tk.n_vec,
                  CHFSI_EINVAL, "bad task block");
      for (int u = 0; u < t; ++u)
        CHFSI_CHECK(tasks[u].X_d != tk.X_d && tasks[u].work_d != tk.work_d, CHFSI_EINVAL,
                    "tasks must not share X or work buffers");
      b->kps.push_back(tk.ctx->kp[tk.ik]);
      b->max_colours = std::max(b->max_colours, tk.ctx->n_colours);
    }
    // tile shapes: timed candidates, or the widest useful one
    b->cb.assign(n_tasks, 4);
    b->tune_ms.assign((size_t)n_tasks * 3, -1.0);
    const int tprec = prec_mode == CHFSI_PREC_MIXED ? CHFSI_PREC_MIXED : CHFSI_PREC_FP64;
    for (int t = 0; t < n_tasks; ++t) {
      const auto& tk = tasks[t];
      if (tk.ctx->form == CHFSI_FORM_MATRIX_FREE) {
        b->cb[t] = 0;   // its own per-task launches, outside the persistent groups
        continue;
      }
      const int widest = tk.n_vec > 64 ? 4 : tk.n_vec > 32 ? 2 : 1;
      b->cb[t] = widest;
      if (!(flags & CHFSI_BATCH_AUTOTUNE)) continue;
      // fastest candidate; a narrower tile must win by more than 1 % (it costs more
      // operator reads per column)
      double best = 1e300;
      for (int cb : {4, 2, 1}) {
        if (cb > widest) continue;
        const double ms = time_cell_stage(tk.ctx, *b->kps[t], cb, tprec, (const double2*)tk.X_d, tk.ldx,
                                          (double2*)tk.work_d, tk.ldw, tk.n_vec, 2);
        b->tune_ms[(size_t)t * 3 + cb_index(cb)] = ms;
        if (ms < best * 0.99) {
          best = ms;
          b->cb[t] = cb;
        }
      }
    }
    std::map<std::tuple<int, int, bool>, int> gid;
    for (int t = 0; t < n_tasks; ++t) {
      if (b->cb[t] == 0) continue;
      auto key = std::make_tuple(t / kBatchLaunchTasks, b->cb[t], !b->kps[t]->gamma);
      if (!gid.count(key)) {
        gid[key] = (int)b->groups.size();
        auto* g = new BatchGroup();
        g->chunk = std::get<0>(key);
        g->cb = std::get<1>(key);
        g->has_s = std::get<2>(key);
        b->groups.push_back(g);
      }
    }
    for (auto* g : b->groups) build_items(b, *g);
    std::vector<BatchTaskDev> dt(n_tasks);
    size_t nl_bytes = 0;
    for (int t = 0; t < n_tasks; ++t) {
      const auto& tk = tasks[t];
      chfsi_ctx* c = tk.ctx;
      KPoint& kp = *b->kps[t];
      dt[t].cm64 = kp.cell64.ptr;
      dt[t].cm32 = kp.cell32.ptr;
      dt[t].cell_nodes = c->cell_nodes.ptr;
      dt[t].buf[0] = (double2*)tk.X_d;
      dt[t].buf[1] = (double2*)tk.work_d;
      dt[t].ld[0] = tk.ldx;
      dt[t].ld[1] = tk.ldw;
      dt[t].n_vec = tk.n_vec;
      dt[t].nloc = c->nloc;
      dt[t].nrb = c->nrb;
      dt[t].nkb = c->nkb;
      dt[t].nmat = kp.nmat;
      dt[t].pad = 0;
      nl_bytes = std::max(nl_bytes, nonlocal_scratch_bytes(kp, tk.n_vec));
      b->gen.push_back(c->gen);
    }
    for (auto* g : b->groups) {
      g->args = BatchTaskArgs{};
      for (int j = 0; j < kBatchLaunchTasks && g->chunk * kBatchLaunchTasks + j < n_tasks; ++j)
        g->args.t[j] = dt[g->chunk * kBatchLaunchTasks + j];
    }
    // the batch's own device memory: captured kernels hold these pointers, which
    // no call on the contexts can move
    b->nl_scratch.alloc(std::max<size_t>(nl_bytes, 16));
    b->coef_tab.alloc((size_t)3 * degree * n_tasks);
    b->alpha_tab.ptr = b->coef_tab.ptr;
    b->bg_tab.ptr = b->coef_tab.ptr + (size_t)degree * n_tasks;
    CHFSI_HIP(hipHostMalloc((void**)&b->coef_h, (size_t)3 * degree * n_tasks * sizeof(double), hipHostMallocDefault));
    CHFSI_HIP(hipEventCreateWithFlags(&b->coef_done, hipEventDisableTiming));
    CHFSI_HIP(hipEventRecord(b->coef_done, b->stream));
    CHFSI_HIP(hipStreamSynchronize(b->stream));
    *out = b;
    return CHFSI_OK;
  } catch (const Error& e) {
    if (b) {
      b->last_error = e.msg;
      delete b;
    }
    return e.code;
  } catch (const std::exception&) {
    delete b;
    return CHFSI_ENOMEM;
  }
}

int chfsi_batch_filter(chfsi_batch* b, const double* a, const double* bb, const double* a0) {
  if (!b) return CHFSI_EINVAL;
  try {
    const int nt = (int)b->tasks.size();
    CHFSI_CHECK(a && bb && a0, CHFSI_EINVAL, "bounds must be non-NULL");
    std::vector<double> bounds(3 * (size_t)nt);
    for (int t = 0; t < nt; ++t) {
      CHFSI_CHECK(std::isfinite(a[t]) && std::isfinite(bb[t]) && std::isfinite(a0[t]) && a0[t] < a[t] &&
                      a[t] < bb[t],
                  CHFSI_EINVAL, "filter bounds must satisfy a0 < a < b");
      bounds[3 * t] = a[t];
      bounds[3 * t + 1] = bb[t];
      bounds[3 * t + 2] = a0[t];
    }
    for (int t = 0; t < nt; ++t)
      CHFSI_CHECK(b->tasks[t].ctx->gen == b->gen[t], CHFSI_ESTATE,
                  "a task's context was rebuilt (set_local, set_atoms or set_apply_form) after "
                  "chfsi_batch_create; create the batch again");
    upload_coeffs(b, bounds);
    if (!(b->flags & CHFSI_BATCH_GRAPH)) {
      run_filter(b);
      return CHFSI_OK;
    }
    if (!b->exec) {
      std::vector<bool> stats(nt);
      for (int t = 0; t < nt; ++t) {
        stats[t] = b->tasks[t].ctx->stats_on;
        b->tasks[t].ctx->stats_on = false;   // no event records inside the capture
      }
      const auto t0 = std::chrono::steady_clock::now();
      CHFSI_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      try {
        run_filter(b);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(b->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        for (int t = 0; t < nt; ++t) b->tasks[t].ctx->stats_on = stats[t];
        throw;
      }
      CHFSI_HIP(hipStreamEndCapture(b->stream, &b->graph));
      for (int t = 0; t < nt; ++t) b->tasks[t].ctx->stats_on = stats[t];
      const auto t1 = std::chrono::steady_clock::now();
      CHFSI_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
      const auto t2 = std::chrono::steady_clock::now();
      b->capture_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
      b->instantiate_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
      ++b->n_captures;
    } else {
      ++b->n_replays;
    }
    CHFSI_HIP(hipGraphLaunch(b->exec, b->stream));
    return CHFSI_OK;
  } catch (const Error& e) {
    b->last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    b->last_error = e.what();
    return CHFSI_ENOMEM;
  }
}

int chfsi_batch_tiles(const chfsi_batch* b, int* cb_out, double* tune_ms) {
  if (!b) return CHFSI_EINVAL;
  for (size_t t = 0; t < b->tasks.size(); ++t) {
    if (cb_out) cb_out[t] = 32 * b->cb[t];
    if (tune_ms)
      for (int j = 0; j < 3; ++j) tune_ms[3 * t + j] = b->tune_ms[3 * t + j];
  }
  return CHFSI_OK;
}

int chfsi_batch_graph_info(const chfsi_batch* b, int* n_captures, int* n_replays, double* capture_ms,
                           double* instantiate_ms) {
  if (!b) return CHFSI_EINVAL;
  if (n_captures) *n_captures = b->n_captures;
  if (n_replays) *n_replays = b->n_replays;
  if (capture_ms) *capture_ms = b->capture_ms;
  if (instantiate_ms) *instantiate_ms = b->instantiate_ms;
  return CHFSI_OK;
}

int chfsi_batch_destroy(chfsi_batch* b) {
  if (!b) return CHFSI_OK;
  (void)hipStreamSynchronize(b->stream);
  delete b;
  return CHFSI_OK;
}

const char* chfsi_batch_last_error(const chfsi_batch* b) { return b ? b->last_error.c_str() : ""; }

}  // extern "C"
