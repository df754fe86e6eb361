// Per-stage HIP-event timing of the library's launches.
#include "internal.h"

namespace chfsi {

static hipEvent_t take_event(chfsi_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  CHFSI_HIP(hipEventCreate(&e));
  return e;
}

StageTimer::StageTimer(chfsi_ctx* c, int stage, double flops, double exec_flops, double bytes)
    : c_(c), on_(c->stats_on) {
  if (!on_) return;
  rec_.stage = stage;
  rec_.flops = flops;
  rec_.exec_flops = exec_flops;
  rec_.bytes = bytes;
  rec_.start = take_event(c);
  rec_.stop = take_event(c);
  CHFSI_HIP(hipEventRecord(rec_.start, c->stream));
}

StageTimer::~StageTimer() {
  if (!on_) return;
  if (hipEventRecord(rec_.stop, c_->stream) == hipSuccess) c_->pending.push_back(rec_);
}

void stats_resolve(chfsi_ctx* c) {
  if (c->pending.empty()) return;
  CHFSI_HIP(hipStreamSynchronize(c->stream));
  for (auto& r : c->pending) {
    float ms = 0.0f;
    CHFSI_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
    auto& s = c->stats[r.stage];
    s.launches += 1;
    s.ms += ms;
    s.flops += r.flops;
    s.exec_flops += r.exec_flops;
    s.bytes += r.bytes;
    c->event_pool.push_back(r.start);
    c->event_pool.push_back(r.stop);
  }
  c->pending.clear();
}

void stats_add_host(chfsi_ctx* c, int stage, double ms) {
  if (!c->stats_on) return;
  auto& s = c->stats[stage];
  s.launches += 1;
  s.ms += ms;
}

}  // namespace chfsi

using namespace chfsi;

extern "C" {

int chfsi_stats_enable(chfsi_ctx* c, int enable) {
  if (!c) return CHFSI_EINVAL;
  c->stats_on = enable != 0;
  return CHFSI_OK;
}

int chfsi_stats_read(chfsi_ctx* c, chfsi_stage_stats* out) {
  if (!c || !out) return CHFSI_EINVAL;
  try {
    stats_resolve(c);
  } catch (const Error& e) {
    c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    c->last_error = e.what();
    return CHFSI_EINVAL;
  }
  for (int i = 0; i < CHFSI_N_STAGES; ++i) out[i] = c->stats[i];
  return CHFSI_OK;
}

int chfsi_stats_reset(chfsi_ctx* c) {
  if (!c) return CHFSI_EINVAL;
  try {
    stats_resolve(c);
  } catch (const Error& e) {
    c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return CHFSI_ENOMEM;
  } catch (const std::exception& e) {
    c->last_error = e.what();
    return CHFSI_EINVAL;
  }
  for (int i = 0; i < CHFSI_N_STAGES; ++i) c->stats[i] = chfsi_stage_stats{};
  return CHFSI_OK;
}

}  // extern "C"
