// Allocation-free form of the Chebyshev filter: the nonlocal coefficient
// scratch of every apply lives in a fixed device array of this file instead of
// the context's growable buffer, so the call issues no device allocation.
#include <mutex>

#include "internal.h"

namespace chfsi {
namespace {

// The array itself.  Its name is a host-side stand-in in host code: kernels get
// the per-device address looked up below, never the name.
static __device__ __align__(256) unsigned char scratch[CHFSI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

void noalloc_scratch_init() {
  int dev = 0;
  CHFSI_HIP(hipGetDevice(&dev));
  CHFSI_CHECK(dev >= 0 && dev < kMaxDevices, CHFSI_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[dev]) return;
  void* p = nullptr;
  CHFSI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  CHFSI_CHECK(p != nullptr, CHFSI_EHIP, "hipGetSymbolAddress returned a null address");
  g_ptr[dev] = p;
  g_done[dev] = true;
}

static void* noalloc_scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (dev >= 0 && dev < kMaxDevices && g_done[dev]) ? g_ptr[dev] : nullptr;
}

}  // namespace chfsi

using namespace chfsi;

extern "C" int chfsi_cheb_filter_noalloc(chfsi_ctx* c, int ik, void* X, int64_t ldx, void* work, int64_t ldw,
                                         int n_vec, int degree, double a, double b, double a0, int prec_mode) {
  if (!c) return CHFSI_EINVAL;
  try {
    check_filter_args(c, X, ldx, work, ldw, n_vec, degree, a, b, a0, prec_mode);
    KPoint& kp = kpoint_of(c, ik);
    const size_t need = nonlocal_scratch_bytes_min(kp, n_vec);
    CHFSI_CHECK(need <= (size_t)CHFSI_NOALLOC_SCRATCH_BYTES, CHFSI_EINVAL,
                "chfsi_cheb_filter_noalloc: the nonlocal coefficients of " + std::to_string(n_vec) +
                    " columns need " + std::to_string(need) + " bytes of scratch, above the fixed " +
                    std::to_string((size_t)CHFSI_NOALLOC_SCRATCH_BYTES) +
                    " (use chfsi_cheb_filter or fewer columns per call)");
    void* p = noalloc_scratch_ptr(c->device);
    CHFSI_CHECK(p != nullptr, CHFSI_ESTATE, "fixed scratch of this device was not looked up");
    // the fixed buffer replaces the context's scratch for this call only; stage
    // timers stay off (their events come from a growable pool)
    struct Guard {
      chfsi_ctx* c;
      bool stats;
      ~Guard() {
        c->nl_fixed = nullptr;
        c->nl_fixed_bytes = 0;
        c->stats_on = stats;
      }
    } g{c, c->stats_on};
    c->nl_fixed = p;
    c->nl_fixed_bytes = CHFSI_NOALLOC_SCRATCH_BYTES;
    c->stats_on = false;
    cheb_filter_run(c, kp, X, ldx, work, ldw, n_vec, degree, a, b, a0, prec_mode);
  } catch (const chfsi::Error& e) {
    c->last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    c->last_error = e.what();
    return CHFSI_EINVAL;
  }
  return CHFSI_OK;
}
