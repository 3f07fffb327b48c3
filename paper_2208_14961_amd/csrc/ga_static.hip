// ga_static.hip -- ga_step_static: one generation, as ga_step computes it,
// with its device workspace in a fixed array of the library instead of
// memory allocated on first use.  For callers that cannot allocate (work
// under HIP graph capture, serving loops that forbid allocation).
#include <hip/hip_runtime.h>

#include <mutex>

#include "ga_internal.h"

namespace ga {

// The workspace of a step: the run state, then one selection workspace
// (radix-select histograms and per-tile counts), which covers populations
// up to kMaxN, the library's limit.  One copy per device, held until the
// process ends; every call on a device shares it.
constexpr size_t kStateBytes = 256;
constexpr size_t kScratchBytes = kStateBytes + ((sizeof(SelWork) + 255) & ~(size_t)255);
constexpr uint32_t kStaticMaxN = kMaxN;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The device address of `scratch` on each device, looked up once per
// device with that device current.  In host code the name `scratch` is a
// host-side stand-in, never a device address: only these pointers are
// passed to kernels.
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};

static ga_status scratch_on_current_device(void** out) {
  int dev = 0;
  ga_status st = hip_status(hipGetDevice(&dev), "hipGetDevice");
  if (st != GA_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d: the fixed workspace supports devices 0..%d", dev, kMaxDevices - 1);
    return GA_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    st = hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st != GA_OK) return st;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GA_OK;
}

// Sets the run state for a step from generation `gen` (no stop condition)
// and clears the selection histograms, which the selection kernels expect
// zero on entry.  One block.
__global__ __launch_bounds__(kBlock) void static_prepare_kernel(RunState* st, SelWork* ws,
                                                                uint32_t gen, uint32_t clear) {
  if (threadIdx.x == 0) {
    st->best = ~0ull;
    st->gen_base = gen;
    st->found_gen = ~0u;
    st->final_gen = gen + 1;
  }
  if (clear)
    for (uint32_t i = threadIdx.x; i < 4096; i += kBlock) {
      ws->h1[i] = 0;
      ws->h2[i] = 0;
    }
}

}  // namespace ga

using namespace ga;

extern "C" ga_status ga_step_static(const ga_config* cfg, const uint32_t* pop_in,
                                    const uint32_t* keys_in, uint32_t* pop_out,
                                    uint32_t* keys_out, uint32_t gen_in, void* stream) {
  ga_status st = validate(cfg);
  if (st != GA_OK) return st;
  if (cfg->n > kStaticMaxN) {
    set_error("n=%u: the fixed workspace holds populations up to %u", cfg->n, kStaticMaxN);
    return GA_EINVAL;
  }
  if (!pop_in || !keys_in || !pop_out || !keys_out || pop_in == pop_out ||
      keys_in == keys_out) {
    set_error("ga_step_static needs four distinct non-NULL buffers");
    return GA_EINVAL;
  }
  if (gen_in == 0xffffffffu) {
    set_error("gen_in too large");
    return GA_EINVAL;
  }
  void* base = nullptr;
  st = scratch_on_current_device(&base);
  if (st != GA_OK) return st;
  RunState* state = reinterpret_cast<RunState*>(base);
  SelWork* sel = reinterpret_cast<SelWork*>(static_cast<unsigned char*>(base) + kStateBytes);
  hipStream_t s = (hipStream_t)stream;
  // generation g lives in the "a" buffers iff g is even
  uint32_t* pi = const_cast<uint32_t*>(pop_in);
  uint32_t* ki = const_cast<uint32_t*>(keys_in);
  const bool odd = gen_in & 1u;
  const PopDesc d = make_desc(cfg, odd ? pop_out : pi, odd ? pi : pop_out,
                              odd ? keys_out : ki, odd ? ki : keys_out, state, 0xffffffffu, 0);
  const uint32_t count = cfg->selection == GA_SEL_PAPER ? cfg->n / 2 : cfg->elite;
  hipLaunchKernelGGL(static_prepare_kernel, dim3(1), dim3(kBlock), 0, s, state, sel, gen_in,
                     count > 0 ? 1u : 0u);
  st = hip_status(hipGetLastError(), "prepare kernel");
  if (st != GA_OK) return st;
  if (count > 0) {
    st = hip_status(launch_select(d, count, sel, 0, nullptr, s), "selection kernels");
    if (st != GA_OK) return st;
  }
  return hip_status(launch_children_one(d, 0, s), "children kernel");
}
