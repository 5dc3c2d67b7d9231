// slq_weight_static: the exact weight of Eq. 1 without a plan and without any
// allocation, for callers that cannot allocate device memory.  The plan's
// workspace is laid out in a file-scope device array, one copy per GPU, whose
// device address is looked up once per device; E and E^{-1} are rebuilt in it
// on every call.  Every call on a GPU shares that GPU's array (calls that
// overlap in time on one GPU race); nothing in it is assumed to persist from
// the previous call: every buffer the evaluation reads is written first
// within the same call (status, D and the reflector counts are filled, the
// factorisations overwrite the rest).
#include <mutex>

#include "slq_internal.h"

namespace slq {

// Host code never uses this name as a device address (on the host it is a
// stand-in); the per-device pointer from hipGetSymbolAddress is used instead.
static __device__ __align__(256) unsigned char scratch[SLQ_STATIC_SCRATCH_BYTES];

static std::mutex g_static_mu;
static void* g_static_ptr[64];  // device address of scratch, per device (null: not looked up)

static int static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= 64) {
    set_error("device index out of range for the static scratch table");
    return SLQ_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return SLQ_ERR_DEVICE;
    }
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  return SLQ_OK;
}

int check_model_public(const slq_model* m);

}  // namespace slq

using namespace slq;

extern "C" {

int slq_weight_static(const slq_model* model, int32_t batch, const int8_t* d_s, double* d_logabs, int8_t* d_sign,
                      int32_t* d_status, hipStream_t stream) {
  SLQ_TRY(check_model_public(model));
  if (batch < 0) {
    set_error("batch must be >= 0");
    return SLQ_ERR_ARG;
  }
  if (batch == 0) return SLQ_OK;
  if (!d_s || !d_logabs || !d_sign) {
    set_error("d_s, d_logabs and d_sign must not be NULL");
    return SLQ_ERR_ARG;
  }
  if (model->chain_prec != SLQ_PREC_FP64 && model->chain_prec != SLQ_PREC_FP64_DENSE &&
      model->chain_prec != SLQ_PREC_CHECKERBOARD) {
    set_error("slq_weight_static evaluates FP64 chains only");
    return SLQ_ERR_ARG;
  }
  Plan p{};
  p.m = *model;
  p.n = model->lx * model->ly;
  p.L = model->n_slices;
  p.max_batch = batch;
  const size_t need = plan_layout(p, 0, nullptr);
  if (need > (size_t)SLQ_STATIC_SCRATCH_BYTES) {
    set_error("the evaluation needs " + std::to_string(need) + " bytes of scratch, more than the " +
              std::to_string((size_t)SLQ_STATIC_SCRATCH_BYTES) + " of slq_weight_static");
    return SLQ_ERR_WORKSPACE;
  }
  int dev = 0;
  SLQ_HIP(hipGetDevice(&dev));
  p.device = dev;
  void* base = nullptr;
  SLQ_TRY(static_scratch(dev, &base));
  plan_layout(p, 0, (char*)base);
  SLQ_TRY(plan_init(p, stream));
  int32_t* status = d_status ? d_status : p.status;
  SLQ_TRY(fill_i32(status, batch, 0, stream));
  SLQ_TRY(launch_check_spins(p, batch, d_s, status, stream));
  SLQ_TRY(run_chain(p, batch, d_s, 0, status, stream));
  return launch_finish(p, batch, nullptr, d_logabs, d_sign, status, stream);
}

}  // extern "C"
