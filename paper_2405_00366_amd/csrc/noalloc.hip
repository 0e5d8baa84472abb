// A CIM run for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation).
//
// l0cim_mfcim_run takes its scratch (exchange words of the resident
// launches, the abort word, per-workgroup energies, the streamed launch's
// ping-pong copy) from a caller workspace.  This variant takes it from a
// file-scope device array of kScratchBytes that every device the library runs
// on holds until the process ends.  Host code never passes the array's name
// to a kernel (on the host it is a stand-in, not a device address): its
// device address is looked up once per device with hipGetSymbolAddress and
// kept.  The launches are the same as l0cim_mfcim_run's except that the
// matrix-core form, whose panel copy of J does not fit, is never taken.
// The launch sequence clears what must start at zero (the exchange words and
// the abort word) with a kernel; calls that overlap on one device race on the
// array.
#include <mutex>

#include "kernels.h"

namespace l0 {
namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's copy of `scratch`, looked up on
// the first call on that device.
l0cim_status scratch_address(void** out) {
  int dev = 0;
  L0_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(L0CIM_ERR_HIP, "mfcim_run_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "mfcim_run_noalloc: hipGetSymbolAddress(scratch)");
    if (!p) return set_error(L0CIM_ERR_HIP, "mfcim_run_noalloc: scratch has no device address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return L0CIM_OK;
}

}  // namespace
}  // namespace l0

using namespace l0;

extern "C" {

size_t l0cim_noalloc_scratch_bytes(void) { return kScratchBytes; }

l0cim_status l0cim_mfcim_run_noalloc(l0cim_dtype dtype, int32_t n, int32_t P, l0cim_dtype j_dtype,
                                     const void* J, int64_t ldj, const float* row_scale, const void* z,
                                     double eta, const l0cim_cim_params* prm, void* c, void* e,
                                     uint8_t* sigma, double* H, void* trace, int32_t trace_steps,
                                     int32_t* status, void* stream) {
  if (dtype != L0CIM_F32 && dtype != L0CIM_F64)
    return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run_noalloc: dtype %d", int(dtype));
  if (!prm) return set_error(L0CIM_ERR_ARG, "mfcim_run_noalloc: cim params is NULL");
  if (prm->launch == L0CIM_LAUNCH_MATRIX)
    return set_error(L0CIM_ERR_UNSUPPORTED, "mfcim_run_noalloc: the matrix-core launch needs a workspace");
  if (n <= 0 || P <= 0) return set_error(L0CIM_ERR_SHAPE, "mfcim_run_noalloc: bad shape");
  const size_t need = mfcim_base_ws_bytes(dtype, n, P);
  if (need > kScratchBytes)
    return set_error(L0CIM_ERR_WORKSPACE,
                     "mfcim_run_noalloc: n = %d, P = %d needs %zu bytes of scratch, above its %zu bytes", n, P, need,
                     kScratchBytes);
  void* ws = nullptr;
  l0cim_status st = scratch_address(&ws);
  if (st != L0CIM_OK) return st;
  return mfcim_run_checked(dtype, n, P, j_dtype, J, ldj, row_scale, z, eta, prm, c, e, sigma, H, trace,
                           trace_steps, status, ws, need, /*allow_matrix=*/false, static_cast<hipStream_t>(stream));
}

}  // extern "C"
