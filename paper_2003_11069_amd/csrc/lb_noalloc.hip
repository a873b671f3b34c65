// lb_noalloc.hip -- lb_get_fields_static: the fields of the current state
// without any device allocation (declaration in include/lbnci.h).
//
// lb_get_fields stages the FIELDS pass's FP64 output (rho1, rho2, u) in device
// buffers it allocates and frees per call.  This variant stages it in one
// file-scope device array instead.  Each device the library runs on holds its
// own copy of the array for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (the array's name is a host-side stand-in, not a device address).
#include "lb_internal.hpp"

#include <hip/hip_runtime.h>
#include <mutex>

using namespace lbk;
using namespace lbi;

namespace {

constexpr size_t SCRATCH_DOUBLES = (size_t)LB_STATIC_SCRATCH_BYTES / sizeof(double);
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_ptr[MAX_DEVICES] = {};  // device address of `scratch`, per device

// The device address of this device's scratch array, looked up once per
// device with that device current.
int scratch_ptr(int dev, double **out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LB_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LB_EDEVICE, "hipGetSymbolAddress returned NULL");
    g_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_ptr[dev];
  return LB_OK;
}

}  // namespace

extern "C" {

int lb_get_fields_static(lb_handle *h, double *rho1, double *rho2, double *u) {
  if (!h || !rho1 || !rho2 || !u) return fail(LB_EINVAL, "NULL argument");
  if (!h->initialised) return fail(LB_ESTATE, "lb_get_fields_static before initialisation");
  const size_t N = (size_t)h->N;
  const size_t need = (size_t)(2 + h->D) * N;
  if (need > SCRATCH_DOUBLES)
    return fail(LB_EINVAL, "fields of %zu nodes need %zu bytes; the static scratch holds %zu", N,
                need * sizeof(double), (size_t)LB_STATIC_SCRATCH_BYTES);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != h->device)
    return fail(LB_EINVAL, "the handle lives on device %d; make it current (device %d is)", h->device, dev);
  double *s = nullptr;
  int rc = scratch_ptr(dev, &s);
  if (rc) return rc;
  // the FIELDS pass leaves wall and solid nodes untouched: clear the region
  // (a fill kernel, not a memset node, in case the caller captures the stream)
  const int words = (int)(2 * need);
  hipLaunchKernelGGL(k_fill_u32, dim3((words + 255) / 256), dim3(256), 0, h->stream,
                     reinterpret_cast<uint32_t *>(s), words, 0u);
  HIP_TRY(hipGetLastError());
  rc = dispatch(h, FIELDS, s, s + N, s + 2 * N, nullptr);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(rho1, s, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(rho2, s + N, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(u, s + 2 * N, (size_t)h->D * N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LB_OK;
}

}  // extern "C"
