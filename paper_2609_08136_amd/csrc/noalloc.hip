// kernel_matvec for callers that cannot allocate device memory (code under graph
// capture, tight serving loops, harnesses that forbid hipMalloc): the scratch the
// product needs (centre, packed points, split V, column-split partial sums, the
// finiteness flag) lives in a file-scope device array instead of a caller-passed
// workspace.  Each GPU the library runs on holds its own copy of the array until the
// process ends.
#include <mutex>
#include <vector>

#include "nys_internal.h"
#include "../../include/nys_noalloc.h"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;   // 256 MiB per device

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // device address of `scratch`, per device ordinal

// The array's device address on the current device, looked up once per device.  In
// host code the name `scratch` is only a host-side stand-in: kernels must be given
// this address.
int32_t scratch_address(void **out) {
  int dev = 0;
  NYS_CHECK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    NYS_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
      nys::set_error("kernel_matvec_noalloc: no device address for the scratch array");
      return NYS_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NYS_OK;
}

}  // namespace

extern "C" {

size_t nys_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

int32_t kernel_matvec_noalloc(nys_kernel k, int32_t deriv, int32_t prec, const double *Xr, int64_t nr,
                              const double *Xc, int64_t nc, int32_t d, const void *V, int32_t m, void *Out,
                              double alpha, double beta, void *stream) {
  if (nr < 0 || nc < 0 || m < 0) {
    nys::set_error("kernel_matvec_noalloc: negative size");
    return NYS_EINVAL;
  }
  size_t need = 0;
  const int32_t rc = nys_workspace_bytes(NYS_OP_KERNEL_MATVEC, nr, nc, d, 0, m, prec, &need);
  if (rc != NYS_OK) return rc;
  if (need > NOALLOC_SCRATCH_BYTES) {
    nys::set_error("kernel_matvec_noalloc: this product needs " + std::to_string(need) +
                   " bytes of scratch, more than the fixed " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                   " (use kernel_matvec with a workspace)");
    return NYS_ENOMEM;
  }
  void *ptr = nullptr;
  NYS_RETURN_IF(scratch_address(&ptr));
  return kernel_matvec(k, deriv, prec, Xr, nr, Xc, nc, d, V, m, Out, alpha, beta, ptr, NOALLOC_SCRATCH_BYTES,
                       stream);
}

}  // extern "C"
