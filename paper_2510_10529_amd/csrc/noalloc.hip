// loss_grad without a caller-supplied work buffer: its scratch (the loss partial sums and the
// Gram partials of the projection B <- (I - Psi Psi^T) B) lives in a fixed device array of this
// library, so the call allocates nothing. For callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace invdft {
namespace {

// 1025 doubles of loss partials + 1024 blocks x one 64 x 64 Gram tile + the nocc x 64 Gram block
// of one column group of B, each rounded to 256 bytes: 33,595,904 bytes at nocc = 64 and
// 33,694,208 at the largest nocc (256), on the largest mesh.
constexpr size_t kScratchBytes = 34u << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU, held from the library's load until the process ends. In host code this
// name is only a stand-in: kernels receive the address that hipGetSymbolAddress returns.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of the current device's copy, looked up once per device.
fe_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FE_EDEVICE, "loss_grad_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(FE_EDEVICE, "loss_grad_noalloc: no device address for the scratch array");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return FE_OK;
}

}  // namespace
}  // namespace invdft

using namespace invdft;

extern "C" size_t loss_grad_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" fe_status loss_grad_noalloc(fe_mesh mesh, const double* Psi, const double* occ_h, int nocc,
                                       const double* rho_data, const double* Q, double tau_bc, double* rho,
                                       double* B, double* grad, double* loss_h, void* stream) {
  const Mesh* m = mesh_tables(mesh);
  if (!m) return fail(FE_EINVAL, "mesh handle is NULL");
  if (!Psi || !occ_h) return fail(FE_EINVAL, "loss_grad_noalloc: Psi and occ_h are required");
  if (nocc < 1 || nocc > kMaxShiftCols) return fail(FE_EINVAL, "loss_grad_noalloc: nocc must be in [1, 256]");
  if (!Q && !rho) return fail(FE_EINVAL, "loss_grad_noalloc: phase 1 needs rho (no density buffer of its own)");
  const size_t need = loss_grad_scratch_bytes(m->nf, nocc);
  if (need > kScratchBytes)
    return fail(FE_EINVAL, "loss_grad_noalloc: the call needs " + std::to_string(need) +
                               " bytes of scratch, more than the fixed " + std::to_string(kScratchBytes));
  int dev = -1;
  INVDFT_HIP(hipGetDevice(&dev));
  if (dev != m->device) return fail(FE_EINVAL, "loss_grad_noalloc: the current device is not the mesh's device");
  void* p = nullptr;
  fe_status st = scratch_address(dev, &p);
  if (st != FE_OK) return st;
  return loss_grad_impl(*m, Psi, occ_h, nocc, rho_data, Q, tau_bc, rho, B, grad, loss_h, nullptr, p,
                        "loss_grad_noalloc", static_cast<hipStream_t>(stream));
}
