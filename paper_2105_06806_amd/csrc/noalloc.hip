// Allocation-free variant of the Lanczos ground state: the same driver and
// kernels as edx_lanczos_ground_state, with the workspace taken from a fixed
// per-device array instead of a caller buffer, for callers that cannot
// allocate device memory.
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds its own copy (kScratchBytes) from module load until the process ends.
// Host code never uses the symbol itself as an address (on the host it is a
// stand-in, not device memory); the device address of each GPU's copy comes
// from hipGetSymbolAddress, taken once per device with that device current,
// and only that pointer reaches kernels and memory calls.  The driver clears
// what must start at zero in the workspace itself, so nothing carries over
// from the previous call.  All calls on one GPU share its copy: calls that
// overlap on that GPU (other host threads or streams) race.
#include <mutex>
#include <string>

#include "edx_internal.h"

namespace edx {

constexpr size_t kScratchBytes = size_t(256) << 20;   // 256 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch`, looked up on first use
edx_status scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("lanczos_ground_state_static: device index out of range");
    return EDX_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return EDX_E_DEVICE;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return EDX_OK;
}

}  // namespace

edx_status lanczos_ground_state_static(const edx_sector* s, const edx_lanczos_opts* o,
                                       double* e0, void* psi0, edx_lanczos_report* rep,
                                       hipStream_t st) {
  int dev = -1;
  EDX_HIP(hipGetDevice(&dev));
  if (dev != s->device) {
    set_error("lanczos_ground_state_static: the sector's device must be the current device");
    return EDX_E_INVALID;
  }
  // the driver aligns the workspace start to 256 bytes; the array already is
  const size_t need = lanczos_workspace_bytes(s, o->vtype, o->niter, o->reorth);
  if (need > kScratchBytes) {
    set_error("lanczos_ground_state_static: this sector needs " + std::to_string(need) +
              " bytes of workspace, above the fixed " + std::to_string(kScratchBytes) +
              "-byte per-device scratch array (use edx_lanczos_ground_state with a workspace)");
    return EDX_E_NOMEM;
  }
  void* ws = nullptr;
  EDX_TRY(scratch_ptr(dev, &ws));
  return lanczos_ground_state_impl(s, o, ws, kScratchBytes, e0, psi0, rep, st);
}

}  // namespace edx
