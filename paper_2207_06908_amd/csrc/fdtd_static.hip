// fdtd_static.hip -- fdtd_bind_static: a grid's workspace in a static device
// array, for callers that cannot allocate device memory.
//
// The array below exists once on every GPU the library runs on and stays
// there until the process ends.  Host code never passes its name to a
// kernel or a copy: in host code the name is a stand-in, not the device
// address.  The device address comes from hipGetSymbolAddress, looked up
// once per device with that device current, and is then handed to the
// ordinary binding path, which places the fields, tables and probe records
// in it, zeroes every field, CPML and wire state and every probe record, and
// uploads the tables -- so nothing a previous context left there survives.
// One context per device can hold the array at a time; a second binding on
// that device is refused until the first context is destroyed.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/fdtd.h"
#include "fdtd_dev.h"

static __device__ __align__(256) unsigned char scratch[FDTD_STATIC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};            // device address of scratch, per device
const fdtd_ctx* g_owner[kMaxDevices] = {}; // context bound to it, per device

}  // namespace

void fdtd_static_release(const fdtd_ctx* c) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (int d = 0; d < kMaxDevices; ++d)
    if (g_owner[d] == c) g_owner[d] = nullptr;
}

extern "C" int fdtd_bind_static(fdtd_ctx* c) {
  if (!c) return FDTD_EINVAL;
  int rc = fdtd_finalize(c);
  if (rc) return rc;
  const size_t need = fdtd_workspace_bytes(c);
  if (need == 0) return FDTD_EINVAL;
  if (need > FDTD_STATIC_BYTES)
    return fdtd_fail_code(c, FDTD_ENOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the " +
                                              std::to_string((size_t)FDTD_STATIC_BYTES) + "-byte static array");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fdtd_fail_code(c, FDTD_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fdtd_fail_code(c, FDTD_EDEVICE, "device index beyond 63");
  void* addr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_owner[dev] && g_owner[dev] != c)
      return fdtd_fail_code(c, FDTD_ESTATE, "the static workspace of this device is bound to another live context");
    if (!g_addr[dev]) {
      e = hipGetSymbolAddress(&g_addr[dev], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        g_addr[dev] = nullptr;
        return fdtd_fail_code(c, FDTD_EDEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
      }
    }
    addr = g_addr[dev];
    g_owner[dev] = c;
  }
  rc = fdtd_bind_workspace(c, addr, FDTD_STATIC_BYTES);
  if (rc) fdtd_static_release(c);
  return rc;
}
