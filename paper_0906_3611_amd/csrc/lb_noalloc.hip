// lb_get_fields_noalloc: lb_get_fields without any device allocation.
//
// lb_get_fields stages the six FP64 fields of a lattice (rho_A, rho_B, u',
// u_phys) in a temporary device buffer that it allocates and frees on every
// call.  This variant stages them in a file-scope device array of fixed
// size instead, for callers that cannot allocate (code under stream capture,
// tight serving loops, harnesses that forbid allocation).  Each GPU the
// library runs on holds its own copy of the array until the process ends;
// every call on one GPU uses that GPU's copy, so calls that overlap in time
// on one GPU (handles on different streams or threads) race and must be
// serialized by the caller.  The observe kernel writes every entry of the
// fields it stages, so nothing needs clearing between calls.
#include "lb.h"
#include "lb_engine.h"

#include <mutex>

namespace {

// Largest lattice the static staging holds: 2^20 sites (e.g. 1024 x 1024),
// six FP64 fields per site, 48 MiB per GPU.
constexpr size_t kMaxSites = size_t(1) << 20;
constexpr size_t kScratchDoubles = 6 * kMaxSites;

__device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on each GPU, looked up once per device with
// that device current.  The array's name in host code is only a host-side
// stand-in for the symbol, never a device address, so it is used nowhere
// but in the lookup.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

int scratch_ptr(int device, double** out, std::string* why) {
  if (device < 0 || device >= kMaxDevices) {
    *why = "device index beyond the static staging table";
    return LB_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *why = std::string("hipGetSymbolAddress of the static staging: ") + hipGetErrorString(e);
      return LB_E_DEVICE;
    }
    g_ptr[device] = (double*)p;
  }
  *out = g_ptr[device];
  return LB_OK;
}

}  // namespace

extern "C" int lb_get_fields_noalloc(lb_lattice* L, double* rho_a, double* rho_b, double* u,
                                     double* u_phys) {
  if (!L) return LB_E_INVAL;
  lbe::Engine& E = L->e;
  if (E.m.empty()) return E.fail(LB_E_STATE, "no lattice");
  const size_t n = (size_t)E.m[0].p.nx * (size_t)E.m[0].p.ny;
  if (n > kMaxSites)
    return E.fail(LB_E_INVAL, "lattice larger than the static field staging (2^20 sites); "
                              "use lb_get_fields");
  lbe::DeviceGuard dg(E.device);  // the lattice's device is current for the lookup
  double* staging = nullptr;
  std::string why;
  const int rc = scratch_ptr(E.device, &staging, &why);
  if (rc != LB_OK) return E.fail(rc, why);
  return lbe::engine_fields_staged(E, 0, staging, rho_a, rho_b, u, u_phys);
}
