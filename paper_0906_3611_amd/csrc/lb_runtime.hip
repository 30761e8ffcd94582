// C ABI of single lattices (lb_*) and batches (lb_batch_*) over the engine
// of lb_engine.hip: a lattice is an engine of one, a batch an engine of n.
#include "lb.h"
#include "lb_engine.h"

#include <cmath>
#include <new>
#include <string>

using lbe::DeviceGuard;
using lbe::Engine;

namespace {

int validate_set(const lb_params* ps, int n) {
  if (!ps || n <= 0) return LB_E_INVAL;
  for (int i = 0; i < n; ++i) {
    const int v = lbe::validate(&ps[i], nullptr);
    if (v != LB_OK) return v;
    if (ps[i].precision != ps[0].precision || ps[i].boundary != ps[0].boundary) return LB_E_INVAL;
  }
  return LB_OK;
}

}  // namespace

extern "C" {

int lb_abi_version(void) { return LB_ABI_VERSION; }

int lb_kolmogorov_force(double u0, int32_t ny, double tau, double* g) {
  if (!g || ny < 5 || !std::isfinite(tau) || !(tau > 0.5) || !std::isfinite(u0)) return LB_E_INVAL;
  const double k = 2.0 * M_PI / (double)ny;
  *g = (tau - 0.5) / 3.0 * k * k * u0;
  return LB_OK;
}

const char* lb_strerror(int status) {
  switch (status) {
    case LB_OK: return "ok";
    case LB_E_INVAL: return "invalid argument";
    case LB_E_NOMEM: return "out of device memory, workspace too small, or not admitted";
    case LB_E_DEVICE: return "HIP runtime error";
    case LB_E_UNSTABLE: return "numerical instability (non-finite or non-positive density)";
    case LB_E_STATE: return "call out of order";
    default: return "unknown status";
  }
}

const char* lb_last_error(const lb_lattice* L) { return lbe::handle_error(L ? &L->e.err : nullptr); }

int lb_workspace_bytes(const lb_params* p, size_t* out) {
  if (!out) return LB_E_INVAL;
  const int v = lbe::validate(p, nullptr);
  if (v != LB_OK) return v;
  *out = lbe::engine_static_bytes(p, 1);
  return LB_OK;
}

int lb_create(const lb_params* p, void* hip_stream, lb_lattice** out) {
  if (!out) return LB_E_INVAL;
  *out = nullptr;
  std::string why;
  const int v = lbe::validate(p, &why);
  lbe::create_error() = why;
  if (v != LB_OK) return v;
  lb_lattice* L = new (std::nothrow) lb_lattice();
  if (!L) return LB_E_NOMEM;
  const int rc = lbe::engine_create_static(L->e, p, 1, p->device_buffer, p->device_bytes,
                                           (hipStream_t)hip_stream);
  if (rc != LB_OK) {
    lbe::create_error() = L->e.err;
    lbe::engine_destroy(L->e);
    delete L;
    return rc;
  }
  *out = L;
  return LB_OK;
}

int lb_set_tune_cache(const char* path) { return lbe::set_tune_cache(path); }

void lb_destroy(lb_lattice* L) {
  if (!L) return;
  lbe::engine_destroy(L->e);
  delete L;
}

int lb_init(lb_lattice* L, const double* rho_a, const double* rho_b, const double* ux,
            const double* uy) {
  return L ? lbe::engine_init(L->e, 0, rho_a, rho_b, ux, uy) : LB_E_INVAL;
}

int lb_init_noise(lb_lattice* L, uint64_t seed, double mean_a, double mean_b, double amp) {
  return L ? lbe::engine_init_noise(L->e, 0, seed, mean_a, mean_b, amp) : LB_E_INVAL;
}

int lb_step(lb_lattice* L, int64_t n) { return L ? lbe::engine_step(L->e, n) : LB_E_INVAL; }

int lb_observables(lb_lattice* L, lb_obs* out) {
  return (L && out) ? lbe::engine_observables(L->e, out) : LB_E_INVAL;
}

int lb_get_fields(lb_lattice* L, double* rho_a, double* rho_b, double* u, double* u_phys) {
  return L ? lbe::engine_fields(L->e, 0, rho_a, rho_b, u, u_phys) : LB_E_INVAL;
}

int lb_get_populations(lb_lattice* L, double* f) {
  return (L && f) ? lbe::engine_pops(L->e, 0, f) : LB_E_INVAL;
}

int lb_set_populations(lb_lattice* L, const double* f, int64_t step) {
  return (L && f) ? lbe::engine_set_pops(L->e, 0, f, step) : LB_E_INVAL;
}

int lb_reset_averages(lb_lattice* L) { return L ? lbe::engine_reset_averages(L->e) : LB_E_INVAL; }

int lb_set_overlap_reference(lb_lattice* L) {
  return L ? lbe::engine_set_reference(L->e) : LB_E_INVAL;
}

int lb_sync(lb_lattice* L) { return L ? lbe::engine_sync(L->e) : LB_E_INVAL; }

int64_t lb_current_step(const lb_lattice* L) { return L ? lbe::member_time(L->e, 0) : -1; }

int lb_get_launch_info(const lb_lattice* L, lb_launch_info* out) {
  if (!L || !out) return LB_E_INVAL;
  lbe::engine_info(L->e, out);
  return LB_OK;
}

int lb_set_launch(lb_lattice* L, int32_t seg_h, int32_t prefetch, int32_t stream_stores,
                  int32_t use_graph, int32_t tiles_per_group) {
  if (!L) return LB_E_INVAL;
  DeviceGuard dg(L->e.device);
  const int rc = lbe::engine_set_variant(L->e, prefetch, stream_stores, use_graph, tiles_per_group);
  if (rc != LB_OK) return rc;
  return seg_h >= 0 ? lbe::engine_regrid(L->e, seg_h) : LB_OK;
}

int lb_autotune(lb_lattice* L, int32_t steps, lb_launch_info* out, double* us_per_step) {
  if (!L) return LB_E_INVAL;
  const int rc = lbe::engine_autotune(L->e, steps, us_per_step);
  if (rc == LB_OK && out) lbe::engine_info(L->e, out);
  return rc;
}

/* ------------------------------ batches ------------------------------ */

const char* lb_batch_last_error(const lb_batch* B) { return lbe::handle_error(B ? &B->e.err : nullptr); }

int lb_batch_workspace_bytes(const lb_params* p, int32_t n, size_t* out) {
  if (!out) return LB_E_INVAL;
  const int v = validate_set(p, n);
  if (v != LB_OK) return v;
  *out = lbe::engine_static_bytes(p, n);
  return LB_OK;
}

int lb_batch_create(const lb_params* p, int32_t n, void* device_buffer, size_t device_bytes,
                    void* hip_stream, lb_batch** out) {
  if (!out) return LB_E_INVAL;
  *out = nullptr;
  const int v = validate_set(p, n);
  lbe::create_error() = v != LB_OK ? "invalid parameters or count" : "";
  if (v != LB_OK) return v;
  lb_batch* B = new (std::nothrow) lb_batch();
  if (!B) return LB_E_NOMEM;
  const int rc = lbe::engine_create_static(B->e, p, n, device_buffer, device_bytes,
                                           (hipStream_t)hip_stream);
  if (rc != LB_OK) {
    lbe::create_error() = B->e.err;
    lbe::engine_destroy(B->e);
    delete B;
    return rc;
  }
  *out = B;
  return LB_OK;
}

void lb_batch_destroy(lb_batch* B) {
  if (!B) return;
  lbe::engine_destroy(B->e);
  delete B;
}

int32_t lb_batch_size(const lb_batch* B) { return B ? (int32_t)B->e.m.size() : -1; }

int lb_batch_init(lb_batch* B, int32_t i, const double* rho_a, const double* rho_b,
                  const double* ux, const double* uy) {
  return B ? lbe::engine_init(B->e, i, rho_a, rho_b, ux, uy) : LB_E_INVAL;
}

int lb_batch_init_noise(lb_batch* B, int32_t i, uint64_t seed, double mean_a, double mean_b,
                        double amp) {
  return B ? lbe::engine_init_noise(B->e, i, seed, mean_a, mean_b, amp) : LB_E_INVAL;
}

int lb_batch_step(lb_batch* B, int64_t n) { return B ? lbe::engine_step(B->e, n) : LB_E_INVAL; }

int lb_batch_observables(lb_batch* B, lb_obs* out) {
  return (B && out) ? lbe::engine_observables(B->e, out) : LB_E_INVAL;
}

int lb_batch_get_fields(lb_batch* B, int32_t i, double* rho_a, double* rho_b, double* u,
                        double* u_phys) {
  return B ? lbe::engine_fields(B->e, i, rho_a, rho_b, u, u_phys) : LB_E_INVAL;
}

int lb_batch_get_populations(lb_batch* B, int32_t i, double* f) {
  return B ? lbe::engine_pops(B->e, i, f) : LB_E_INVAL;
}

int lb_batch_sync(lb_batch* B) { return B ? lbe::engine_sync(B->e) : LB_E_INVAL; }

int lb_batch_get_launch_info(const lb_batch* B, lb_launch_info* out) {
  if (!B || !out) return LB_E_INVAL;
  lbe::engine_info(B->e, out);
  return LB_OK;
}

int lb_batch_set_launch(lb_batch* B, int32_t seg_h, int32_t prefetch, int32_t stream_stores,
                        int32_t use_graph, int32_t tiles_per_group) {
  if (!B) return LB_E_INVAL;
  DeviceGuard dg(B->e.device);
  const int rc = lbe::engine_set_variant(B->e, prefetch, stream_stores, use_graph, tiles_per_group);
  if (rc != LB_OK) return rc;
  return seg_h >= 0 ? lbe::engine_regrid(B->e, seg_h) : LB_OK;
}

int lb_batch_reset_averages(lb_batch* B) {
  return B ? lbe::engine_reset_averages(B->e) : LB_E_INVAL;
}

int lb_batch_set_overlap_reference(lb_batch* B) {
  return B ? lbe::engine_set_reference(B->e) : LB_E_INVAL;
}

int lb_batch_autotune(lb_batch* B, int32_t steps, lb_launch_info* out, double* us_per_step) {
  if (!B) return LB_E_INVAL;
  const int rc = lbe::engine_autotune(B->e, steps, us_per_step);
  if (rc == LB_OK && out) lbe::engine_info(B->e, out);
  return rc;
}

}  // extern "C"
