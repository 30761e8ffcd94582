// Runtime behind the C ABI of include/lb.h: parameter validation, device
// workspace, ping-pong bookkeeping, transfers and fixed-order reductions.
#include "lb.h"
#include "lb_internal.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

struct lb_lattice {
  lb_params p{};
  lbk::Geometry g{};
  lbk::Coefs c{};
  hipStream_t stream = nullptr;
  int device = 0;
  bool fp64 = true, walls = false;
  size_t elem = 8;
  char* base = nullptr;
  bool owns = false;
  size_t bytes = 0, pop_bytes = 0;
  void* buf[2] = {nullptr, nullptr};
  void* wall[2] = {nullptr, nullptr};
  double* wave_red = nullptr;
  double* wave_wall = nullptr;
  double* red_out = nullptr;
  int* flag = nullptr;
  int64_t step = 0, avg_start = 0;
  lbk::StepVariant variant{1, 0};
  bool initialized = false;
  std::string err;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t buf, wall, wave_red, wave_wall, red_out, flag, total, pop_bytes;
};

// Weights of the interaction lattice (Table I): w on the first belt,
// p on both belts, by class |c|^2 = 1, 2, 4, 5, 8.
constexpr double kW1 = 1.0 / 9.0, kW2 = 1.0 / 36.0;
constexpr double kP1 = 4.0 / 63.0, kP2 = 4.0 / 135.0, kP4 = 1.0 / 180.0, kP5 = 2.0 / 945.0,
                 kP8 = 1.0 / 15120.0;

bool is_finite(double v) { return std::isfinite(v); }

int validate(const lb_params* p, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return LB_E_INVAL;
  };
  if (!p) return bad("params is NULL");
  if (p->nx < 5 || p->ny < 5) return bad("nx and ny must be >= 5");
  if ((long long)p->nx * p->ny > (1LL << 30)) return bad("lattice larger than 2^30 sites");
  if (p->boundary != LB_PERIODIC && p->boundary != LB_COUETTE_Y) return bad("unknown boundary");
  if (p->precision != LB_FP64 && p->precision != LB_FP32_DEV) return bad("unknown precision");
  for (int s = 0; s < 2; ++s) {
    if (!is_finite(p->tau[s]) || !(p->tau[s] > 0.5)) return bad("tau must be > 1/2");
    if (!is_finite(p->G_a[s]) || !is_finite(p->G_r[s])) return bad("couplings must be finite");
    if (!is_finite(p->rho_ref[s])) return bad("rho_ref must be finite");
  }
  if (!is_finite(p->rho0) || !(p->rho0 > 0)) return bad("rho0 must be > 0");
  if (!is_finite(p->G_AB)) return bad("G_AB must be finite");
  if (!is_finite(p->u_wall)) return bad("u_wall must be finite");
  return LB_OK;
}

lbk::Geometry make_geometry(const lb_params* p) {
  lbk::Geometry g{};
  g.nx = p->nx;
  g.ny = p->ny;
  g.pitch = (p->nx + lbk::kWave - 1) / lbk::kWave * lbk::kWave;  // strips start on a line
  g.row_elems = (long long)(g.pitch / lbk::kWave) * 18 * lbk::kWave;
  g.nstrips = (p->nx + lbk::kWave - 1) / lbk::kWave;
  // Aim for about 2048 wavefronts (8 per CU) with segments of 8..64 rows:
  // fewer, taller segments re-read fewer ring rows, more keep HBM busy.
  int nsegs = (2048 + g.nstrips - 1) / g.nstrips;
  nsegs = std::min(nsegs, std::max(1, p->ny / 8));
  nsegs = std::max(nsegs, (p->ny + 63) / 64);
  if (const char* e = std::getenv("LBSOFT_SEG_H")) {
    const int h = std::atoi(e);
    if (h >= 1) nsegs = (p->ny + h - 1) / h;
  }
  nsegs = std::max(1, std::min(nsegs, p->ny));
  g.nsegs = nsegs;
  g.seg_h = (p->ny + nsegs - 1) / nsegs;
  g.ntiles = g.nstrips * g.nsegs;
  g.tiles_per_xcd = (g.ntiles + 7) / 8;
  return g;
}

Layout make_layout(const lb_params* p, const lbk::Geometry& g) {
  const size_t elem = p->precision == LB_FP64 ? 8 : 4;
  Layout L{};
  L.pop_bytes = align_up((size_t)g.row_elems * (size_t)g.ny * elem);
  size_t off = 0;
  L.buf = off;
  off += 2 * L.pop_bytes;
  L.wall = off;
  off += 2 * align_up(12ull * (size_t)g.nx * elem);
  L.wave_red = off;
  off += align_up((size_t)g.ntiles * lbk::kNRed * sizeof(double));
  L.wave_wall = off;
  off += align_up((size_t)g.ntiles * 2 * sizeof(double));
  L.red_out = off;
  off += align_up(16 * sizeof(double));
  L.flag = off;
  off += kAlign;
  L.total = off;
  return L;
}

// Derived reference values and FP32 copies of the constants for the FP32
// kernels.  rho_ref is first rounded to FP32 so both precisions of the
// kernels see the same reference.
void round_coefs(lbk::Coefs& c) {
  for (int s = 0; s < 2; ++s) {
    c.rho_ref[s] = (double)(float)c.rho_ref[s];
    c.psi_ref[s] = c.rho0 * -std::expm1(-c.rho_ref[s] / c.rho0);
    c.psi_scale[s] = c.rho0 * std::exp(-c.rho_ref[s] / c.rho0);
    c.f_psi_ref[s] = (float)c.psi_ref[s];
    c.f_psi_scale[s] = (float)c.psi_scale[s];
  }
  for (int s = 0; s < 2; ++s) {
    for (int m = 0; m < 5; ++m) c.f_kself[s][m] = (float)c.kself[s][m];
    c.f_tau[s] = (float)c.tau[s];
    c.f_omega[s] = (float)c.omega[s];
    c.f_rho_ref[s] = (float)c.rho_ref[s];
  }
  c.f_kcross[0] = (float)c.kcross[0];
  c.f_kcross[1] = (float)c.kcross[1];
  c.f_rho0 = (float)c.rho0;
  c.f_inv_rho0 = (float)c.inv_rho0;
  c.f_u_wall = (float)c.u_wall;
}

lbk::Coefs make_coefs(const lb_params* p) {
  lbk::Coefs c{};
  for (int s = 0; s < 2; ++s) {
    c.kself[s][0] = p->G_a[s] * kW1 + p->G_r[s] * kP1;
    c.kself[s][1] = p->G_a[s] * kW2 + p->G_r[s] * kP2;
    c.kself[s][2] = p->G_r[s] * kP4;
    c.kself[s][3] = p->G_r[s] * kP5;
    c.kself[s][4] = p->G_r[s] * kP8;
    c.tau[s] = p->tau[s];
    c.omega[s] = 1.0 / p->tau[s];
    c.rho_ref[s] = p->rho_ref[s];
  }
  const double g = p->G_AB / (p->rho0 * p->rho0);
  c.kcross[0] = g * kW1;
  c.kcross[1] = g * kW2;
  c.rho0 = p->rho0;
  c.inv_rho0 = 1.0 / p->rho0;
  c.u_wall = p->u_wall;
  round_coefs(c);
  return c;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

int fail(lb_lattice* L, int code, const std::string& msg) {
  if (L) L->err = msg;
  return code;
}

#define HIPCK(L, expr)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail((L), LB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

// Temporary device array freed at scope exit.
struct DevTmp {
  void* p = nullptr;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
};

lbk::StepArgs base_args(const lb_lattice* L, int parity) {
  lbk::StepArgs a{};
  a.src = L->buf[parity];
  a.dst = L->buf[parity ^ 1];
  a.wall_in = L->wall[parity];
  a.wall_out = L->wall[parity ^ 1];
  a.wave_red = L->wave_red;
  a.wave_wall = L->wave_wall;
  a.flag = L->flag;
  a.g = L->g;
  a.c = L->c;
  return a;
}

int check_flag(lb_lattice* L, int* flag_out) {
  int f = 0;
  HIPCK(L, hipMemcpyAsync(&f, L->flag, sizeof(int), hipMemcpyDeviceToHost, L->stream));
  HIPCK(L, hipStreamSynchronize(L->stream));
  if (flag_out) *flag_out = f;
  if (f & 1) return fail(L, LB_E_UNSTABLE, "non-finite or non-positive density on the device");
  return LB_OK;
}

// Observe the current state: per-tile partials, and optionally fields / pops.
int observe(lb_lattice* L, double* fields, double* pops) {
  lbk::StepArgs a = base_args(L, (int)(L->step & 1));
  a.fields = fields;
  a.pops = pops;
  HIPCK(L, lbk::launch_observe(a, L->fp64, L->walls, L->stream));
  return LB_OK;
}

int set_rho_ref_from(lb_lattice* L, const double* ra, const double* rb, size_t n) {
  if (L->fp64) return LB_OK;
  const double* r[2] = {ra, rb};
  for (int s = 0; s < 2; ++s) {
    if (L->p.rho_ref[s] > 0) {
      L->c.rho_ref[s] = L->p.rho_ref[s];
      continue;
    }
    double acc = 0;
    for (size_t k = 0; k < n; ++k) acc += r[s][k];
    L->c.rho_ref[s] = acc / (double)n;
  }
  round_coefs(L->c);
  return LB_OK;
}

int reset_counters(lb_lattice* L, int64_t step) {
  HIPCK(L, hipMemsetAsync(L->wave_wall, 0, (size_t)L->g.ntiles * 2 * sizeof(double), L->stream));
  HIPCK(L, hipMemsetAsync(L->flag, 0, sizeof(int), L->stream));
  L->step = step;
  L->avg_start = step;
  return LB_OK;
}

}  // namespace

extern "C" {

int lb_abi_version(void) { return LB_ABI_VERSION; }

const char* lb_strerror(int status) {
  switch (status) {
    case LB_OK: return "ok";
    case LB_E_INVAL: return "invalid argument";
    case LB_E_NOMEM: return "out of device memory or workspace too small";
    case LB_E_DEVICE: return "HIP runtime error";
    case LB_E_UNSTABLE: return "numerical instability (non-finite or non-positive density)";
    case LB_E_STATE: return "call out of order";
    default: return "unknown status";
  }
}

const char* lb_last_error(const lb_lattice* L) { return L ? L->err.c_str() : "null handle"; }

int lb_workspace_bytes(const lb_params* p, size_t* out) {
  if (!out) return LB_E_INVAL;
  const int v = validate(p, nullptr);
  if (v != LB_OK) return v;
  const lbk::Geometry g = make_geometry(p);
  *out = make_layout(p, g).total;
  return LB_OK;
}

int lb_create(const lb_params* p, void* hip_stream, lb_lattice** out) {
  if (!out) return LB_E_INVAL;
  *out = nullptr;
  std::string why;
  const int v = validate(p, &why);
  if (v != LB_OK) return v;
  lb_lattice* L = new (std::nothrow) lb_lattice();
  if (!L) return LB_E_NOMEM;
  L->p = *p;
  L->g = make_geometry(p);
  L->c = make_coefs(p);
  L->fp64 = p->precision == LB_FP64;
  L->walls = p->boundary == LB_COUETTE_Y;
  L->elem = L->fp64 ? 8 : 4;
  L->stream = (hipStream_t)hip_stream;
  // Defaults: prefetch for FP32 (registers allow it), streaming stores when
  // the two population buffers exceed the 256 MB Infinity Cache.
  L->variant.prefetch = L->fp64 ? 0 : 1;
  L->variant.stream_stores = 0;
  if (hipGetDevice(&L->device) != hipSuccess) {
    delete L;
    return LB_E_DEVICE;
  }
  const Layout lay = make_layout(p, L->g);
  L->bytes = lay.total;
  L->pop_bytes = lay.pop_bytes;
  L->variant.stream_stores = 2 * lay.pop_bytes > (256ull << 20) ? 1 : 0;
  if (const char* e = std::getenv("LBSOFT_PREFETCH")) L->variant.prefetch = std::atoi(e) ? 1 : 0;
  if (const char* e = std::getenv("LBSOFT_STREAM_STORES")) L->variant.stream_stores = std::atoi(e) ? 1 : 0;
  if (p->device_buffer) {
    if (p->device_bytes < lay.total || ((uintptr_t)p->device_buffer % kAlign) != 0) {
      delete L;
      return LB_E_NOMEM;
    }
    L->base = (char*)p->device_buffer;
    L->owns = false;
  } else {
    void* b = nullptr;
    if (hipMalloc(&b, lay.total) != hipSuccess) {
      (void)hipGetLastError();
      delete L;
      return LB_E_NOMEM;
    }
    L->base = (char*)b;
    L->owns = true;
  }
  L->buf[0] = L->base + lay.buf;
  L->buf[1] = L->base + lay.buf + lay.pop_bytes;
  const size_t wall_bytes = align_up(12ull * (size_t)L->g.nx * L->elem);
  L->wall[0] = L->base + lay.wall;
  L->wall[1] = L->base + lay.wall + wall_bytes;
  L->wave_red = (double*)(L->base + lay.wave_red);
  L->wave_wall = (double*)(L->base + lay.wave_wall);
  L->red_out = (double*)(L->base + lay.red_out);
  L->flag = (int*)(L->base + lay.flag);
  if (hipMemsetAsync(L->base, 0, lay.total, L->stream) != hipSuccess ||
      hipStreamSynchronize(L->stream) != hipSuccess) {
    if (L->owns) (void)hipFree(L->base);
    delete L;
    return LB_E_DEVICE;
  }
  *out = L;
  return LB_OK;
}

void lb_destroy(lb_lattice* L) {
  if (!L) return;
  {
    DeviceGuard dg(L->device);
    (void)hipStreamSynchronize(L->stream);
    if (L->owns && L->base) (void)hipFree(L->base);
  }
  delete L;
}

static int init_from_device_rho(lb_lattice* L, const double* d_rho, const double* d_u) {
  HIPCK(L, lbk::launch_init(L->g, L->c, L->fp64, L->walls, d_rho, d_u, L->buf[0], L->wall[0],
                            L->stream));
  const int rc = reset_counters(L, 0);
  if (rc != LB_OK) return rc;
  HIPCK(L, hipStreamSynchronize(L->stream));
  L->initialized = true;
  return LB_OK;
}

int lb_init(lb_lattice* L, const double* rho_a, const double* rho_b, const double* ux,
            const double* uy) {
  if (!L) return LB_E_INVAL;
  if (!rho_a || !rho_b) return fail(L, LB_E_INVAL, "rho_a and rho_b are required");
  if ((ux == nullptr) != (uy == nullptr)) return fail(L, LB_E_INVAL, "give both ux and uy or neither");
  const size_t n = (size_t)L->g.nx * L->g.ny;
  for (size_t k = 0; k < n; ++k) {
    if (!is_finite(rho_a[k]) || !(rho_a[k] > 0) || !is_finite(rho_b[k]) || !(rho_b[k] > 0))
      return fail(L, LB_E_INVAL, "densities must be finite and > 0");
    if (ux && (!is_finite(ux[k]) || !is_finite(uy[k]))) return fail(L, LB_E_INVAL, "velocities must be finite");
  }
  DeviceGuard dg(L->device);
  set_rho_ref_from(L, rho_a, rho_b, n);
  DevTmp t;
  const size_t nb = n * sizeof(double);
  HIPCK(L, hipMalloc(&t.p, (ux ? 4 : 2) * nb));
  double* d = (double*)t.p;
  HIPCK(L, hipMemcpyAsync(d, rho_a, nb, hipMemcpyHostToDevice, L->stream));
  HIPCK(L, hipMemcpyAsync(d + n, rho_b, nb, hipMemcpyHostToDevice, L->stream));
  if (ux) {
    HIPCK(L, hipMemcpyAsync(d + 2 * n, ux, nb, hipMemcpyHostToDevice, L->stream));
    HIPCK(L, hipMemcpyAsync(d + 3 * n, uy, nb, hipMemcpyHostToDevice, L->stream));
  }
  return init_from_device_rho(L, d, ux ? d + 2 * n : nullptr);
}

int lb_init_noise(lb_lattice* L, uint64_t seed, double mean_a, double mean_b, double amp) {
  if (!L) return LB_E_INVAL;
  if (!is_finite(mean_a) || !is_finite(mean_b) || !is_finite(amp) || !(std::fabs(amp) < std::min(mean_a, mean_b)))
    return fail(L, LB_E_INVAL, "need |amp| < min(mean_a, mean_b) and finite values");
  DeviceGuard dg(L->device);
  if (!L->fp64) {
    L->c.rho_ref[0] = L->p.rho_ref[0] > 0 ? L->p.rho_ref[0] : mean_a;
    L->c.rho_ref[1] = L->p.rho_ref[1] > 0 ? L->p.rho_ref[1] : mean_b;
    round_coefs(L->c);
  }
  const size_t n = (size_t)L->g.nx * L->g.ny;
  DevTmp t;
  HIPCK(L, hipMalloc(&t.p, 2 * n * sizeof(double)));
  HIPCK(L, lbk::launch_noise(L->g.nx, L->g.ny, seed, mean_a, mean_b, amp, (double*)t.p, L->stream));
  return init_from_device_rho(L, (const double*)t.p, nullptr);
}

int lb_step(lb_lattice* L, int64_t n) {
  if (!L) return LB_E_INVAL;
  if (n < 0) return fail(L, LB_E_INVAL, "n must be >= 0");
  if (!L->initialized) return fail(L, LB_E_STATE, "lb_step before lb_init");
  DeviceGuard dg(L->device);
  for (int64_t k = 0; k < n; ++k) {
    lbk::StepArgs a = base_args(L, (int)(L->step & 1));
    a.accumulate_wall = L->walls ? 1 : 0;
    HIPCK(L, lbk::launch_step(a, L->fp64, L->walls, L->variant, L->stream));
    ++L->step;
  }
  return LB_OK;
}

int lb_observables(lb_lattice* L, lb_obs* out) {
  if (!L || !out) return LB_E_INVAL;
  if (!L->initialized) return fail(L, LB_E_STATE, "lb_observables before lb_init");
  DeviceGuard dg(L->device);
  int rc = observe(L, nullptr, nullptr);
  if (rc != LB_OK) return rc;
  HIPCK(L, lbk::launch_reduce_tiles(L->wave_red, L->g.ntiles, lbk::kNRed, L->red_out, L->stream));
  HIPCK(L, lbk::launch_reduce_tiles(L->wave_wall, L->g.ntiles, 2, L->red_out + lbk::kNRed, L->stream));
  double h[lbk::kNRed + 2];
  HIPCK(L, hipMemcpyAsync(h, L->red_out, sizeof(h), hipMemcpyDeviceToHost, L->stream));
  int flag = 0;
  rc = check_flag(L, &flag);
  std::memset(out, 0, sizeof(*out));
  out->step = L->step;
  out->mass[0] = h[0];
  out->mass[1] = h[1];
  out->mom[0] = h[2];
  out->mom[1] = h[3];
  out->mom_phys[0] = h[4];
  out->mom_phys[1] = h[5];
  out->pxy_kin = h[6];
  out->avg_count = L->step - L->avg_start;
  if (out->avg_count > 0 && L->walls) {
    out->wall_stress[0] = h[lbk::kNRed + 0] / (double)out->avg_count / (double)L->g.nx;
    out->wall_stress[1] = h[lbk::kNRed + 1] / (double)out->avg_count / (double)L->g.nx;
  }
  out->flags = flag;
  return rc;
}

int lb_get_fields(lb_lattice* L, double* rho_a, double* rho_b, double* u, double* u_phys) {
  if (!L) return LB_E_INVAL;
  if (!L->initialized) return fail(L, LB_E_STATE, "lb_get_fields before lb_init");
  DeviceGuard dg(L->device);
  const size_t n = (size_t)L->g.nx * L->g.ny, nb = n * sizeof(double);
  DevTmp t;
  HIPCK(L, hipMalloc(&t.p, 6 * nb));
  double* d = (double*)t.p;
  int rc = observe(L, d, nullptr);
  if (rc != LB_OK) return rc;
  if (rho_a) HIPCK(L, hipMemcpyAsync(rho_a, d, nb, hipMemcpyDeviceToHost, L->stream));
  if (rho_b) HIPCK(L, hipMemcpyAsync(rho_b, d + n, nb, hipMemcpyDeviceToHost, L->stream));
  if (u) HIPCK(L, hipMemcpyAsync(u, d + 2 * n, 2 * nb, hipMemcpyDeviceToHost, L->stream));
  if (u_phys) HIPCK(L, hipMemcpyAsync(u_phys, d + 4 * n, 2 * nb, hipMemcpyDeviceToHost, L->stream));
  return check_flag(L, nullptr);
}

int lb_get_populations(lb_lattice* L, double* f) {
  if (!L || !f) return LB_E_INVAL;
  if (!L->initialized) return fail(L, LB_E_STATE, "lb_get_populations before lb_init");
  DeviceGuard dg(L->device);
  const size_t n = (size_t)L->g.nx * L->g.ny, nb = 18 * n * sizeof(double);
  DevTmp t;
  HIPCK(L, hipMalloc(&t.p, nb));
  int rc = observe(L, nullptr, (double*)t.p);
  if (rc != LB_OK) return rc;
  HIPCK(L, hipMemcpyAsync(f, t.p, nb, hipMemcpyDeviceToHost, L->stream));
  return check_flag(L, nullptr);
}

int lb_set_populations(lb_lattice* L, const double* f, int64_t step) {
  if (!L || !f) return LB_E_INVAL;
  if (step < 0) return fail(L, LB_E_INVAL, "step must be >= 0");
  const size_t n = (size_t)L->g.nx * L->g.ny;
  for (size_t k = 0; k < 18 * n; ++k)
    if (!is_finite(f[k])) return fail(L, LB_E_INVAL, "populations must be finite");
  DeviceGuard dg(L->device);
  if (!L->fp64 && !L->initialized) {
    // reference densities from these populations when none were given
    std::vector<double> ra(n, 0.0), rb(n, 0.0);
    for (int i = 0; i < 9; ++i)
      for (size_t k = 0; k < n; ++k) {
        ra[k] += f[(size_t)i * n + k];
        rb[k] += f[(size_t)(9 + i) * n + k];
      }
    set_rho_ref_from(L, ra.data(), rb.data(), n);
  }
  DevTmp t;
  HIPCK(L, hipMalloc(&t.p, 18 * n * sizeof(double)));
  HIPCK(L, hipMemcpyAsync(t.p, f, 18 * n * sizeof(double), hipMemcpyHostToDevice, L->stream));
  const int par = (int)(step & 1);
  HIPCK(L, lbk::launch_set_pops(L->g, L->c, L->fp64, L->walls, (const double*)t.p, L->buf[par],
                                L->wall[par], L->stream));
  const int rc = reset_counters(L, step);
  if (rc != LB_OK) return rc;
  HIPCK(L, hipStreamSynchronize(L->stream));
  L->initialized = true;
  return LB_OK;
}

int lb_reset_averages(lb_lattice* L) {
  if (!L) return LB_E_INVAL;
  DeviceGuard dg(L->device);
  HIPCK(L, hipMemsetAsync(L->wave_wall, 0, (size_t)L->g.ntiles * 2 * sizeof(double), L->stream));
  L->avg_start = L->step;
  return LB_OK;
}

int lb_sync(lb_lattice* L) {
  if (!L) return LB_E_INVAL;
  DeviceGuard dg(L->device);
  return check_flag(L, nullptr);
}

int64_t lb_current_step(const lb_lattice* L) { return L ? L->step : -1; }

int lb_get_launch_info(const lb_lattice* L, lb_launch_info* out) {
  if (!L || !out) return LB_E_INVAL;
  out->nstrips = L->g.nstrips;
  out->nsegs = L->g.nsegs;
  out->ntiles = L->g.ntiles;
  out->grid_blocks = 8 * L->g.tiles_per_xcd;
  out->block_threads = lbk::kWave;
  out->pitch = L->g.pitch;
  out->workspace_bytes = L->bytes;
  out->population_bytes = L->pop_bytes;
  return LB_OK;
}

}  // extern "C"
