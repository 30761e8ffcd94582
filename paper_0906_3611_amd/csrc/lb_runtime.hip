// Runtime behind the C ABI of include/lb.h: parameter validation, device
// workspace, ping-pong bookkeeping, transfers, fixed-order reductions, and
// step launches for one lattice or for a batch of lattices.
//
// Both the single lattice (lb_lattice) and the batch (lb_batch) are an
// Engine: a set of lattices of one precision and boundary type that advance
// together, one kernel launch per time step over the tiles of all of them.
#include "lb.h"
#include "lb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Weights of the interaction lattice (Table I): w on the first belt,
// p on both belts, by class |c|^2 = 1, 2, 4, 5, 8.
constexpr double kW1 = 1.0 / 9.0, kW2 = 1.0 / 36.0;
constexpr double kP1 = 4.0 / 63.0, kP2 = 4.0 / 135.0, kP4 = 1.0 / 180.0, kP5 = 2.0 / 945.0,
                 kP8 = 1.0 / 15120.0;
constexpr size_t kInfinityCacheBytes = 256ull << 20;

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

// Tiles: 64-column strips x row segments.  Aim for about 2048 wavefronts
// (8 per CU) with segments of 8..64 rows: fewer, taller segments re-read
// fewer ring rows, more keep HBM busy.  seg_h > 0 forces the segment height.
lbk::Geometry make_geometry(const lb_params* p, int seg_h) {
  lbk::Geometry g{};
  g.nx = p->nx;
  g.ny = p->ny;
  g.pitch = (p->nx + lbk::kWave - 1) / lbk::kWave * lbk::kWave;  // strips start on a line
  g.row_elems = (long long)(g.pitch / lbk::kWave) * 18 * lbk::kWave;
  g.nstrips = (p->nx + lbk::kWave - 1) / lbk::kWave;
  int nsegs = (2048 + g.nstrips - 1) / g.nstrips;
  nsegs = std::min(nsegs, std::max(1, p->ny / 8));
  nsegs = std::max(nsegs, (p->ny + 63) / 64);
  if (seg_h <= 0) {
    if (const char* e = std::getenv("LBSOFT_SEG_H")) seg_h = std::atoi(e);
  }
  if (seg_h >= 1) nsegs = (p->ny + seg_h - 1) / seg_h;
  nsegs = std::max(1, std::min(nsegs, p->ny));
  g.nsegs = nsegs;
  g.seg_h = (p->ny + nsegs - 1) / nsegs;
  g.ntiles = g.nstrips * g.nsegs;
  return g;
}

// The most tiles any segment height >= 4 can give (sizes the per-tile slots).
int max_tiles(const lb_params* p) {
  const int nstrips = (p->nx + lbk::kWave - 1) / lbk::kWave;
  const int nsegs = std::max(1, std::min(p->ny, (p->ny + 3) / 4));
  return std::max(nstrips * nsegs, make_geometry(p, 0).ntiles);
}

size_t elem_size(const lb_params* p) { return p->precision == LB_FP64 ? 8 : 4; }
size_t pop_bytes_of(const lb_params* p, const lbk::Geometry& g) {
  return align_up((size_t)g.row_elems * (size_t)g.ny * elem_size(p));
}
size_t wall_bytes_of(const lb_params* p) { return align_up(12ull * (size_t)p->nx * elem_size(p)); }

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
    c.rho_ref[s] = p->rho_ref[s] > 0 ? p->rho_ref[s] : 1.0;
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

// Temporary device array freed at scope exit.
struct DevTmp {
  void* p = nullptr;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
};

// One lattice of an engine (host view; the pointers are device addresses).
struct Member {
  lb_params p{};
  lbk::LatticeDesc d{};
  size_t pop_bytes = 0, wall_bytes = 0;
  bool initialized = false;
  int64_t t_base = 0;      // member time at engine step e_base
  int64_t e_base = 0;
  int64_t avg_start = 0;   // engine step at which the wall averages restarted
};

// Lattices of one precision and boundary type advancing together.
struct Engine {
  std::vector<Member> m;
  bool fp64 = true, walls = false;
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  int device = 0;
  char* base = nullptr;
  bool owns = false;
  size_t bytes = 0;
  int slot_tiles = 0;  // per-tile slot capacity
  int ntiles = 0;
  lbk::LatticeDesc* d_descs = nullptr;
  int* d_tile_lattice = nullptr;
  double* wave_red = nullptr;
  double* wave_wall = nullptr;
  double* red_out = nullptr;  // [n][16]
  int* flags = nullptr;       // [n]
  int64_t step = 0;           // engine step count
  lbk::StepVariant variant{1, 0};
  bool use_graph = false;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // two-step graphs, by starting parity
  std::string err;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
};

#define HIPCK(E, expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return (E).fail(LB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct EngineLayout {
  size_t descs, tile_lattice, wave_red, wave_wall, red_out, flags, members, total;
  std::vector<size_t> member_off;
};

EngineLayout engine_layout(const std::vector<lb_params>& ps, const std::vector<lbk::Geometry>& gs,
                           int slot_tiles) {
  EngineLayout L{};
  const int n = (int)ps.size();
  size_t off = 0;
  L.descs = off;
  off += align_up((size_t)n * sizeof(lbk::LatticeDesc));
  L.tile_lattice = off;
  off += align_up((size_t)slot_tiles * sizeof(int));
  L.wave_red = off;
  off += align_up((size_t)slot_tiles * lbk::kNRed * sizeof(double));
  L.wave_wall = off;
  off += align_up((size_t)slot_tiles * 2 * sizeof(double));
  L.red_out = off;
  off += align_up((size_t)n * 16 * sizeof(double));
  L.flags = off;
  off += align_up((size_t)n * sizeof(int));
  L.members = off;
  for (int i = 0; i < n; ++i) {
    L.member_off.push_back(off);
    off += 2 * pop_bytes_of(&ps[i], gs[i]) + 2 * wall_bytes_of(&ps[i]);
  }
  L.total = off;
  return L;
}

int validate_set(const lb_params* ps, int n, std::string* why) {
  if (!ps || n <= 0) {
    if (why) *why = "need at least one lattice";
    return LB_E_INVAL;
  }
  for (int i = 0; i < n; ++i) {
    const int v = validate(&ps[i], why);
    if (v != LB_OK) return v;
    if (ps[i].precision != ps[0].precision || ps[i].boundary != ps[0].boundary) {
      if (why) *why = "all lattices of a batch must share precision and boundary type";
      return LB_E_INVAL;
    }
  }
  return LB_OK;
}

size_t engine_bytes(const lb_params* ps, int n) {
  std::vector<lb_params> v(ps, ps + n);
  std::vector<lbk::Geometry> gs;
  int slots = 0;
  for (int i = 0; i < n; ++i) {
    gs.push_back(make_geometry(&ps[i], 0));
    slots += max_tiles(&ps[i]);
  }
  return engine_layout(v, gs, slots).total;
}

int upload_descs(Engine& E) {
  std::vector<lbk::LatticeDesc> h;
  for (auto& mm : E.m) h.push_back(mm.d);
  HIPCK(E, hipMemcpyAsync(E.d_descs, h.data(), h.size() * sizeof(lbk::LatticeDesc),
                          hipMemcpyHostToDevice, E.stream));
  // the host vector dies at return: make the copy complete first
  HIPCK(E, hipStreamSynchronize(E.stream));
  return LB_OK;
}

void drop_graphs(Engine& E) {
  for (auto*& gexec : E.graph) {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }
}

// Assign tile bases from the members' geometries and rebuild the tile map.
int retile(Engine& E) {
  int base = 0;
  std::vector<int> map;
  for (int i = 0; i < (int)E.m.size(); ++i) {
    E.m[i].d.tile_base = base;
    base += E.m[i].d.g.ntiles;
    map.insert(map.end(), E.m[i].d.g.ntiles, i);
  }
  if (base > E.slot_tiles) return E.fail(LB_E_NOMEM, "tile slots exhausted");
  E.ntiles = base;
  if (E.m.size() > 1) {
    HIPCK(E, hipMemcpyAsync(E.d_tile_lattice, map.data(), map.size() * sizeof(int),
                            hipMemcpyHostToDevice, E.stream));
    HIPCK(E, hipStreamSynchronize(E.stream));
  }
  drop_graphs(E);
  return upload_descs(E);
}

int engine_create(Engine& E, const lb_params* ps, int n, void* buffer, size_t buffer_bytes,
                  hipStream_t stream) {
  std::string why;
  if (validate_set(ps, n, &why) != LB_OK) return E.fail(LB_E_INVAL, why);
  E.fp64 = ps[0].precision == LB_FP64;
  E.walls = ps[0].boundary == LB_COUETTE_Y;
  E.stream = stream;
  if (hipGetDevice(&E.device) != hipSuccess) return E.fail(LB_E_DEVICE, "no HIP device");
  std::vector<lb_params> v(ps, ps + n);
  std::vector<lbk::Geometry> gs;
  int slots = 0;
  for (int i = 0; i < n; ++i) {
    gs.push_back(make_geometry(&ps[i], 0));
    slots += max_tiles(&ps[i]);
  }
  const EngineLayout L = engine_layout(v, gs, slots);
  E.bytes = L.total;
  E.slot_tiles = slots;
  if (buffer) {
    if (buffer_bytes < L.total || ((uintptr_t)buffer % kAlign) != 0)
      return E.fail(LB_E_NOMEM, "device_buffer too small or not 256-byte aligned");
    E.base = (char*)buffer;
    E.owns = false;
  } else {
    void* b = nullptr;
    if (hipMalloc(&b, L.total) != hipSuccess) {
      (void)hipGetLastError();
      return E.fail(LB_E_NOMEM, "hipMalloc of the workspace failed");
    }
    E.base = (char*)b;
    E.owns = true;
  }
  E.d_descs = (lbk::LatticeDesc*)(E.base + L.descs);
  E.d_tile_lattice = (int*)(E.base + L.tile_lattice);
  E.wave_red = (double*)(E.base + L.wave_red);
  E.wave_wall = (double*)(E.base + L.wave_wall);
  E.red_out = (double*)(E.base + L.red_out);
  E.flags = (int*)(E.base + L.flags);
  size_t total_pop = 0;
  for (int i = 0; i < n; ++i) {
    Member mm;
    mm.p = ps[i];
    mm.d.g = gs[i];
    mm.d.c = make_coefs(&ps[i]);
    mm.pop_bytes = pop_bytes_of(&ps[i], gs[i]);
    mm.wall_bytes = wall_bytes_of(&ps[i]);
    char* mb = E.base + L.member_off[i];
    mm.d.buf[0] = mb;
    mm.d.buf[1] = mb + mm.pop_bytes;
    mm.d.wall[0] = mb + 2 * mm.pop_bytes;
    mm.d.wall[1] = mb + 2 * mm.pop_bytes + mm.wall_bytes;
    mm.d.flag = E.flags + i;
    mm.d.phase = 0;
    total_pop += 2 * mm.pop_bytes;
    E.m.push_back(mm);
  }
  // Defaults: prefetch for FP32 (registers allow it), streaming stores when
  // the population buffers exceed the 256 MB Infinity Cache.
  E.variant.prefetch = E.fp64 ? 0 : 1;
  E.variant.stream_stores = total_pop > kInfinityCacheBytes ? 1 : 0;
  if (const char* e = std::getenv("LBSOFT_PREFETCH")) E.variant.prefetch = std::atoi(e) ? 1 : 0;
  if (const char* e = std::getenv("LBSOFT_STREAM_STORES"))
    E.variant.stream_stores = std::atoi(e) ? 1 : 0;
  HIPCK(E, hipMemsetAsync(E.base, 0, L.total, E.stream));
  const int rc = retile(E);
  if (rc != LB_OK) return rc;
  HIPCK(E, hipStreamSynchronize(E.stream));
  return LB_OK;
}

void engine_destroy(Engine& E) {
  DeviceGuard dg(E.device);
  (void)hipStreamSynchronize(E.stream);
  drop_graphs(E);
  if (E.capture_stream) (void)hipStreamDestroy(E.capture_stream);
  E.capture_stream = nullptr;
  if (E.owns && E.base) (void)hipFree(E.base);
  E.base = nullptr;
}

lbk::LaunchArgs launch_args(const Engine& E, int parity) {
  lbk::LaunchArgs a{};
  a.descs = E.d_descs;
  a.tile_lattice = E.m.size() > 1 ? E.d_tile_lattice : nullptr;
  a.ntiles = E.ntiles;
  a.tiles_per_xcd = (E.ntiles + 7) / 8;
  a.parity = parity;
  a.wave_red = E.wave_red;
  a.wave_wall = E.wave_wall;
  a.accumulate_wall = E.walls ? 1 : 0;
  return a;
}

// Launch args for one member alone (observe / fields).
lbk::LaunchArgs member_args(const Engine& E, int i) {
  lbk::LaunchArgs a{};
  a.descs = E.d_descs + i;
  a.tile_lattice = nullptr;
  a.ntiles = E.m[i].d.g.ntiles;
  a.tiles_per_xcd = (a.ntiles + 7) / 8;
  a.parity = (int)(E.step & 1);
  a.wave_red = E.wave_red + (size_t)E.m[i].d.tile_base * lbk::kNRed;
  a.wave_wall = E.wave_wall + (size_t)E.m[i].d.tile_base * 2;
  return a;
}

int check_flags(Engine& E, std::vector<int>* out) {
  std::vector<int> f(E.m.size(), 0);
  HIPCK(E, hipMemcpyAsync(f.data(), E.flags, f.size() * sizeof(int), hipMemcpyDeviceToHost,
                          E.stream));
  HIPCK(E, hipStreamSynchronize(E.stream));
  bool bad = false;
  for (int v : f) bad |= (v & 1) != 0;
  if (out) *out = f;
  if (bad) return E.fail(LB_E_UNSTABLE, "non-finite or non-positive density on the device");
  return LB_OK;
}

// Member i's state is set at engine step E.step: it starts in buf[0].
void begin_member(Engine& E, int i, int64_t member_t) {
  Member& mm = E.m[i];
  mm.d.phase = (int)(E.step & 1);
  mm.t_base = member_t;
  mm.e_base = E.step;
  mm.avg_start = E.step;
  mm.initialized = true;
}

int zero_member_slots(Engine& E, int i) {
  const Member& mm = E.m[i];
  HIPCK(E, hipMemsetAsync(E.wave_wall + (size_t)mm.d.tile_base * 2, 0,
                          (size_t)mm.d.g.ntiles * 2 * sizeof(double), E.stream));
  HIPCK(E, hipMemsetAsync(E.flags + i, 0, sizeof(int), E.stream));
  return LB_OK;
}

void set_rho_ref(Engine& E, int i, const double* ra, const double* rb, size_t n) {
  Member& mm = E.m[i];
  if (E.fp64) return;
  const double* r[2] = {ra, rb};
  for (int s = 0; s < 2; ++s) {
    if (mm.p.rho_ref[s] > 0) {
      mm.d.c.rho_ref[s] = mm.p.rho_ref[s];
      continue;
    }
    double acc = 0;
    for (size_t k = 0; k < n; ++k) acc += r[s][k];
    mm.d.c.rho_ref[s] = acc / (double)n;
  }
  round_coefs(mm.d.c);
}

int init_from_device_rho(Engine& E, int i, const double* d_rho, const double* d_u) {
  Member& mm = E.m[i];
  begin_member(E, i, 0);
  int rc = upload_descs(E);
  if (rc != LB_OK) return rc;
  HIPCK(E, lbk::launch_init(mm.d.g, mm.d.c, E.fp64, E.walls, d_rho, d_u, mm.d.buf[0], mm.d.wall[0],
                            E.stream));
  rc = zero_member_slots(E, i);
  if (rc != LB_OK) return rc;
  HIPCK(E, hipStreamSynchronize(E.stream));
  return LB_OK;
}

int engine_init(Engine& E, int i, const double* rho_a, const double* rho_b, const double* ux,
                const double* uy) {
  if (i < 0 || i >= (int)E.m.size()) return E.fail(LB_E_INVAL, "lattice index out of range");
  if (!rho_a || !rho_b) return E.fail(LB_E_INVAL, "rho_a and rho_b are required");
  if ((ux == nullptr) != (uy == nullptr)) return E.fail(LB_E_INVAL, "give both ux and uy or neither");
  const Member& mm = E.m[i];
  const size_t n = (size_t)mm.d.g.nx * mm.d.g.ny;
  for (size_t k = 0; k < n; ++k) {
    if (!is_finite(rho_a[k]) || !(rho_a[k] > 0) || !is_finite(rho_b[k]) || !(rho_b[k] > 0))
      return E.fail(LB_E_INVAL, "densities must be finite and > 0");
    if (ux && (!is_finite(ux[k]) || !is_finite(uy[k])))
      return E.fail(LB_E_INVAL, "velocities must be finite");
  }
  DeviceGuard dg(E.device);
  set_rho_ref(E, i, rho_a, rho_b, n);
  DevTmp t;
  const size_t nb = n * sizeof(double);
  HIPCK(E, hipMalloc(&t.p, (ux ? 4 : 2) * nb));
  double* d = (double*)t.p;
  HIPCK(E, hipMemcpyAsync(d, rho_a, nb, hipMemcpyHostToDevice, E.stream));
  HIPCK(E, hipMemcpyAsync(d + n, rho_b, nb, hipMemcpyHostToDevice, E.stream));
  if (ux) {
    HIPCK(E, hipMemcpyAsync(d + 2 * n, ux, nb, hipMemcpyHostToDevice, E.stream));
    HIPCK(E, hipMemcpyAsync(d + 3 * n, uy, nb, hipMemcpyHostToDevice, E.stream));
  }
  return init_from_device_rho(E, i, d, ux ? d + 2 * n : nullptr);
}

int engine_init_noise(Engine& E, int i, uint64_t seed, double mean_a, double mean_b, double amp) {
  if (i < 0 || i >= (int)E.m.size()) return E.fail(LB_E_INVAL, "lattice index out of range");
  if (!is_finite(mean_a) || !is_finite(mean_b) || !is_finite(amp) ||
      !(std::fabs(amp) < std::min(mean_a, mean_b)))
    return E.fail(LB_E_INVAL, "need |amp| < min(mean_a, mean_b) and finite values");
  DeviceGuard dg(E.device);
  Member& mm = E.m[i];
  if (!E.fp64) {
    mm.d.c.rho_ref[0] = mm.p.rho_ref[0] > 0 ? mm.p.rho_ref[0] : mean_a;
    mm.d.c.rho_ref[1] = mm.p.rho_ref[1] > 0 ? mm.p.rho_ref[1] : mean_b;
    round_coefs(mm.d.c);
  }
  const size_t n = (size_t)mm.d.g.nx * mm.d.g.ny;
  DevTmp t;
  HIPCK(E, hipMalloc(&t.p, 2 * n * sizeof(double)));
  HIPCK(E, lbk::launch_noise(mm.d.g.nx, mm.d.g.ny, seed, mean_a, mean_b, amp, (double*)t.p, E.stream));
  return init_from_device_rho(E, i, (const double*)t.p, nullptr);
}

// Capture two consecutive steps starting at the given parity into a graph.
// Capture runs on a private non-blocking stream (the caller's stream may be
// the null stream, which cannot be captured); replays go to the caller's
// stream.  The graph holds the two kernel nodes only.
int capture_pair(Engine& E, int parity) {
  if (!E.capture_stream) HIPCK(E, hipStreamCreateWithFlags(&E.capture_stream, hipStreamNonBlocking));
  HIPCK(E, hipStreamBeginCapture(E.capture_stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < 2; ++k) {
    const hipError_t le = lbk::launch_step(launch_args(E, (parity + k) & 1), E.fp64, E.walls,
                                           E.variant, E.capture_stream);
    if (le != hipSuccess) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(E.capture_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      return E.fail(LB_E_DEVICE, std::string("capture: ") + hipGetErrorString(le));
    }
  }
  hipGraph_t g = nullptr;
  HIPCK(E, hipStreamEndCapture(E.capture_stream, &g));
  const hipError_t ie = hipGraphInstantiate(&E.graph[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    E.graph[parity] = nullptr;
    return E.fail(LB_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  }
  return LB_OK;
}

int engine_step(Engine& E, int64_t n) {
  if (n < 0) return E.fail(LB_E_INVAL, "n must be >= 0");
  for (auto& mm : E.m)
    if (!mm.initialized) return E.fail(LB_E_STATE, "step before every lattice is initialized");
  DeviceGuard dg(E.device);
  int64_t k = 0;
  if (E.use_graph && n >= 2) {
    const int par = (int)(E.step & 1);
    if (!E.graph[par]) {
      const int rc = capture_pair(E, par);
      if (rc != LB_OK) return rc;
    }
    for (; k + 2 <= n; k += 2) {
      HIPCK(E, hipGraphLaunch(E.graph[par], E.stream));
      E.step += 2;
    }
  }
  for (; k < n; ++k) {
    HIPCK(E, lbk::launch_step(launch_args(E, (int)(E.step & 1)), E.fp64, E.walls, E.variant, E.stream));
    ++E.step;
  }
  return LB_OK;
}

void fill_obs(const Engine& E, int i, const double* h, int flag, lb_obs* out) {
  const Member& mm = E.m[i];
  std::memset(out, 0, sizeof(*out));
  out->step = mm.t_base + (E.step - mm.e_base);
  out->mass[0] = h[0];
  out->mass[1] = h[1];
  out->mom[0] = h[2];
  out->mom[1] = h[3];
  out->mom_phys[0] = h[4];
  out->mom_phys[1] = h[5];
  out->pxy_kin = h[6];
  out->avg_count = E.step - mm.avg_start;
  if (out->avg_count > 0 && E.walls) {
    out->wall_stress[0] = h[lbk::kNRed + 0] / (double)out->avg_count / (double)mm.d.g.nx;
    out->wall_stress[1] = h[lbk::kNRed + 1] / (double)out->avg_count / (double)mm.d.g.nx;
  }
  out->flags = flag;
}

int engine_observables(Engine& E, lb_obs* out /*[n]*/) {
  for (auto& mm : E.m)
    if (!mm.initialized) return E.fail(LB_E_STATE, "observables before every lattice is initialized");
  DeviceGuard dg(E.device);
  const int n = (int)E.m.size();
  HIPCK(E, lbk::launch_observe(launch_args(E, (int)(E.step & 1)), E.fp64, E.walls, E.stream));
  HIPCK(E, lbk::launch_reduce_lattices(E.d_descs, n, E.wave_red, lbk::kNRed, E.red_out, 16, E.stream));
  HIPCK(E, lbk::launch_reduce_lattices(E.d_descs, n, E.wave_wall, 2, E.red_out + lbk::kNRed, 16,
                                       E.stream));
  std::vector<double> h((size_t)n * 16);
  HIPCK(E, hipMemcpyAsync(h.data(), E.red_out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                          E.stream));
  std::vector<int> flags;
  const int rc = check_flags(E, &flags);
  if (flags.size() != (size_t)n) return rc;
  for (int i = 0; i < n; ++i) fill_obs(E, i, h.data() + (size_t)i * 16, flags[i], out + i);
  return rc;
}

int engine_fields(Engine& E, int i, double* rho_a, double* rho_b, double* u, double* u_phys) {
  if (i < 0 || i >= (int)E.m.size()) return E.fail(LB_E_INVAL, "lattice index out of range");
  if (!E.m[i].initialized) return E.fail(LB_E_STATE, "fields before lb_init");
  DeviceGuard dg(E.device);
  const size_t n = (size_t)E.m[i].d.g.nx * E.m[i].d.g.ny, nb = n * sizeof(double);
  DevTmp t;
  HIPCK(E, hipMalloc(&t.p, 6 * nb));
  double* d = (double*)t.p;
  lbk::LaunchArgs a = member_args(E, i);
  a.fields = d;
  HIPCK(E, lbk::launch_observe(a, E.fp64, E.walls, E.stream));
  if (rho_a) HIPCK(E, hipMemcpyAsync(rho_a, d, nb, hipMemcpyDeviceToHost, E.stream));
  if (rho_b) HIPCK(E, hipMemcpyAsync(rho_b, d + n, nb, hipMemcpyDeviceToHost, E.stream));
  if (u) HIPCK(E, hipMemcpyAsync(u, d + 2 * n, 2 * nb, hipMemcpyDeviceToHost, E.stream));
  if (u_phys) HIPCK(E, hipMemcpyAsync(u_phys, d + 4 * n, 2 * nb, hipMemcpyDeviceToHost, E.stream));
  return check_flags(E, nullptr);
}

int engine_pops(Engine& E, int i, double* f) {
  if (i < 0 || i >= (int)E.m.size() || !f) return E.fail(LB_E_INVAL, "bad lattice index or NULL f");
  if (!E.m[i].initialized) return E.fail(LB_E_STATE, "populations before lb_init");
  DeviceGuard dg(E.device);
  const size_t n = (size_t)E.m[i].d.g.nx * E.m[i].d.g.ny, nb = 18 * n * sizeof(double);
  DevTmp t;
  HIPCK(E, hipMalloc(&t.p, nb));
  lbk::LaunchArgs a = member_args(E, i);
  a.pops = (double*)t.p;
  HIPCK(E, lbk::launch_observe(a, E.fp64, E.walls, E.stream));
  HIPCK(E, hipMemcpyAsync(f, t.p, nb, hipMemcpyDeviceToHost, E.stream));
  return check_flags(E, nullptr);
}

int engine_set_pops(Engine& E, int i, const double* f, int64_t member_t) {
  if (i < 0 || i >= (int)E.m.size() || !f) return E.fail(LB_E_INVAL, "bad lattice index or NULL f");
  if (member_t < 0) return E.fail(LB_E_INVAL, "step must be >= 0");
  Member& mm = E.m[i];
  const size_t n = (size_t)mm.d.g.nx * mm.d.g.ny;
  for (size_t k = 0; k < 18 * n; ++k)
    if (!is_finite(f[k])) return E.fail(LB_E_INVAL, "populations must be finite");
  DeviceGuard dg(E.device);
  if (!E.fp64 && !mm.initialized) {
    // reference densities from these populations when none were given
    std::vector<double> ra(n, 0.0), rb(n, 0.0);
    for (int q = 0; q < 9; ++q)
      for (size_t k = 0; k < n; ++k) {
        ra[k] += f[(size_t)q * n + k];
        rb[k] += f[(size_t)(9 + q) * n + k];
      }
    set_rho_ref(E, i, ra.data(), rb.data(), n);
  }
  DevTmp t;
  HIPCK(E, hipMalloc(&t.p, 18 * n * sizeof(double)));
  HIPCK(E, hipMemcpyAsync(t.p, f, 18 * n * sizeof(double), hipMemcpyHostToDevice, E.stream));
  begin_member(E, i, member_t);
  int rc = upload_descs(E);
  if (rc != LB_OK) return rc;
  HIPCK(E, lbk::launch_set_pops(mm.d.g, mm.d.c, E.fp64, E.walls, (const double*)t.p, mm.d.buf[0],
                                mm.d.wall[0], E.stream));
  rc = zero_member_slots(E, i);
  if (rc != LB_OK) return rc;
  HIPCK(E, hipStreamSynchronize(E.stream));
  return LB_OK;
}

int engine_reset_averages(Engine& E) {
  DeviceGuard dg(E.device);
  HIPCK(E, hipMemsetAsync(E.wave_wall, 0, (size_t)E.ntiles * 2 * sizeof(double), E.stream));
  for (auto& mm : E.m) mm.avg_start = E.step;
  return LB_OK;
}

void engine_info(const Engine& E, lb_launch_info* out) {
  std::memset(out, 0, sizeof(*out));
  const auto& g = E.m[0].d.g;
  out->nstrips = g.nstrips;
  out->nsegs = g.nsegs;
  out->ntiles = E.ntiles;
  out->grid_blocks = 8 * ((E.ntiles + 7) / 8);
  out->block_threads = lbk::kWave;
  out->pitch = g.pitch;
  out->workspace_bytes = E.bytes;
  size_t pb = 0;
  for (auto& mm : E.m) pb += mm.pop_bytes;
  out->population_bytes = pb;
  out->seg_h = g.seg_h;
  out->prefetch = E.variant.prefetch;
  out->stream_stores = E.variant.stream_stores;
  out->use_graph = E.use_graph ? 1 : 0;
}

int set_variant(Engine& E, int32_t prefetch, int32_t stream_stores, int32_t use_graph) {
  if (prefetch >= 0) E.variant.prefetch = prefetch ? 1 : 0;
  if (stream_stores >= 0) E.variant.stream_stores = stream_stores ? 1 : 0;
  if (use_graph >= 0) E.use_graph = use_graph != 0;
  drop_graphs(E);
  return LB_OK;
}

}  // namespace

struct lb_lattice {
  Engine e;
};
struct lb_batch {
  Engine e;
};

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

const char* lb_last_error(const lb_lattice* L) { return L ? L->e.err.c_str() : "null handle"; }

int lb_workspace_bytes(const lb_params* p, size_t* out) {
  if (!out) return LB_E_INVAL;
  const int v = validate(p, nullptr);
  if (v != LB_OK) return v;
  *out = engine_bytes(p, 1);
  return LB_OK;
}

int lb_create(const lb_params* p, void* hip_stream, lb_lattice** out) {
  if (!out) return LB_E_INVAL;
  *out = nullptr;
  const int v = validate(p, nullptr);
  if (v != LB_OK) return v;
  lb_lattice* L = new (std::nothrow) lb_lattice();
  if (!L) return LB_E_NOMEM;
  const int rc = engine_create(L->e, p, 1, p->device_buffer, p->device_bytes, (hipStream_t)hip_stream);
  if (rc != LB_OK) {
    engine_destroy(L->e);
    delete L;
    return rc;
  }
  *out = L;
  return LB_OK;
}

void lb_destroy(lb_lattice* L) {
  if (!L) return;
  engine_destroy(L->e);
  delete L;
}

int lb_init(lb_lattice* L, const double* rho_a, const double* rho_b, const double* ux,
            const double* uy) {
  if (!L) return LB_E_INVAL;
  return engine_init(L->e, 0, rho_a, rho_b, ux, uy);
}

int lb_init_noise(lb_lattice* L, uint64_t seed, double mean_a, double mean_b, double amp) {
  if (!L) return LB_E_INVAL;
  return engine_init_noise(L->e, 0, seed, mean_a, mean_b, amp);
}

int lb_step(lb_lattice* L, int64_t n) {
  if (!L) return LB_E_INVAL;
  return engine_step(L->e, n);
}

int lb_observables(lb_lattice* L, lb_obs* out) {
  if (!L || !out) return LB_E_INVAL;
  return engine_observables(L->e, out);
}

int lb_get_fields(lb_lattice* L, double* rho_a, double* rho_b, double* u, double* u_phys) {
  if (!L) return LB_E_INVAL;
  return engine_fields(L->e, 0, rho_a, rho_b, u, u_phys);
}

int lb_get_populations(lb_lattice* L, double* f) {
  if (!L || !f) return LB_E_INVAL;
  return engine_pops(L->e, 0, f);
}

int lb_set_populations(lb_lattice* L, const double* f, int64_t step) {
  if (!L || !f) return LB_E_INVAL;
  return engine_set_pops(L->e, 0, f, step);
}

int lb_reset_averages(lb_lattice* L) {
  if (!L) return LB_E_INVAL;
  return engine_reset_averages(L->e);
}

int lb_sync(lb_lattice* L) {
  if (!L) return LB_E_INVAL;
  DeviceGuard dg(L->e.device);
  return check_flags(L->e, nullptr);
}

int64_t lb_current_step(const lb_lattice* L) {
  if (!L) return -1;
  const Member& mm = L->e.m[0];
  return mm.t_base + (L->e.step - mm.e_base);
}

int lb_get_launch_info(const lb_lattice* L, lb_launch_info* out) {
  if (!L || !out) return LB_E_INVAL;
  engine_info(L->e, out);
  return LB_OK;
}

int lb_set_launch(lb_lattice* L, int32_t seg_h, int32_t prefetch, int32_t stream_stores,
                  int32_t use_graph) {
  if (!L) return LB_E_INVAL;
  Engine& E = L->e;
  DeviceGuard dg(E.device);
  set_variant(E, prefetch, stream_stores, use_graph);
  if (seg_h >= 0) {
    for (auto& mm : E.m) mm.d.g = make_geometry(&mm.p, seg_h);
    const int rc = retile(E);
    if (rc != LB_OK) return rc;
    return engine_reset_averages(E);
  }
  return LB_OK;
}

/* ------------------------------ batches ------------------------------ */

const char* lb_batch_last_error(const lb_batch* B) { return B ? B->e.err.c_str() : "null handle"; }

int lb_batch_workspace_bytes(const lb_params* p, int32_t n, size_t* out) {
  if (!out) return LB_E_INVAL;
  const int v = validate_set(p, n, nullptr);
  if (v != LB_OK) return v;
  *out = engine_bytes(p, n);
  return LB_OK;
}

int lb_batch_create(const lb_params* p, int32_t n, void* device_buffer, size_t device_bytes,
                    void* hip_stream, lb_batch** out) {
  if (!out) return LB_E_INVAL;
  *out = nullptr;
  const int v = validate_set(p, n, nullptr);
  if (v != LB_OK) return v;
  lb_batch* B = new (std::nothrow) lb_batch();
  if (!B) return LB_E_NOMEM;
  const int rc = engine_create(B->e, p, n, device_buffer, device_bytes, (hipStream_t)hip_stream);
  if (rc != LB_OK) {
    engine_destroy(B->e);
    delete B;
    return rc;
  }
  *out = B;
  return LB_OK;
}

void lb_batch_destroy(lb_batch* B) {
  if (!B) return;
  engine_destroy(B->e);
  delete B;
}

int32_t lb_batch_size(const lb_batch* B) { return B ? (int32_t)B->e.m.size() : -1; }

int lb_batch_init(lb_batch* B, int32_t i, const double* rho_a, const double* rho_b,
                  const double* ux, const double* uy) {
  if (!B) return LB_E_INVAL;
  return engine_init(B->e, i, rho_a, rho_b, ux, uy);
}

int lb_batch_init_noise(lb_batch* B, int32_t i, uint64_t seed, double mean_a, double mean_b,
                        double amp) {
  if (!B) return LB_E_INVAL;
  return engine_init_noise(B->e, i, seed, mean_a, mean_b, amp);
}

int lb_batch_step(lb_batch* B, int64_t n) {
  if (!B) return LB_E_INVAL;
  return engine_step(B->e, n);
}

int lb_batch_observables(lb_batch* B, lb_obs* out) {
  if (!B || !out) return LB_E_INVAL;
  return engine_observables(B->e, out);
}

int lb_batch_get_fields(lb_batch* B, int32_t i, double* rho_a, double* rho_b, double* u,
                        double* u_phys) {
  if (!B) return LB_E_INVAL;
  return engine_fields(B->e, i, rho_a, rho_b, u, u_phys);
}

int lb_batch_get_populations(lb_batch* B, int32_t i, double* f) {
  if (!B) return LB_E_INVAL;
  return engine_pops(B->e, i, f);
}

int lb_batch_sync(lb_batch* B) {
  if (!B) return LB_E_INVAL;
  DeviceGuard dg(B->e.device);
  return check_flags(B->e, nullptr);
}

int lb_batch_get_launch_info(const lb_batch* B, lb_launch_info* out) {
  if (!B || !out) return LB_E_INVAL;
  engine_info(B->e, out);
  return LB_OK;
}

int lb_batch_set_launch(lb_batch* B, int32_t prefetch, int32_t stream_stores, int32_t use_graph) {
  if (!B) return LB_E_INVAL;
  DeviceGuard dg(B->e.device);
  return set_variant(B->e, prefetch, stream_stores, use_graph);
}

}  // extern "C"
