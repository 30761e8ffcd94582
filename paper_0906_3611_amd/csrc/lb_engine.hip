// Engine: lattices of one precision and boundary type advancing together,
// one step launch over the tiles of all of them (see lb_engine.h).
#include "lb_engine.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include <unistd.h>

namespace lbe {
static_assert(lbk::kNRed + 2 <= 16, "reduction output rows hold 16 doubles");
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

// Default tile policy (measured).  The population kernels run fastest with
// about one wave of resident workgroups: ~2048 tiles for FP32 (k_split,
// two-wave workgroups, ~10 per CU) and ~1024 for FP64 (k_march, one wave
// per SIMD), whatever height that gives: at 4096^2 128-row segments beat
// 32-row ones by 2% periodic and 9% with walls (more tiles than fit at once
// lose the L2 reuse of the halo rows between segments: 1.21x the
// algorithmic reads at 32 rows).  The moment kernel, bound by instruction
// issue, prefers more tiles: segments of at most base_seg_h rows (4096^2:
// 66.0 G site updates/s at 32 rows, 60.3 at 128).  Segments get shorter
// (down to 4 rows) only to reach the tile count: a lattice too small to fill
// the GPU is bound by the latency of one tile's march, which 4-row segments
// cut from 12 to 8 rows (128^2: 10.1 us per step against 14.7 with 8-row
// segments, FP64 17.3 against 26.7; 512^2: 14.0 against 18.6).
int target_tiles(const lb_params* p) { return p->precision == LB_FP64 ? 1024 : 2048; }
int base_seg_h(const lb_params* p) { return p->precision == LB_FP64 ? 64 : 32; }

// Tiles: 64-column strips x row segments (see target_tiles).  seg_h > 0
// forces the segment height.
lbk::Geometry make_geometry(const lb_params* p, int seg_h) {
  lbk::Geometry g{};
  g.nx = p->nx;
  g.ny = p->ny;
  g.pitch = (p->nx + lbk::kWave - 1) / lbk::kWave * lbk::kWave;  // strips start on a line
  g.row_elems = (long long)(g.pitch / lbk::kWave) * (p->precision == LB_FP32_MOM ? 6 : 18) * lbk::kWave;
  g.nstrips = (p->nx + lbk::kWave - 1) / lbk::kWave;
  int nsegs = (target_tiles(p) + g.nstrips - 1) / g.nstrips;
  if (p->precision == LB_FP32_MOM) {
    const int h0 = base_seg_h(p);
    nsegs = std::max(nsegs, (p->ny + h0 - 1) / h0);
  }
  nsegs = std::min(nsegs, std::max(1, p->ny / 4));
  if (seg_h >= 4) nsegs = (p->ny + seg_h - 1) / seg_h;
  nsegs = std::max(1, std::min(nsegs, p->ny));
  g.nsegs = nsegs;
  g.seg_h = (p->ny + nsegs - 1) / nsegs;
  g.ntiles = g.nstrips * g.nsegs;
  return g;
}

// Reduction slots: observables per (row, strip), wall momentum per strip;
// neither depends on the segment height.
size_t red_slots(const lb_params* p) {
  return (size_t)p->ny * (size_t)((p->nx + lbk::kWave - 1) / lbk::kWave);
}
size_t wall_slots(const lb_params* p) { return (size_t)((p->nx + lbk::kWave - 1) / lbk::kWave); }

// The most tiles any segment height >= 4 can give (sizes the tile map).
int max_tiles_of(const lb_params* p) {
  const int nstrips = (p->nx + lbk::kWave - 1) / lbk::kWave;
  const int nsegs = std::max(1, std::min(p->ny, (p->ny + 3) / 4));
  return std::max(nstrips * nsegs, make_geometry(p, 0).ntiles);
}

size_t elem_size(const lb_params* p) { return p->precision == LB_FP64 ? 8 : 4; }

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
  c.f_g_body = (float)c.g_body;
  c.f_g_uniform = (float)c.g_uniform;
  c.f_inv_ny2 = (float)c.inv_ny2;
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
  c.g_body = p->body_force;
  c.g_uniform = p->body_force_x;
  c.inv_ny2 = 2.0 / (double)p->ny;
  round_coefs(c);
  return c;
}

// Temporary device array freed at scope exit.
struct DevTmp {
  void* p = nullptr;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
};

#define HIPCK(E, expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return (E).fail(LB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t shared_bytes(int cap_members, int cap_tiles) {
  return align_up((size_t)cap_members * sizeof(lbk::LatticeDesc)) +
         align_up((size_t)cap_tiles * sizeof(int)) + align_up((size_t)cap_members * 16 * sizeof(double));
}

void carve_shared(Engine& E, char* p, int cap_members, int cap_tiles) {
  E.shared = p;
  E.cap_members = cap_members;
  E.cap_tiles = cap_tiles;
  E.d_descs = (lbk::LatticeDesc*)p;
  p += align_up((size_t)cap_members * sizeof(lbk::LatticeDesc));
  E.d_tile_lattice = (int*)p;
  p += align_up((size_t)cap_tiles * sizeof(int));
  E.red_out = (double*)p;
}

// Build a member record for parameters p over the device region `region`.
Member make_member(const lb_params* p, char* region, bool owns, int64_t tag) {
  Member mm;
  mm.p = *p;
  mm.p.device_buffer = nullptr;
  mm.p.device_bytes = 0;
  mm.d.g = make_geometry(p, 0);
  mm.d.c = make_coefs(p);
  mm.pop_bytes = align_up((size_t)mm.d.g.row_elems * (size_t)mm.d.g.ny * elem_size(p));
  mm.wall_bytes = align_up(12ull * (size_t)p->nx * elem_size(p));
  mm.max_tiles = max_tiles_of(p);
  mm.region_bytes = member_region_bytes(p);
  mm.region = region;
  mm.owns_region = owns;
  mm.tag = tag;
  char* q = region;
  mm.d.buf[0] = q;
  mm.d.buf[1] = q + mm.pop_bytes;
  q += 2 * mm.pop_bytes;
  mm.d.wall[0] = q;
  mm.d.wall[1] = q + mm.wall_bytes;
  q += 2 * mm.wall_bytes;
  mm.d.wave_red = (double*)q;
  q += align_up(red_slots(p) * lbk::kNRed * sizeof(double));
  mm.d.wave_wall = (double*)q;
  q += align_up(wall_slots(p) * 2 * sizeof(double));
  mm.d.phi_ref = (double*)q;
  q += align_up((size_t)p->nx * (size_t)p->ny * sizeof(double));
  mm.d.flag = (int*)q;
  mm.d.phase = 0;
  return mm;
}

int upload_descs(Engine& E) {
  if (E.m.empty()) return LB_OK;
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

// Grow the shared region of a dynamic engine to hold `members` lattices
// and `tiles` tiles.
int reserve_shared(Engine& E, int members, int tiles) {
  if (members <= E.cap_members && tiles <= E.cap_tiles) return LB_OK;
  if (!E.owns_shared) return E.fail(LB_E_NOMEM, "engine capacity exhausted");
  const int cm = std::max(members, 2 * E.cap_members), ct = std::max(tiles, 2 * E.cap_tiles);
  void* b = nullptr;
  if (hipMalloc(&b, shared_bytes(cm, ct)) != hipSuccess) {
    (void)hipGetLastError();
    return E.fail(LB_E_NOMEM, "hipMalloc of the engine tables failed");
  }
  HIPCK(E, hipStreamSynchronize(E.stream));
  if (E.shared) {
    (void)hipFree(E.shared);
    E.bytes -= shared_bytes(E.cap_members, E.cap_tiles);
  }
  carve_shared(E, (char*)b, cm, ct);
  E.bytes += shared_bytes(cm, ct);
  return LB_OK;
}

void choose_default_variant(Engine& E);

// Whether the FP32 deviation step may group tiles: every (selected)
// lattice has a whole number of groups of strips, so that the tiles of a
// group lie in one segment of one lattice.
bool group_allowed(const Engine& E, const std::vector<int>* sel) {
  if (!split_kernel(E)) return false;
  auto ok = [&](const Member& mm) { return mm.d.g.nstrips % lbk::kGroupTiles == 0; };
  if (sel) {
    for (int i : *sel)
      if (!ok(E.m[i])) return false;
  } else {
    for (auto& mm : E.m)
      if (!ok(mm)) return false;
  }
  return true;
}

// Member geometries.  A forced height applies to every member.  Otherwise a
// single lattice uses make_geometry's policy, and several lattices share one
// segment height: base_seg_h, halved (down to 4) only while the engine's
// tiles stay under target_tiles, so that small members are not cut into
// short segments when the whole launch has tiles to spare.
// The storage layout does not depend on the segment height, so a launch
// over some of the members may tile them as if they were alone (sel: member
// indices; null: every member).
std::vector<lbk::Geometry> geometries(const Engine& E, int seg_h,
                                      const std::vector<int>* sel = nullptr) {
  std::vector<const lb_params*> ps;
  if (sel)
    for (int i : *sel) ps.push_back(&E.m[i].p);
  else
    for (auto& mm : E.m) ps.push_back(&mm.p);
  std::vector<lbk::Geometry> g;
  int h = seg_h;
  if (seg_h < 4 && ps.size() > 1) {
    const lb_params* p0 = ps[0];  // members share the precision
    for (h = base_seg_h(p0); h > 4; h /= 2) {
      long long tiles = 0;
      for (auto* p : ps) tiles += (long long)make_geometry(p, h).ntiles;
      if (tiles >= target_tiles(p0)) break;
    }
  }
  for (auto* p : ps) g.push_back(make_geometry(p, h));
  return g;
}

void apply_geometry(Engine& E) {
  const auto g = geometries(E, E.seg_h);
  for (size_t i = 0; i < E.m.size(); ++i) E.m[i].d.g = g[i];
}

// Assign tile bases from the members' geometries and rebuild the tile map.
int retile(Engine& E) {
  apply_geometry(E);
  int base = 0;
  std::vector<int> map;
  for (int i = 0; i < (int)E.m.size(); ++i) {
    E.m[i].d.tile_base = base;
    base += E.m[i].d.g.ntiles;
    map.insert(map.end(), E.m[i].d.g.ntiles, i);
  }
  const int rc = reserve_shared(E, (int)E.m.size(), base);
  if (rc != LB_OK) return rc;
  E.ntiles = base;
  choose_default_variant(E);
  if (E.m.size() > 1) {
    HIPCK(E, hipMemcpyAsync(E.d_tile_lattice, map.data(), map.size() * sizeof(int),
                            hipMemcpyHostToDevice, E.stream));
    HIPCK(E, hipStreamSynchronize(E.stream));
  }
  drop_graphs(E);
  return upload_descs(E);
}

void choose_default_variant(Engine& E) {
  // Defaults (measured): streaming stores when the population buffers
  // exceed the 256 MB Infinity Cache.  A one-row prefetch for the
  // population storages with one tile per workgroup: FP32 deviations (one
  // wave per species) step 1.6-3.7% faster with it than without at 1024^2 to
  // 4096^2, periodic and with walls; FP64 (one wave per SIMD) likewise, and
  // more so with two rows (below).  Grouped tiles step 1.5-4% faster without it (2048^2 to 8192 x 1024,
  // periodic and with walls; 1024 x 4096 and 2048 x 1024 the same): the
  // group's eight waves meet at every row's barrier, and loads issued
  // there, all waves at once, gain nothing from being issued a row early.
  E.group_ok = group_allowed(E, nullptr);
  if (E.variant_forced) return;
  size_t total_pop = 0;
  for (auto& mm : E.m) total_pop += 2 * mm.pop_bytes;
  const bool hbm = total_pop > kInfinityCacheBytes;
  // FP64 (k_march, which turns its march round at every step) keeps plain
  // stores up to twice the Infinity Cache: a step then reads much of what
  // the previous one wrote from it (1024^2 2.9-3.7% faster than with
  // streaming stores, 512 x 2048 2%, 768 x 2048 0.8%; 4096 x 1024 1% slower).
  const bool march = E.fp64;
  E.variant.stream_stores = hbm && !(march && total_pop <= 2 * kInfinityCacheBytes) ? 1 : 0;
  // Four tiles of adjacent strips per workgroup for lattices larger than the
  // Infinity Cache (measured 1-5% faster from 8192 x 512 to 4096^2 and on the
  // 4096 x 1024 channel with walls; 8% slower on the cache-resident 1024^2
  // emulsion).
  E.variant.group = (E.group_ok && hbm) ? lbk::kGroupTiles : 1;
  // FP64 (k_march, one wave per SIMD at any depth) keeps two rows in flight:
  // 0.5-1.5% faster than one from 512 x 2048 to 4096 x 1024.
  E.variant.prefetch = (hbm && (E.mom || E.variant.group > 1)) ? 0 : (E.fp64 ? 2 : 1);
}

lbk::LaunchArgs launch_args(const Engine& E, int parity) {
  lbk::LaunchArgs a{};
  a.descs = E.d_descs;
  a.tile_lattice = E.m.size() > 1 ? E.d_tile_lattice : nullptr;
  a.ntiles = E.ntiles;
  a.tiles_per_xcd = (E.ntiles + 7) / 8;
  a.parity = parity;
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
  return a;
}

// Status of a member's device flag word: bit 0, a non-finite or
// non-positive density; bit 1, a grouped step launch whose tiles did not
// march equally far (those tiles were not stepped; the host's grouping rule
// excludes it).
int flag_status(Engine& E, int v) {
  if (v & 2) return E.fail(LB_E_DEVICE, "a grouped step launch met tiles of unequal heights");
  if (v & 1) return E.fail(LB_E_UNSTABLE, "non-finite or non-positive density on the device");
  return LB_OK;
}

int read_flags(Engine& E, std::vector<int>* out) {
  std::vector<int> f(E.m.size(), 0);
  for (size_t i = 0; i < E.m.size(); ++i)
    HIPCK(E, hipMemcpyAsync(&f[i], E.m[i].d.flag, sizeof(int), hipMemcpyDeviceToHost, E.stream));
  HIPCK(E, hipStreamSynchronize(E.stream));
  int any = 0;
  for (int v : f) any |= v;
  if (out) *out = f;
  return flag_status(E, any);
}

// Member i's state is set at engine step E.step: it starts in buf[0].
void begin_member(Engine& E, int i, int64_t member_t) {
  Member& mm = E.m[i];
  mm.d.phase = (int)(E.step & 1);
  mm.t_base = member_t;
  mm.e_base = E.step;
  mm.avg_start = E.step;
  mm.initialized = true;
  mm.d.has_ref = 0;  // a new state has no overlap reference yet
  mm.ref_time = -1;
}

int zero_member_slots(Engine& E, int i) {
  const Member& mm = E.m[i];
  HIPCK(E, hipMemsetAsync(mm.d.wave_wall, 0, wall_slots(&mm.p) * 2 * sizeof(double), E.stream));
  HIPCK(E, hipMemsetAsync(mm.d.flag, 0, sizeof(int), E.stream));
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
  mm.d.local[0] = E.mom ? 1 : 0;  // buf[0] becomes the current buffer
  mm.d.local[1] = 0;
  int rc = upload_descs(E);
  if (rc != LB_OK) return rc;
  if (E.mom)
    HIPCK(E, lbk::launch_moment_init(mm.d.g, mm.d.c, d_rho, d_u, mm.d.buf[0], E.stream));
  else
    HIPCK(E, lbk::launch_init(mm.d.g, mm.d.c, E.fp64, E.walls, d_rho, d_u, mm.d.buf[0],
                              mm.d.wall[0], E.stream));
  rc = zero_member_slots(E, i);
  if (rc != LB_OK) return rc;
  HIPCK(E, hipStreamSynchronize(E.stream));
  return LB_OK;
}

// Capture two consecutive steps starting at the given parity into a graph.
// Capture runs on a private non-blocking stream (the caller's stream may be
// the null stream, which cannot be captured); replays go to the caller's
// stream.  The graph holds the two kernel nodes only.
hipError_t step_launch(const Engine& E, const lbk::LaunchArgs& a, hipStream_t st,
                       bool allow_group) {
  if (E.mom) return lbk::launch_moment_step(a, E.variant, st);
  if (split_kernel(E)) {
    lbk::StepVariant v = E.variant;
    if (!allow_group) v.group = 1;
    return lbk::launch_split_step(a, E.fp64, E.walls, v, st);
  }
  return lbk::launch_step(a, E.fp64, E.walls, E.variant, st);
}

hipError_t observe_launch(const Engine& E, const lbk::LaunchArgs& a, hipStream_t st) {
  return E.mom ? lbk::launch_moment_observe(a, st) : lbk::launch_observe(a, E.fp64, E.walls, st);
}

int capture_pair(Engine& E, int parity) {
  if (!E.capture_stream) HIPCK(E, hipStreamCreateWithFlags(&E.capture_stream, hipStreamNonBlocking));
  HIPCK(E, hipStreamBeginCapture(E.capture_stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < 2; ++k) {
    const hipError_t le = step_launch(E, launch_args(E, (parity + k) & 1), E.capture_stream, E.group_ok);
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

void fill_obs(const Engine& E, int i, const double* h, int flag, lb_obs* out) {
  const Member& mm = E.m[i];
  std::memset(out, 0, sizeof(*out));
  out->step = member_time(E, i);
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
  out->u_mode = h[7] * 2.0 / ((double)mm.d.g.nx * (double)mm.d.g.ny);
  out->i_ab = h[8];
  out->phi_overlap = h[9];
  out->phi_ref_sq = h[10];
  out->ref_step = mm.ref_time;
  out->flags = flag;
}

}  // namespace

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != dev) (void)hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard() {
  int cur = -1;
  if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

std::string& create_error() {
  thread_local std::string msg;
  return msg;
}

const char* handle_error(const std::string* handle_err) {
  if (handle_err) return handle_err->c_str();
  return create_error().empty() ? "null handle" : create_error().c_str();
}

int validate(const lb_params* p, std::string* why) {
  auto bad = [&](const char* msg) {
    if (why) *why = msg;
    return LB_E_INVAL;
  };
  if (!p) return bad("params is NULL");
  if (p->nx < 5 || p->ny < 5) return bad("nx and ny must be >= 5");
  if ((long long)p->nx * p->ny > (1LL << 30)) return bad("lattice larger than 2^30 sites");
  if (p->boundary != LB_PERIODIC && p->boundary != LB_COUETTE_Y) return bad("unknown boundary");
  if (p->precision != LB_FP64 && p->precision != LB_FP32_DEV && p->precision != LB_FP32_MOM)
    return bad("unknown precision");
  if (p->precision == LB_FP32_MOM) {
    if (p->tau[0] != 1.0 || p->tau[1] != 1.0) return bad("moment storage needs tau_A = tau_B = 1");
    if (p->boundary != LB_PERIODIC) return bad("moment storage supports periodic boundaries only");
  }
  {
    // The kernels address a site within its row by a 32-bit byte offset and
    // the wall links by a 32-bit index (12 nx of them): both must stay below
    // 2^31.
    const long long pitch = ((long long)p->nx + lbk::kWave - 1) / lbk::kWave * lbk::kWave;
    const long long row_bytes =
        pitch * (p->precision == LB_FP32_MOM ? 6 * 4 : 18 * (p->precision == LB_FP64 ? 8 : 4));
    if (row_bytes >= (1LL << 31)) return bad("lattice row too long for 32-bit in-row offsets");
    if (12LL * p->nx >= (1LL << 31)) return bad("nx too large for 32-bit wall-link indices");
  }
  for (int s = 0; s < 2; ++s) {
    if (!is_finite(p->tau[s]) || !(p->tau[s] > 0.5)) return bad("tau must be > 1/2");
    if (!is_finite(p->G_a[s]) || !is_finite(p->G_r[s])) return bad("couplings must be finite");
    if (!is_finite(p->rho_ref[s])) return bad("rho_ref must be finite");
  }
  if (!is_finite(p->rho0) || !(p->rho0 > 0)) return bad("rho0 must be > 0");
  if (!is_finite(p->G_AB)) return bad("G_AB must be finite");
  if (!is_finite(p->u_wall)) return bad("u_wall must be finite");
  if (!is_finite(p->body_force)) return bad("body_force must be finite");
  if (!is_finite(p->body_force_x)) return bad("body_force_x must be finite");
  return LB_OK;
}

size_t member_region_bytes(const lb_params* p) {
  const lbk::Geometry g = make_geometry(p, 0);
  const size_t pop = align_up((size_t)g.row_elems * (size_t)g.ny * elem_size(p));
  const size_t wall = align_up(12ull * (size_t)p->nx * elem_size(p));
  return 2 * pop + 2 * wall + align_up(red_slots(p) * lbk::kNRed * sizeof(double)) +
         align_up(wall_slots(p) * 2 * sizeof(double)) +
         align_up((size_t)p->nx * (size_t)p->ny * sizeof(double)) + kAlign;
}

size_t engine_static_bytes(const lb_params* ps, int n) {
  int tiles = 0;
  size_t regions = 0;
  for (int i = 0; i < n; ++i) {
    tiles += max_tiles_of(&ps[i]);
    regions += member_region_bytes(&ps[i]);
  }
  return shared_bytes(n, tiles) + regions;
}

int engine_create_static(Engine& E, const lb_params* ps, int n, void* buffer, size_t buffer_bytes,
                         hipStream_t stream) {
  E.fp64 = ps[0].precision == LB_FP64;
  E.mom = ps[0].precision == LB_FP32_MOM;
  E.walls = ps[0].boundary == LB_COUETTE_Y;
  E.stream = stream;
  if (hipGetDevice(&E.device) != hipSuccess) return E.fail(LB_E_DEVICE, "no HIP device");
  const size_t total = engine_static_bytes(ps, n);
  if (buffer) {
    if (buffer_bytes < total || ((uintptr_t)buffer % kAlign) != 0)
      return E.fail(LB_E_NOMEM, "device_buffer too small or not 256-byte aligned");
    E.block = (char*)buffer;
    E.owns_block = false;
  } else {
    void* b = nullptr;
    if (hipMalloc(&b, total) != hipSuccess) {
      (void)hipGetLastError();
      return E.fail(LB_E_NOMEM, "hipMalloc of the workspace failed");
    }
    E.block = (char*)b;
    E.owns_block = true;
  }
  E.bytes = total;
  int tiles = 0;
  for (int i = 0; i < n; ++i) tiles += max_tiles_of(&ps[i]);
  carve_shared(E, E.block, n, tiles);
  E.owns_shared = false;
  char* q = E.block + shared_bytes(n, tiles);
  for (int i = 0; i < n; ++i) {
    E.m.push_back(make_member(&ps[i], q, false, i));
    q += E.m.back().region_bytes;
  }
  choose_default_variant(E);
  HIPCK(E, hipMemsetAsync(E.block, 0, total, E.stream));
  const int rc = retile(E);
  if (rc != LB_OK) return rc;
  HIPCK(E, hipStreamSynchronize(E.stream));
  return LB_OK;
}

int engine_create_dynamic(Engine& E, bool fp64, bool walls, hipStream_t stream) {
  E.fp64 = fp64;
  E.walls = walls;
  E.stream = stream;
  E.owns_shared = true;
  if (hipGetDevice(&E.device) != hipSuccess) return E.fail(LB_E_DEVICE, "no HIP device");
  choose_default_variant(E);
  return reserve_shared(E, 16, 4096);
}

int engine_add(Engine& E, const lb_params* p, int64_t tag, int* index) {
  std::string why;
  if (validate(p, &why) != LB_OK) return E.fail(LB_E_INVAL, why);
  if ((p->precision == LB_FP64) != E.fp64 || (p->precision == LB_FP32_MOM) != E.mom ||
      (p->boundary == LB_COUETTE_Y) != E.walls)
    return E.fail(LB_E_INVAL, "lattice precision / boundary differ from the engine's");
  DeviceGuard dg(E.device);
  const size_t rb = member_region_bytes(p);
  void* r = nullptr;
  if (hipMalloc(&r, rb) != hipSuccess) {
    (void)hipGetLastError();
    return E.fail(LB_E_NOMEM, "hipMalloc of a lattice failed");
  }
  HIPCK(E, hipMemsetAsync(r, 0, rb, E.stream));
  E.m.push_back(make_member(p, (char*)r, true, tag));
  E.bytes += rb;
  const int rc = retile(E);
  if (rc != LB_OK) {
    (void)hipStreamSynchronize(E.stream);
    (void)hipFree(r);
    E.bytes -= rb;
    E.m.pop_back();
    return rc;
  }
  if (index) *index = (int)E.m.size() - 1;
  return LB_OK;
}

int engine_remove(Engine& E, int index) {
  if (index < 0 || index >= (int)E.m.size()) return E.fail(LB_E_INVAL, "lattice index out of range");
  DeviceGuard dg(E.device);
  HIPCK(E, hipStreamSynchronize(E.stream));
  if (E.m[index].owns_region) {
    (void)hipFree(E.m[index].region);
    E.bytes -= E.m[index].region_bytes;
  }
  E.m.erase(E.m.begin() + index);
  return retile(E);
}

void engine_destroy(Engine& E) {
  DeviceGuard dg(E.device);
  (void)hipStreamSynchronize(E.stream);
  drop_graphs(E);
  if (E.capture_stream) (void)hipStreamDestroy(E.capture_stream);
  E.capture_stream = nullptr;
  for (auto& mm : E.m)
    if (mm.owns_region && mm.region) (void)hipFree(mm.region);
  E.m.clear();
  if (E.owns_shared && E.shared) (void)hipFree(E.shared);
  if (E.owns_block && E.block) (void)hipFree(E.block);
  if (E.sub) (void)hipFree(E.sub);
  E.shared = nullptr;
  E.block = nullptr;
  E.sub = nullptr;
  E.sub_bytes = 0;
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

int engine_step(Engine& E, int64_t n) {
  if (n < 0) return E.fail(LB_E_INVAL, "n must be >= 0");
  if (E.m.empty()) return n == 0 ? LB_OK : E.fail(LB_E_STATE, "no lattices to step");
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
    HIPCK(E, step_launch(E, launch_args(E, (int)(E.step & 1)), E.stream, E.group_ok));
    ++E.step;
  }
  // every buffer written by a moment step is in pull form; the kernels
  // cleared their destinations' flags, keep the host copy in step
  if (E.mom && n > 0)
    for (auto& mm : E.m) mm.d.local[0] = mm.d.local[1] = 0;
  return LB_OK;
}

// Each launch runs over the selected members' tiles only, through a
// descriptor array and tile map of their own (copies of the members'
// records, tiled as if the selected members were the whole engine, tile
// bases renumbered from 0), so the kernels are those of a whole-engine
// step.  A member left out of n steps keeps its buffers; its
// buffer phase and time bases move by n, so that the engine's parity still
// selects its current buffer and its time and wall averages count only its
// own steps.
int engine_step_subset(Engine& E, const std::vector<int>& sel, int64_t n) {
  if (n < 0) return E.fail(LB_E_INVAL, "n must be >= 0");
  if (E.mom) return E.fail(LB_E_INVAL, "subset steps need population storage");
  std::vector<char> in(E.m.size(), 0);
  for (int i : sel) {
    if (i < 0 || i >= (int)E.m.size() || in[i])
      return E.fail(LB_E_INVAL, "subset indices out of range or repeated");
    if (!E.m[i].initialized) return E.fail(LB_E_STATE, "step before every lattice is initialized");
    in[i] = 1;
  }
  if (sel.empty() || n == 0) return LB_OK;
  if (sel.size() == E.m.size()) return engine_step(E, n);
  DeviceGuard dg(E.device);
  const auto geo = geometries(E, E.seg_h, &sel);
  std::vector<lbk::LatticeDesc> d;
  std::vector<int> map;
  int base = 0;
  for (int k = 0; k < (int)sel.size(); ++k) {
    lbk::LatticeDesc x = E.m[sel[k]].d;
    x.g = geo[k];
    x.tile_base = base;
    base += x.g.ntiles;
    map.insert(map.end(), x.g.ntiles, k);
    d.push_back(x);
  }
  const size_t bd = align_up(d.size() * sizeof(lbk::LatticeDesc));
  const size_t need = bd + align_up(map.size() * sizeof(int));
  if (E.sub_bytes < need) {
    HIPCK(E, hipStreamSynchronize(E.stream));  // the old tables may still be read
    if (E.sub) (void)hipFree(E.sub);
    E.bytes -= E.sub_bytes;
    E.sub = nullptr;
    E.sub_bytes = 0;
    void* b = nullptr;
    if (hipMalloc(&b, need) != hipSuccess) {
      (void)hipGetLastError();
      return E.fail(LB_E_NOMEM, "hipMalloc of the subset tables failed");
    }
    E.sub = (char*)b;
    E.sub_bytes = need;
    E.bytes += need;
  }
  HIPCK(E, hipMemcpyAsync(E.sub, d.data(), d.size() * sizeof(lbk::LatticeDesc),
                          hipMemcpyHostToDevice, E.stream));
  HIPCK(E, hipMemcpyAsync(E.sub + bd, map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice,
                          E.stream));
  HIPCK(E, hipStreamSynchronize(E.stream));  // the host vectors die at return
  lbk::LaunchArgs a{};
  a.descs = (const lbk::LatticeDesc*)E.sub;
  a.tile_lattice = (const int*)(E.sub + bd);
  a.ntiles = base;
  a.tiles_per_xcd = (base + 7) / 8;
  a.accumulate_wall = E.walls ? 1 : 0;
  const bool grp = group_allowed(E, &sel);
  for (int64_t k = 0; k < n; ++k) {
    a.parity = (int)(E.step & 1);
    HIPCK(E, step_launch(E, a, E.stream, grp));
    ++E.step;
  }
  for (size_t i = 0; i < E.m.size(); ++i) {
    if (in[i]) continue;
    Member& mm = E.m[i];
    mm.d.phase ^= (int)(n & 1);
    mm.e_base += n;
    mm.avg_start += n;
  }
  return upload_descs(E);
}

int engine_observables(Engine& E, lb_obs* out /*[n]*/) {
  for (auto& mm : E.m)
    if (!mm.initialized) return E.fail(LB_E_STATE, "observables before every lattice is initialized");
  if (E.m.empty()) return LB_OK;
  DeviceGuard dg(E.device);
  const int n = (int)E.m.size();
  HIPCK(E, observe_launch(E, launch_args(E, (int)(E.step & 1)), E.stream));
  long long max_slots = 0;
  for (auto& mm : E.m) max_slots = std::max(max_slots, (long long)mm.d.g.ny * mm.d.g.nstrips);
  HIPCK(E, lbk::launch_reduce_lattices(E.d_descs, n, 0, E.red_out, 16, max_slots, E.stream));
  HIPCK(E, lbk::launch_reduce_lattices(E.d_descs, n, 1, E.red_out + lbk::kNRed, 16, 0, E.stream));
  std::vector<double> h((size_t)n * 16);
  HIPCK(E, hipMemcpyAsync(h.data(), E.red_out, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                          E.stream));
  std::vector<int> flags;
  const int rc = read_flags(E, &flags);
  if (flags.size() != (size_t)n) return rc;
  for (int i = 0; i < n; ++i) fill_obs(E, i, h.data() + (size_t)i * 16, flags[i], out + i);
  return rc;
}

int engine_member_observables(Engine& E, int i, lb_obs* out) {
  if (i < 0 || i >= (int)E.m.size()) return E.fail(LB_E_INVAL, "lattice index out of range");
  if (!E.m[i].initialized) return E.fail(LB_E_STATE, "observables before lb_init");
  DeviceGuard dg(E.device);
  HIPCK(E, observe_launch(E, member_args(E, i), E.stream));
  double* row = E.red_out + (size_t)i * 16;
  HIPCK(E, lbk::launch_reduce_lattices(E.d_descs + i, 1, 0, row, 16,
                                       (long long)E.m[i].d.g.ny * E.m[i].d.g.nstrips, E.stream));
  HIPCK(E, lbk::launch_reduce_lattices(E.d_descs + i, 1, 1, row + lbk::kNRed, 16, 0, E.stream));
  double h[16];
  int flag = 0;
  HIPCK(E, hipMemcpyAsync(h, row, sizeof(h), hipMemcpyDeviceToHost, E.stream));
  HIPCK(E, hipMemcpyAsync(&flag, E.m[i].d.flag, sizeof(int), hipMemcpyDeviceToHost, E.stream));
  HIPCK(E, hipStreamSynchronize(E.stream));
  fill_obs(E, i, h, flag, out);
  if (flag & 3) return flag_status(E, flag);
  return LB_OK;
}

int engine_fields_staged(Engine& E, int i, double* staging, double* rho_a, double* rho_b,
                         double* u, double* u_phys) {
  if (i < 0 || i >= (int)E.m.size()) return E.fail(LB_E_INVAL, "lattice index out of range");
  if (!E.m[i].initialized) return E.fail(LB_E_STATE, "fields before lb_init");
  DeviceGuard dg(E.device);
  const size_t n = (size_t)E.m[i].d.g.nx * E.m[i].d.g.ny, nb = n * sizeof(double);
  double* d = staging;
  lbk::LaunchArgs a = member_args(E, i);
  a.fields = d;  // every site of all six fields is written
  HIPCK(E, observe_launch(E, a, E.stream));
  if (rho_a) HIPCK(E, hipMemcpyAsync(rho_a, d, nb, hipMemcpyDeviceToHost, E.stream));
  if (rho_b) HIPCK(E, hipMemcpyAsync(rho_b, d + n, nb, hipMemcpyDeviceToHost, E.stream));
  if (u) HIPCK(E, hipMemcpyAsync(u, d + 2 * n, 2 * nb, hipMemcpyDeviceToHost, E.stream));
  if (u_phys) HIPCK(E, hipMemcpyAsync(u_phys, d + 4 * n, 2 * nb, hipMemcpyDeviceToHost, E.stream));
  // the member's own flag word, read without host containers
  int flag = 0;
  HIPCK(E, hipMemcpyAsync(&flag, E.m[i].d.flag, sizeof(int), hipMemcpyDeviceToHost, E.stream));
  HIPCK(E, hipStreamSynchronize(E.stream));
  if (flag & 3) return flag_status(E, flag);
  return LB_OK;
}

int engine_fields(Engine& E, int i, double* rho_a, double* rho_b, double* u, double* u_phys) {
  if (i < 0 || i >= (int)E.m.size()) return E.fail(LB_E_INVAL, "lattice index out of range");
  if (!E.m[i].initialized) return E.fail(LB_E_STATE, "fields before lb_init");
  DeviceGuard dg(E.device);
  const size_t n = (size_t)E.m[i].d.g.nx * E.m[i].d.g.ny, nb = n * sizeof(double);
  DevTmp t;
  HIPCK(E, hipMalloc(&t.p, 6 * nb));
  const int rc = engine_fields_staged(E, i, (double*)t.p, rho_a, rho_b, u, u_phys);
  if (rc != LB_OK) return rc;
  return read_flags(E, nullptr);
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
  HIPCK(E, observe_launch(E, a, E.stream));
  HIPCK(E, hipMemcpyAsync(f, t.p, nb, hipMemcpyDeviceToHost, E.stream));
  return read_flags(E, nullptr);
}

int engine_set_pops(Engine& E, int i, const double* f, int64_t member_t) {
  if (i < 0 || i >= (int)E.m.size() || !f) return E.fail(LB_E_INVAL, "bad lattice index or NULL f");
  if (E.mom) return E.fail(LB_E_INVAL, "moment storage cannot hold arbitrary populations");
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
  for (auto& mm : E.m) {
    HIPCK(E, hipMemsetAsync(mm.d.wave_wall, 0, wall_slots(&mm.p) * 2 * sizeof(double), E.stream));
    mm.avg_start = E.step;
  }
  return LB_OK;
}

int engine_set_reference(Engine& E) {
  for (auto& mm : E.m)
    if (!mm.initialized) return E.fail(LB_E_STATE, "reference before every lattice is initialized");
  if (E.m.empty()) return LB_OK;
  DeviceGuard dg(E.device);
  lbk::LaunchArgs a = launch_args(E, (int)(E.step & 1));
  a.write_ref = 1;
  HIPCK(E, observe_launch(E, a, E.stream));
  for (int i = 0; i < (int)E.m.size(); ++i) {
    E.m[i].d.has_ref = 1;
    E.m[i].ref_time = member_time(E, i);
  }
  drop_graphs(E);
  const int rc = upload_descs(E);  // synchronizes
  if (rc != LB_OK) return rc;
  return read_flags(E, nullptr);
}

int engine_sync(Engine& E) {
  DeviceGuard dg(E.device);
  return read_flags(E, nullptr);
}

int engine_set_variant(Engine& E, int32_t prefetch, int32_t stream_stores, int32_t use_graph,
                       int32_t group) {
  if (group >= 0 && group != 1 && group != lbk::kGroupTiles)
    return E.fail(LB_E_INVAL, "tiles_per_group must be 1 or 4");
  if (prefetch >= 0) E.variant.prefetch = std::min(prefetch, 2);
  if (stream_stores >= 0) E.variant.stream_stores = stream_stores ? 1 : 0;
  if (group >= 0) E.variant.group = group;
  if (prefetch >= 0 || stream_stores >= 0 || group >= 0) E.variant_forced = true;
  if (use_graph >= 0) E.use_graph = use_graph != 0;
  drop_graphs(E);
  return LB_OK;
}

int engine_regrid(Engine& E, int seg_h) {
  DeviceGuard dg(E.device);
  E.seg_h = seg_h >= 4 ? seg_h : 0;
  return retile(E);  // reduction slots do not follow the tiles: averages carry on
}

namespace {

struct Events {
  hipEvent_t e[2] = {nullptr, nullptr};
  ~Events() {
    for (auto ev : e)
      if (ev) (void)hipEventDestroy(ev);
  }
};

// Per-member segment counts: two candidates that give the same counts are
// the same launch.
std::vector<int> seg_signature(const Engine& E, int seg_h) {
  std::vector<int> s;
  for (const auto& g : geometries(E, seg_h)) s.push_back(g.nsegs);
  return s;
}

}  // namespace

// Candidates: the default shape and forced segment heights 4..256 rows with
// the current variant, then the six prefetch-depth (0..2) / streaming-store
// variants at the best height.  Each candidate runs 2 untimed steps
// (capturing its graph when graphs are on), then `steps` steps timed with
// HIP events on the engine's stream.  The current shape first steps untimed
// for about 30 ms: after idle or other work the GPU runs a streaming kernel
// a few per cent slower for its first tens of milliseconds, and a candidate
// timed in that window would lose to later ones that are no faster.  Every
// candidate is timed twice, in two passes, and keeps its better time; the
// default height and the current variant are kept unless another candidate
// is more than 1% faster.  The chosen shape then steps untimed for about
// 20 ms before the state is restored.  The members' whole device regions (populations, wall
// links, reduction slots, flag) are copied aside first and copied back at the
// end, so the state, the wall-stress averages included, is unchanged.
namespace {

// Autotuner results, by library ABI, GPU architecture, storage, boundary
// type, graph use and the members' shapes: kept for the life of the
// process and, after lb_set_tune_cache, in a text file (one result per
// line: key, segment height, prefetch, streaming stores, tiles per group,
// us per step).  A
// result only selects among launch shapes that give the same numbers bit
// for bit, so a stale one costs speed, never correctness.
struct TuneResult {
  int seg_h;
  lbk::StepVariant v;
  double us;
};
std::mutex g_tune_mu;
std::map<std::string, TuneResult> g_tune_cache;
std::string g_tune_path;  // "" = not persisted

std::string tune_key(const Engine& E) {
  hipDeviceProp_t prop{};
  std::string arch = hipGetDeviceProperties(&prop, E.device) == hipSuccess ? prop.gcnArchName : "?";
  // the architecture name may carry feature flags (gfx950:sramecc+:xnack-)
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  std::vector<std::pair<int, int>> shapes;
  for (const auto& mm : E.m) shapes.emplace_back(mm.p.nx, mm.p.ny);
  std::sort(shapes.begin(), shapes.end());
  std::string k = "abi" + std::to_string(LB_ABI_VERSION) + "/" + arch +
                  (E.fp64 ? "/f64" : (E.mom ? "/f32mom" : "/f32dev")) +
                  (E.walls ? "/walls" : "/periodic") + (E.use_graph ? "/graph" : "/launch");
  for (auto& s : shapes) k += "/" + std::to_string(s.first) + "x" + std::to_string(s.second);
  return k;
}

// Caller holds g_tune_mu.  Lines that do not parse or hold values out of
// range are skipped.
void load_tune_file(const std::string& path) {
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string key;
    TuneResult r{};
    if (!(ls >> key >> r.seg_h >> r.v.prefetch >> r.v.stream_stores >> r.v.group >> r.us)) continue;
    if (r.seg_h < 0 || r.v.prefetch < 0 || r.v.prefetch > 2 || (r.v.stream_stores & ~1) ||
        (r.v.group != 1 && r.v.group != lbk::kGroupTiles) || !(r.us > 0.0))
      continue;
    g_tune_cache[key] = r;
  }
}

// Caller holds g_tune_mu.  Writes the whole cache next to the file, under
// a name of this process's own, and renames it into place, so a reader never
// sees half a file and processes saving at once do not mix their lines (the
// last rename wins).
bool save_tune_file(const std::string& path) {
  const std::string tmp = path + ".tmp." + std::to_string((long long)getpid());
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return false;
    out.precision(17);  // times round-trip
    for (const auto& kv : g_tune_cache)
      out << kv.first << ' ' << kv.second.seg_h << ' ' << kv.second.v.prefetch << ' '
          << kv.second.v.stream_stores << ' ' << kv.second.v.group << ' ' << kv.second.us << '\n';
    if (!out) return false;
  }
  return std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

int engine_autotune(Engine& E, int steps, double* us_per_step) {
  if (steps < 0) return E.fail(LB_E_INVAL, "autotune needs steps >= 0");
  if (E.m.empty()) return E.fail(LB_E_STATE, "no lattices to tune");
  for (auto& mm : E.m)
    if (!mm.initialized) return E.fail(LB_E_STATE, "autotune before every lattice is initialized");
  const std::string key = tune_key(E);
  if (steps == 0) {
    TuneResult hit{};
    bool found = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) hit = it->second, found = true;
    }
    if (found) {
      if (seg_signature(E, hit.seg_h) != seg_signature(E, E.seg_h)) {
        const int rc = engine_regrid(E, hit.seg_h);
        if (rc != LB_OK) return rc;
      } else {
        E.seg_h = hit.seg_h;
      }
      E.variant = hit.v;
      E.variant_forced = true;
      drop_graphs(E);
      if (us_per_step) *us_per_step = hit.us;
      return LB_OK;
    }
    steps = 16;
  }
  steps = std::max(steps, 2);
  steps += steps & 1;  // whole two-step graphs
  DeviceGuard dg(E.device);
  size_t total = 0;
  for (auto& mm : E.m) total += mm.region_bytes;
  DevTmp save;
  if (hipMalloc(&save.p, total) != hipSuccess) {
    (void)hipGetLastError();
    return E.fail(LB_E_NOMEM, "no device memory for the autotuner's copy of the state");
  }
  size_t off = 0;
  for (auto& mm : E.m) {
    HIPCK(E, hipMemcpyAsync((char*)save.p + off, mm.region, mm.region_bytes, hipMemcpyDeviceToDevice,
                            E.stream));
    off += mm.region_bytes;
  }
  const int64_t step0 = E.step;
  const int seg0 = E.seg_h;
  std::vector<std::array<int, 2>> local0;  // buffer forms of the moment storage
  for (auto& mm : E.m) local0.push_back({mm.d.local[0], mm.d.local[1]});
  Events ev;
  HIPCK(E, hipEventCreate(&ev.e[0]));
  HIPCK(E, hipEventCreate(&ev.e[1]));

  const bool forced0 = E.variant_forced;
  E.variant_forced = true;  // retile must keep each candidate's variant
  auto run = [&](int seg_h, lbk::StepVariant v, double* us) -> int {
    E.variant = v;
    E.seg_h = seg_h;
    int rc = retile(E);  // sets the geometries, drops the graphs
    if (rc != LB_OK) return rc;
    rc = engine_step(E, 2);
    if (rc != LB_OK) return rc;
    HIPCK(E, hipEventRecord(ev.e[0], E.stream));
    rc = engine_step(E, steps);
    if (rc != LB_OK) return rc;
    HIPCK(E, hipEventRecord(ev.e[1], E.stream));
    HIPCK(E, hipEventSynchronize(ev.e[1]));
    float ms = 0.f;
    HIPCK(E, hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    *us = 1e3 * (double)ms / steps;
    return LB_OK;
  };

  int ny_max = 0;
  for (auto& mm : E.m) ny_max = std::max(ny_max, mm.p.ny);
  std::vector<int> heights = {0};
  for (int h : {4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256})
    if (h < ny_max + 8) heights.push_back(h);
  std::vector<std::vector<int>> seen;
  std::vector<int> hs;  // candidate heights, one per distinct launch; hs[0] = 0, the default
  for (int h : heights) {
    const auto sig = seg_signature(E, h);
    if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
    seen.push_back(sig);
    hs.push_back(h);
  }
  int best_h = seg0;
  const lbk::StepVariant v0 = E.variant;
  lbk::StepVariant best_v = v0;
  double best = 1e300;
  int rc = LB_OK;
  // untimed steps of the current shape for about `ms` milliseconds (at most
  // 16 rounds of `steps` steps)
  auto hold = [&](int ms) {
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < 16 && rc == LB_OK; ++i) {
      rc = engine_step(E, steps);
      if (rc == LB_OK && hipStreamSynchronize(E.stream) != hipSuccess)
        rc = E.fail(LB_E_DEVICE, "autotune: stream synchronize failed");
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(ms)) break;
    }
  };
  hold(30);  // settle
  // keeps candidate 0 unless another is more than 1% faster
  auto pick = [](const std::vector<double>& t) {
    size_t b = 0;
    for (size_t c = 1; c < t.size(); ++c)
      if (t[c] < t[b]) b = c;
    return (b != 0 && !(t[b] < 0.99 * t[0])) ? size_t(0) : b;
  };
  if (rc == LB_OK) {
    std::vector<double> t(hs.size(), 1e300);
    for (int pass = 0; pass < 2 && rc == LB_OK; ++pass)
      for (size_t c = 0; c < hs.size() && rc == LB_OK; ++c) {
        double us = 0.0;
        rc = run(hs[c], v0, &us);
        if (rc == LB_OK) t[c] = std::min(t[c], us);
      }
    if (rc == LB_OK) {
      const size_t b = pick(t);
      best_h = hs[b];
      best = t[b];
    }
  }
  if (rc == LB_OK) {
    std::vector<lbk::StepVariant> vs = {v0};
    std::vector<double> t = {best};
    const int npf = E.mom ? 1 : 3;  // the moment kernel has no prefetch variants
    for (int pf = 0; pf < npf; ++pf)
      for (int nt = 0; nt < 2; ++nt)
        if (!(pf == v0.prefetch && nt == v0.stream_stores)) {
          vs.push_back(lbk::StepVariant{pf, nt, v0.group});
          t.push_back(1e300);
        }
    for (int pass = 0; pass < 2 && rc == LB_OK; ++pass)
      for (size_t c = 1; c < vs.size() && rc == LB_OK; ++c) {
        double us = 0.0;
        rc = run(best_h, vs[c], &us);
        if (rc == LB_OK) t[c] = std::min(t[c], us);
      }
    if (rc == LB_OK) {
      const size_t b = pick(t);
      best_v = vs[b];
      best = t[b];
    }
  }
  if (rc == LB_OK && E.group_ok) {
    // tiles per workgroup at the best height and variant
    lbk::StepVariant other = best_v;
    other.group = best_v.group == 1 ? lbk::kGroupTiles : 1;
    std::vector<double> t = {best, 1e300};
    for (int pass = 0; pass < 2 && rc == LB_OK; ++pass) {
      double us = 0.0;
      rc = run(best_h, other, &us);
      if (rc == LB_OK) t[1] = std::min(t[1], us);
    }
    if (rc == LB_OK && pick(t) == 1) {
      best_v = other;
      best = t[1];
    }
  }
  // The chosen shape runs last, for about 20 ms, so that steps after the
  // tuner start from the state that shape runs in rather than from the
  // last candidate's.
  if (rc == LB_OK) {
    E.variant = best_v;
    E.seg_h = best_h;
    rc = retile(E);
    if (rc == LB_OK) hold(20);
  }
  // restore the state under the chosen shape (or the original one on error)
  if (rc != LB_OK) best_h = seg0;
  E.variant = best_v;
  E.variant_forced = true;
  E.seg_h = best_h;
  for (size_t i = 0; i < E.m.size(); ++i) {
    E.m[i].d.local[0] = local0[i][0];
    E.m[i].d.local[1] = local0[i][1];
  }
  const int rc2 = retile(E);  // uploads the descriptors with the restored forms
  off = 0;
  for (auto& mm : E.m) {
    HIPCK(E, hipMemcpyAsync(mm.region, (char*)save.p + off, mm.region_bytes, hipMemcpyDeviceToDevice,
                            E.stream));
    off += mm.region_bytes;
  }
  HIPCK(E, hipStreamSynchronize(E.stream));
  E.step = step0;
  if (rc != LB_OK) {
    E.variant_forced = forced0;
    return rc;
  }
  if (rc2 != LB_OK) return rc2;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = TuneResult{best_h, best_v, best};
    if (!g_tune_path.empty() && !save_tune_file(g_tune_path))
      E.err = "autotune result kept, but writing " + g_tune_path + " failed";
  }
  if (us_per_step) *us_per_step = best;
  return LB_OK;
}

int set_tune_cache(const char* path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!path || !*path) {
    g_tune_path.clear();
    return LB_OK;
  }
  g_tune_path = path;
  load_tune_file(g_tune_path);
  return save_tune_file(g_tune_path) ? LB_OK : LB_E_INVAL;
}

void engine_info(const Engine& E, lb_launch_info* out) {
  std::memset(out, 0, sizeof(*out));
  const int grp = (split_kernel(E) && E.group_ok) ? E.variant.group : 1;
  out->ntiles = E.ntiles;
  out->grid_blocks = 8 * ((E.ntiles / grp + 7) / 8);
  out->block_threads = split_kernel(E) ? 2 * lbk::kWave * grp : lbk::kWave;
  out->tiles_per_group = grp;
  out->workspace_bytes = E.bytes;
  size_t pb = 0;
  for (auto& mm : E.m) pb += mm.pop_bytes;
  out->population_bytes = pb;
  if (!E.m.empty()) {
    const auto& g = E.m[0].d.g;
    out->nstrips = g.nstrips;
    out->nsegs = g.nsegs;
    out->pitch = g.pitch;
    out->seg_h = g.seg_h;
  }
  out->prefetch = E.variant.prefetch;
  out->stream_stores = E.variant.stream_stores;
  out->use_graph = E.use_graph ? 1 : 0;
}

int64_t member_time(const Engine& E, int i) {
  const Member& mm = E.m[i];
  return mm.t_base + (E.step - mm.e_base);
}

int member_index(const Engine& E, int64_t tag) {
  for (int i = 0; i < (int)E.m.size(); ++i)
    if (E.m[i].tag == tag) return i;
  return -1;
}

}  // namespace lbe
