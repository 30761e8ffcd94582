// Internal engine shared by the C ABI of single lattices, batches and the
// serving pool (lb_runtime.hip, lb_pool.hip).  Not installed.
//
// An Engine is a set of lattices of one precision and boundary type that
// advance together: each time step is one kernel launch over the tiles of
// all member lattices.  Members can be added and removed between steps
// (the pool does this as jobs arrive and finish).
#pragma once

#include "lb.h"
#include "lb_internal.h"

#include <cstdint>
#include <string>
#include <vector>

namespace lbe {

// One lattice of an engine (host view; pointers are device addresses).
// Its device region holds, in order: two population buffers, two wall-link
// buffers, its per-tile reduction slots, its wall accumulators, its
// reference order parameter (FP64 per site) and its flag word.
struct Member {
  lb_params p{};
  lbk::LatticeDesc d{};
  size_t pop_bytes = 0, wall_bytes = 0, region_bytes = 0;
  int max_tiles = 0;           // slot capacity (any segment height >= 4)
  char* region = nullptr;
  bool owns_region = false;    // allocated by the engine for this member alone
  bool initialized = false;
  int64_t t_base = 0;          // member time at engine step e_base
  int64_t e_base = 0;
  int64_t avg_start = 0;       // engine step at which the wall averages restarted
  int64_t tag = 0;             // caller's identifier (pool job id)
  int64_t ref_time = -1;       // member time of the overlap reference (-1: none)
};

struct Engine {
  std::vector<Member> m;
  bool fp64 = true, walls = false;
  bool mom = false;           // LB_FP32_MOM storage (moment kernels)
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  int device = 0;
  // shared region: lattice descriptors, tile map, reduction outputs
  char* shared = nullptr;
  bool owns_shared = false;
  int cap_members = 0, cap_tiles = 0;
  lbk::LatticeDesc* d_descs = nullptr;
  int* d_tile_lattice = nullptr;
  double* red_out = nullptr;  // [cap_members][16]
  char* block = nullptr;      // single allocation holding everything (static engines)
  bool owns_block = false;
  size_t bytes = 0;           // device bytes held (static: the block; dynamic: shared + regions)
  int ntiles = 0;
  int64_t step = 0;           // engine step count
  lbk::StepVariant variant{1, 0};
  bool variant_forced = false;  // set by the caller or the autotuner: keep it
  bool group_ok = false;        // every member allows grouped tiles (set by retile)
  int seg_h = 0;              // forced segment height of every member (0: per-lattice default)
  bool use_graph = false;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // two-step graphs by starting parity
  // device tables of the last subset launch (engine_step_subset)
  char* sub = nullptr;
  size_t sub_bytes = 0;
  std::string err;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
};

int validate(const lb_params* p, std::string* why);
// Why the calling thread's last create call failed ("" after a success);
// read through the last-error functions with a null handle.
std::string& create_error();
const char* handle_error(const std::string* handle_err);
size_t member_region_bytes(const lb_params* p);

// Static engine: n lattices carved from one block (caller's buffer or one
// hipMalloc).  engine_static_bytes gives the block size.
size_t engine_static_bytes(const lb_params* ps, int n);
int engine_create_static(Engine& E, const lb_params* ps, int n, void* buffer, size_t buffer_bytes,
                         hipStream_t stream);
// Dynamic engine: starts empty; members get their own allocations.
int engine_create_dynamic(Engine& E, bool fp64, bool walls, hipStream_t stream);
// FP32-deviation lattices (periodic or with walls) step with one wavefront
// per species (k_split); FP64 and the moment storage use their own kernels.
// The choice depends only on the engine's class, never on tuning, so a
// lattice evolves bit for bit alike alone, batched or pooled.
inline bool split_kernel(const Engine& E) { return !E.fp64 && !E.mom; }
int engine_add(Engine& E, const lb_params* p, int64_t tag, int* index);
int engine_remove(Engine& E, int index);
void engine_destroy(Engine& E);

int engine_init(Engine& E, int i, const double* rho_a, const double* rho_b, const double* ux,
                const double* uy);
int engine_init_noise(Engine& E, int i, uint64_t seed, double mean_a, double mean_b, double amp);
int engine_step(Engine& E, int64_t n);
// Advance only the members sel[] (distinct indices) by n steps; the others
// keep their state, time and wall averages as if the engine had not
// stepped.  Population storages only (LB_E_INVAL for the moment storage).
int engine_step_subset(Engine& E, const std::vector<int>& sel, int64_t n);
int engine_observables(Engine& E, lb_obs* out /*[members]*/);
int engine_member_observables(Engine& E, int i, lb_obs* out);
int engine_fields(Engine& E, int i, double* rho_a, double* rho_b, double* u, double* u_phys);
// The same through a caller's device staging buffer of 6 nx ny doubles
// (allocates nothing; checks member i's flag only).
int engine_fields_staged(Engine& E, int i, double* staging, double* rho_a, double* rho_b,
                         double* u, double* u_phys);
int engine_pops(Engine& E, int i, double* f);
int engine_set_pops(Engine& E, int i, const double* f, int64_t member_t);
int engine_reset_averages(Engine& E);
// Store every member's current order parameter rho_A - rho_B as the
// reference of its overlap sums (synchronizes).
int engine_set_reference(Engine& E);
int engine_sync(Engine& E);
int engine_set_variant(Engine& E, int32_t prefetch, int32_t stream_stores, int32_t use_graph,
                       int32_t group);
int engine_regrid(Engine& E, int seg_h);
// Time candidate launch shapes on the engine's own state and keep the
// fastest; the state and step count are restored.  *us_per_step (may be
// NULL) receives the chosen shape's time per step.
int engine_autotune(Engine& E, int steps, double* us_per_step);
// Persist autotuner results in a text file (see lb_set_tune_cache).
int set_tune_cache(const char* path);
void engine_info(const Engine& E, lb_launch_info* out);
int64_t member_time(const Engine& E, int i);
int member_index(const Engine& E, int64_t tag);

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

// Disc-emulsion initial densities (lb_init_spec.hip).
int disc_fields(int nx, int ny, uint64_t seed, double phi, double rmin, double rmax, double in_a,
                double in_b, double out_a, double out_b, std::vector<double>& ra,
                std::vector<double>& rb);

}  // namespace lbe

// Opaque handles of the C ABI: a lattice is an engine of one, a batch an
// engine of n.
struct lb_lattice {
  lbe::Engine e;
};
struct lb_batch {
  lbe::Engine e;
};
