// Internal declarations shared by the kernels (lb_kernels.hip) and the
// runtime behind the C ABI (lb_runtime.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbk {

// One wavefront marches along a strip of kWave lattice columns (plus a
// 2-column stencil ring on each side).  The density / pseudopotential rows
// of the 5-row stencil live in a ring of kRing LDS rows.
constexpr int kWave = 64;
constexpr int kRing = 5;

enum Mode : int { kStep = 0, kObserve = 1 };

// Population layout: lattice row y is (pitch / 64) blocks of 64 sites; a
// block holds the 18 populations (species-major, D2Q9 order) of its sites,
// each as 64 consecutive values.  Element (s, i, y, x) is at
//   y * row_elems + (x / 64) * 18 * 64 + (s * 9 + i) * 64 + x % 64,
// so a wavefront touches one contiguous block per lattice row.
__host__ __device__ inline long long pop_index(long long row_elems, int s, int i, int y, int x) {
  return (long long)y * row_elems + (long long)(x >> 6) * (18 * 64) + (s * 9 + i) * 64 + (x & 63);
}

// Number of FP64 values each wave writes in observe mode: massA, massB,
// momx, momy, momphys_x, momphys_y, pxy, u_mode, i_ab, and the two sums of
// the overlap against the reference order parameter, sum phi_ref phi and
// sum phi_ref^2.
constexpr int kNRed = 11;

// Physical constants of one lattice, in FP64 (converted per kernel).
struct Coefs {
  // Self-force weights per species by class |c|^2 = 1, 2, 4, 5, 8:
  // G^a w + G^r p on the first belt, G^r p on the second (Eq. (2), Table I).
  double kself[2][5];
  // Cross-force weights G_AB / rho0^2 * w for |c|^2 = 1, 2.
  double kcross[2];
  double rho0, inv_rho0;
  double tau[2], omega[2];
  double rho_ref[2];  // deviation references (deviation storage only; FP32-representable)
  double psi_ref[2];  // psi(rho_ref)
  double psi_scale[2];  // rho0 exp(-rho_ref / rho0): psi(rho_ref + d) - psi_ref = -psi_scale expm1(-d / rho0)
  double u_wall;      // +u_wall at the top wall, -u_wall at the bottom
  double g_body;      // shear forcing amplitude: rho_s g_body sin(2 pi y / ny) along x
  double g_uniform;   // uniform body force per unit mass along x: rho_s g_uniform
  double inv_ny2;     // 2 / ny (argument of sinpi for row y)
  // The same constants rounded to FP32 on the host, so FP32 kernels read
  // them straight into scalar registers.
  float f_kself[2][5], f_kcross[2], f_rho0, f_inv_rho0, f_tau[2], f_omega[2], f_rho_ref[2],
      f_psi_ref[2], f_psi_scale[2], f_u_wall, f_g_body, f_g_uniform, f_inv_ny2;
};

struct Geometry {
  int nx, ny, pitch;
  long long row_elems;  // elements of one lattice row: (pitch / 64) blocks x 18 x 64
                        // (x 6 x 64 for moment storage)
  int nstrips, seg_h, nsegs, ntiles;  // tiles = strips x segments, one wavefront each
};

// One lattice as the kernels see it (device memory, one record per lattice
// of a launch; read with scalar loads).
struct LatticeDesc {
  Geometry g;
  Coefs c;
  void* buf[2];   // population buffers (pull layout)
  void* wall[2];  // wall-link buffers
  int* flag;      // bit 0 set when a density is non-finite or <= 0
  double* wave_red;   // observe: kNRed partials per (row, strip) of this lattice
  double* wave_wall;  // step: wall-momentum accumulators (bottom, top) per strip
  double* phi_ref;    // reference order parameter rho_A - rho_B per site [ny][nx] (FP64)
  int has_ref;        // phi_ref holds a reference: observe adds the overlap sums
  int tile_base;  // first tile of this lattice in its launch's tile list
  int phase;      // with launch step parity p the lattice reads buf[p ^ phase]
  int local[2];   // moment storage: buf[k] holds site-local equilibria (t = 0 form)
};

// Arguments of one step / observe launch over a set of lattices that share
// precision and boundary type.
struct LaunchArgs {
  const LatticeDesc* descs;  // device array of the lattices
  const int* tile_lattice;   // device array: lattice of each tile; null = all tiles are lattice 0
  int ntiles;                // tiles in the launch
  int tiles_per_xcd;         // ceil(ntiles / 8): tiles are handed out XCD-major
  int parity;                // launch step parity
  double* fields;            // observe, single lattice: [6][ny][nx] or null
  double* pops;              // observe, single lattice: [2][9][ny][nx] or null
  int accumulate_wall;       // step: add wall momentum to the lattices' wave_wall
  int write_ref;             // observe: store each lattice's phi as its reference first
};

// Code variants of the step kernel (tuning choices, same arithmetic).
struct StepVariant {
  int prefetch;       // rows pulled ahead of the current one (0, 1 or 2)
  int stream_stores;  // nontemporal population stores
  int group = 1;      // tiles per workgroup of the FP32 deviation step: 1 or kGroupTiles
                      // (periodic only; every lattice of a grouped launch needs a
                      // multiple of kGroupTiles strips)
};
constexpr int kGroupTiles = 4;

// Launchers (lb_kernels.hip).  All return hipError_t of the launch.
// launch_step: FP64 steps (FP32 deviation storage steps through
// launch_split_step; fp64 = false returns hipErrorInvalidValue).
hipError_t launch_step(const LaunchArgs& a, bool fp64, bool walls, const StepVariant& v,
                       hipStream_t st);
hipError_t launch_observe(const LaunchArgs& a, bool fp64, bool walls, hipStream_t st);
// FP32-deviation step with one wavefront per species, periodic or with
// walls (lb_split.hip); fp64 = true returns hipErrorInvalidValue.
hipError_t launch_split_step(const LaunchArgs& a, bool fp64, bool walls, const StepVariant& v,
                             hipStream_t st);
// Fixed-order per-lattice sums of the per-tile slots of each lattice of
// descs[0..n): its kNRed observe values (which = 0) or its 2 wall
// accumulators (which = 1), into out[m * out_stride + 0 ..).  max_slots:
// the largest slot count among them (ny * nstrips for which = 0); n at
// most 65535.  The observe partials are consumed (overwritten in part).
hipError_t launch_reduce_lattices(const LatticeDesc* descs, int n, int which, double* out,
                                  int out_stride, long long max_slots, hipStream_t st);
// Write the t = 0 state: src buffer in pull layout plus the wall links, from
// FP64 densities / velocities on the device (u may be null).
hipError_t launch_init(const Geometry& g, const Coefs& c, bool fp64, bool walls,
                       const double* rho /*[2][ny][nx]*/, const double* u /*[2][ny][nx]*/,
                       void* buf, void* wall, hipStream_t st);
// Same from host-supplied populations f[2][9][ny][nx] (device copy).
hipError_t launch_set_pops(const Geometry& g, const Coefs& c, bool fp64, bool walls,
                           const double* f, void* buf, void* wall, hipStream_t st);
// Moment storage at tau = 1 (lb_moment.hip): step and observe launches over
// the same LaunchArgs, and the t = 0 state in local form from FP64 fields.
hipError_t launch_moment_step(const LaunchArgs& a, const StepVariant& v, hipStream_t st);
hipError_t launch_moment_observe(const LaunchArgs& a, hipStream_t st);
hipError_t launch_moment_init(const Geometry& g, const Coefs& c, const double* rho /*[2][ny][nx]*/,
                              const double* u /*[2][ny][nx] or null*/, void* buf, hipStream_t st);
// Counter-based noise densities rho_s = mean_s + amp (2U - 1) into rho[2][ny][nx].
hipError_t launch_noise(int nx, int ny, uint64_t seed, double mean_a, double mean_b, double amp,
                        double* rho, hipStream_t st);

}  // namespace lbk
