// Device helpers shared by the kernels of lb_kernels.hip (populations) and
// lb_moment.hip (equilibrium moments): D2Q9 tables, per-launch constants,
// memory access helpers, the pseudopotential and the interaction pairs.
// Internal; included by the kernel sources only.
#pragma once

#include "lb_internal.h"

#include <cmath>
#include <type_traits>
#include <utility>

namespace lbk {
namespace {

// D2Q9 velocities, order: rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1).
__host__ __device__ constexpr int cx(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cy(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
// D2Q9 weights (Table I, w): 4/9, 1/9 on the axes, 1/36 on the diagonals.
template <typename T>
__host__ __device__ constexpr T wq(int i) {
  return i == 0 ? T(4) / T(9) : (i < 5 ? T(1) / T(9) : T(1) / T(36));
}
// Wall links.  Bottom wall: a site in row 0 receives directions 2, 5, 6
// back from the wall, which left it as 4, 7, 8.  Top wall: row ny-1
// receives 4, 7, 8, which left as 2, 5, 6.
__host__ __device__ constexpr int wall_in_dir(int wall, int j) {
  return wall == 0 ? (j == 0 ? 2 : (j == 1 ? 5 : 6)) : (j == 0 ? 4 : (j == 1 ? 7 : 8));
}
__host__ __device__ constexpr int wall_out_dir(int wall, int j) {
  return wall == 0 ? (j == 0 ? 4 : (j == 1 ? 7 : 8)) : (j == 0 ? 2 : (j == 1 ? 5 : 6));
}

template <typename CT>
struct Fld {
  CT pa, pb, ra, rb;  // psi_A, psi_B, rho_A, rho_B
};

// One LDS ring entry of one field for both species.  psi and rho live in
// separate planes, so the 24 psi reads and the 8 rho reads of a site are
// unit-stride across the wave (no bank conflicts, no unused bytes).
template <typename CT>
struct Pr {
  CT a, b;
};

template <typename CT>
__device__ __forceinline__ CT exp_ct(CT x);
template <>
__device__ __forceinline__ float exp_ct<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double exp_ct<double>(double x) { return exp(x); }
template <typename CT>
__device__ __forceinline__ CT expm1_ct(CT x);
// FP32 expm1 by range reduction (written from the mathematics, not taken
// from a library): x = k ln2 + t with |t| <= ln2 / 2 (Cody-Waite: ln2 split
// so that k * ln2_hi is exact), expm1(t) from its Taylor series to t^7
// (truncation < 2e-8 relative on that interval), and
// expm1(x) = 2^k expm1(t) + (2^k - 1) in one fused rounding.  Within 1.5 ulp
// of the exact value on [-20, 5] (checked against FP64 expm1 on the host);
// about 15 instructions against 25 for the general library routine.
__device__ __forceinline__ float expm1_rr(float x) {
  const float k = __builtin_rintf(x * 1.44269504f);
  float t = __builtin_fmaf(-k, 0.693145751953125f, x);  // ln2 to 16 bits
  t = __builtin_fmaf(-k, 1.42860677e-06f, t);           // the rest of ln2
  float b = 1.f / 5040.f;
  b = __builtin_fmaf(b, t, 1.f / 720.f);
  b = __builtin_fmaf(b, t, 1.f / 120.f);
  b = __builtin_fmaf(b, t, 1.f / 24.f);
  b = __builtin_fmaf(b, t, 1.f / 6.f);
  b = __builtin_fmaf(b, t, 0.5f);
  const float p = __builtin_fmaf(t * t, b, t);
  const float s = __builtin_ldexpf(1.f, (int)k);
  return __builtin_fmaf(s, p, s - 1.f);
}
template <>
__device__ __forceinline__ float expm1_ct<float>(float x) { return expm1_rr(x); }
template <>
__device__ __forceinline__ double expm1_ct<double>(double x) { return expm1(x); }

// Ordering point for LDS traffic of a single-wave workgroup: every earlier
// LDS access has completed and no access moves across it.
__device__ __forceinline__ void lds_fence() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

template <typename CT, bool DEV>
struct Params;

template <bool DEV>
struct Params<double, DEV> {
  double k[2][5], kx[2], rho0, inv_rho0, tau[2], om[2], rref[2], pref[2], pscale[2], uw, g, g0, iny2;
  __device__ explicit Params(const Coefs& c) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int m = 0; m < 5; ++m) k[s][m] = c.kself[s][m];
      tau[s] = c.tau[s];
      om[s] = c.omega[s];
      rref[s] = DEV ? c.rho_ref[s] : 0.0;
      pref[s] = DEV ? c.psi_ref[s] : 0.0;
      pscale[s] = c.psi_scale[s];
    }
    kx[0] = c.kcross[0];
    kx[1] = c.kcross[1];
    rho0 = c.rho0;
    inv_rho0 = c.inv_rho0;
    uw = c.u_wall;
    g = c.g_body;
    g0 = c.g_uniform;
    iny2 = c.inv_ny2;
  }
};

template <bool DEV>
struct Params<float, DEV> {
  float k[2][5], kx[2], rho0, inv_rho0, tau[2], om[2], rref[2], pref[2], pscale[2], uw, g, g0, iny2;
  __device__ explicit Params(const Coefs& c) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int m = 0; m < 5; ++m) k[s][m] = c.f_kself[s][m];
      tau[s] = c.f_tau[s];
      om[s] = c.f_omega[s];
      rref[s] = DEV ? c.f_rho_ref[s] : 0.0f;
      pref[s] = DEV ? c.f_psi_ref[s] : 0.0f;
      pscale[s] = c.f_psi_scale[s];
    }
    kx[0] = c.f_kcross[0];
    kx[1] = c.f_kcross[1];
    rho0 = c.f_rho0;
    inv_rho0 = c.f_inv_rho0;
    uw = c.f_u_wall;
    g = c.f_g_body;
    g0 = c.f_g_uniform;
    iny2 = c.f_inv_ny2;
  }
};

template <typename CT>
__device__ __forceinline__ CT sinpi_ct(CT x);
template <>
__device__ __forceinline__ float sinpi_ct<float>(float x) { return sinpif(x); }
template <>
__device__ __forceinline__ double sinpi_ct<double>(double x) { return sinpi(x); }

template <typename CT>
__device__ __forceinline__ CT rcp_ct(CT x);
template <>
__device__ __forceinline__ float rcp_ct<float>(float x) {
  // hardware reciprocal (1 ulp) refined by one Newton step
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}
template <>
__device__ __forceinline__ double rcp_ct<double>(double x) { return 1.0 / x; }

// Global-memory (address space 1) views of device pointers.  The buffer
// pointers of a lattice are read from its record in memory, so the compiler
// cannot tell that they are global and would emit flat instructions; those
// also count on the LDS/scalar wait counter (4 bits), which caps the loads a
// wave keeps in flight and makes every LDS wait drain the HBM loads too.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ gmem<T>* to_global(T* p) {
  return (gmem<T>*)p;
}

// Loads and stores at a wave-uniform base plus a 32-bit per-lane byte
// offset, so the address is an SGPR pair plus one VGPR (no 64-bit per-lane
// address arithmetic).
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t byte_off) {
  const gmem<const char>* b = (const gmem<const char>*)base;
  return *(const gmem<const T>*)(b + byte_off);
}
// Population stores.  NT (streaming) stores keep the written buffer out of
// the caches: right for lattices larger than the 256 MB Infinity Cache, whose
// next-step reads come from HBM anyway, wrong for smaller ones, whose reads
// the Infinity Cache would serve.
template <bool NT, typename T>
__device__ __forceinline__ void st_at(T* base, uint32_t byte_off, T v) {
  gmem<T>* p = (gmem<T>*)((gmem<char>*)base + byte_off);
  if (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <typename CT, bool DEV>
__device__ __forceinline__ CT psi_of(const Params<CT, DEV>& P, int s, CT r) {
  // select, not index: a lane-varying index would move P to scratch
  if (DEV) return -(s ? P.pscale[1] : P.pscale[0]) * expm1_ct(-r * P.inv_rho0);
  return P.rho0 * (CT(1) - exp_ct(-r * P.inv_rho0));
}

// The twelve +-c pairs of the 24 interaction neighbours: (cx, cy, class),
// class 0..4 for |c|^2 = 1, 2, 4, 5, 8.  The first four are the first belt.
__host__ __device__ constexpr int pair_cx(int m) {
  return m == 0 ? 1 : m == 1 ? 0 : m == 2 ? 1 : m == 3 ? 1 : m == 4 ? 2 : m == 5 ? 0 :
         m == 6 ? 2 : m == 7 ? 2 : m == 8 ? 1 : m == 9 ? 1 : m == 10 ? 2 : 2;
}
__host__ __device__ constexpr int pair_cy(int m) {
  return m == 0 ? 0 : m == 1 ? 1 : m == 2 ? 1 : m == 3 ? -1 : m == 4 ? 0 : m == 5 ? 2 :
         m == 6 ? 1 : m == 7 ? -1 : m == 8 ? 2 : m == 9 ? -2 : m == 10 ? 2 : -2;
}
__host__ __device__ constexpr int pair_class(int m) {
  return m < 2 ? 0 : m < 4 ? 1 : m < 6 ? 2 : m < 10 ? 3 : 4;
}

template <int N, typename Fn, int... I>
__device__ __forceinline__ void static_for_impl(Fn&& fn, std::integer_sequence<int, I...>) {
  (fn(std::integral_constant<int, I>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  static_for_impl<N>(fn, std::make_integer_sequence<int, N>{});
}

// Wave sums of the kNRed per-lane observe values of one strip row, each by
// the same fixed xor tree, taken level by level across all values so that
// their cross-lane round trips overlap; lane 0 stores them at out[0 ..
// kNRed) and the values are cleared for the next row.
__device__ __forceinline__ void wave_sums_store(double (&acc)[kNRed], double* out, int lane) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int m = 0; m < kNRed; ++m) acc[m] += __shfl_xor(acc[m], off);
  }
  if (lane == 0) {
#pragma unroll
    for (int m = 0; m < kNRed; ++m) out[m] = acc[m];
  }
#pragma unroll
  for (int m = 0; m < kNRed; ++m) acc[m] = 0.0;
}

// Observables of one site at time t, in FP64 (observe launches): fields
// (rho_s, u', u_phys), optionally the 18 populations, and the partials of
// mass, momentum, half-force momentum, kinetic P_xy (Sec. III, Eq. (10)),
// the response mode (Sec. VIII, Eq. (66)) and the interface indicator
// (Eq. (67)).  f holds the pulled populations (deviations under DEV), atr
// reads the LDS rho ring at (dy, dx).
// phi_ref (may be null): the lattice's reference order parameter; with
// write_ref this site's phi = rho_A - rho_B is stored there first.  Either
// way the site adds phi_ref phi and phi_ref^2 to the overlap partials (the
// ageing correlation of Sec. VIII B, Eq. (68)).
template <typename CT, bool DEV, typename RingR>
__device__ __forceinline__ void observe_site(double* fields, double* pops, const Geometry& g,
                                             const Params<CT, DEV>& P, int y, int col,
                                             const CT (&rho)[2], const CT (&jx)[2],
                                             const CT (&jy)[2], const CT (&F)[2][2], CT ux, CT uy,
                                             const CT (&f)[2][9], RingR atr,
                                             double (&acc)[kNRed], double* phi_ref,
                                             bool write_ref) {
  const long long site = (long long)y * g.nx + col;
  const long long n = (long long)g.nx * g.ny;
  const double rt = (double)rho[0] + (double)rho[1];
  const double jtx = (double)jx[0] + (double)jx[1], jty = (double)jy[0] + (double)jy[1];
  const double Ftx = (double)F[0][0] + (double)F[1][0], Fty = (double)F[0][1] + (double)F[1][1];
  if (fields) {
    fields[0 * n + site] = (double)rho[0];
    fields[1 * n + site] = (double)rho[1];
    fields[2 * n + site] = (double)ux;
    fields[3 * n + site] = (double)uy;
    fields[4 * n + site] = (jtx + 0.5 * Ftx) / rt;
    fields[5 * n + site] = (jty + 0.5 * Fty) / rt;
  }
  if (pops) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
      for (int i = 0; i < 9; ++i)
        pops[(long long)(sp * 9 + i) * n + site] =
            (double)f[sp][i] + (DEV ? wq<double>(i) * (double)P.rref[sp] : 0.0);
  }
  acc[0] += (double)rho[0];
  acc[1] += (double)rho[1];
  acc[2] += jtx;
  acc[3] += jty;
  acc[4] += jtx + 0.5 * Ftx;
  acc[5] += jty + 0.5 * Fty;
  double pxy = 0;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
    pxy += ((double)f[sp][5] - (double)f[sp][6]) + ((double)f[sp][7] - (double)f[sp][8]);
  acc[6] += pxy;
  // response mode: u_phys,x against sin(2 pi y / ny)
  acc[7] += (jtx + 0.5 * Ftx) / rt * sinpi((double)y * (2.0 / (double)g.ny));
  // interface indicator with grad phi = 3 sum_{belt 1} w_i phi(r + c_i) c_i;
  // the ring holds density deviations, whose differences are the densities'
  double gax = 0, gay = 0, gbx = 0, gby = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int px = pair_cx(m), py = pair_cy(m);
    const double w3 = pair_class(m) == 0 ? 3.0 / 9.0 : 3.0 / 36.0;
    const Pr<CT>& hi = atr(py, px);
    const Pr<CT>& lo = atr(-py, -px);
    const double da = (double)hi.a - (double)lo.a, db = (double)hi.b - (double)lo.b;
    gax += w3 * px * da;
    gay += w3 * py * da;
    gbx += w3 * px * db;
    gby += w3 * py * db;
  }
  acc[8] -= gax * gbx + gay * gby;
  if (phi_ref) {
    const double phi = (double)rho[0] - (double)rho[1];
    if (write_ref) phi_ref[site] = phi;
    const double w = write_ref ? phi : phi_ref[site];
    acc[9] += w * phi;
    acc[10] += w * w;
  }
}

}  // namespace
}  // namespace lbk
