// HIP kernels for gfx950 of the two-species Shan-Chen lattice Boltzmann step
// (Benzi et al., arXiv:0906.3611, Sec. II).
//
// Layout.  Populations are structure-of-arrays planes [s][i][y][pitch] in
// "pull" form: the buffer for time t holds, at site q and direction i, the
// post-collision value that site q + c_i pulls when it streams into time t.
// A step reads one buffer and writes the other (ping-pong).  Under moving
// walls the three links of a wall-adjacent site that come back from the
// wall are kept in a small side buffer [wall][s][link][nx], written by the
// collision that sends them out.
//
// Decomposition.  One 64-lane wavefront owns a strip of at most 60 columns
// plus a 2-column ring on each side, and marches down a segment of rows.
// For every row it pulls the 18 populations (2 species x 9 directions) of
// its 64 columns, forms rho_s and psi_s into a 5-row LDS ring, and collides
// the row two behind, whose 25-point stencil is then complete.  Interior
// rows keep their pulled populations in registers until their collision, so
// every population is read from HBM once per step apart from the ring
// re-reads, which the neighbouring strips have just brought into L2.
#include "lb_internal.h"

#include <cmath>
#include <type_traits>

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

template <typename CT>
__device__ __forceinline__ CT exp_ct(CT x);
template <>
__device__ __forceinline__ float exp_ct<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double exp_ct<double>(double x) { return exp(x); }

// Ordering point for LDS traffic of a single-wave workgroup: every earlier
// LDS access has completed and no access moves across it.
__device__ __forceinline__ void lds_fence() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

template <typename CT, bool DEV>
struct Params {
  CT k[2][5];
  CT kx[2];
  CT rho0, inv_rho0, tau[2], om[2], rref[2], uw;
  __device__ explicit Params(const Coefs& c) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int m = 0; m < 5; ++m) k[s][m] = (CT)c.kself[s][m];
      tau[s] = (CT)c.tau[s];
      om[s] = (CT)c.omega[s];
      rref[s] = DEV ? (CT)c.rho_ref[s] : CT(0);
    }
    kx[0] = (CT)c.kcross[0];
    kx[1] = (CT)c.kcross[1];
    rho0 = (CT)c.rho0;
    inv_rho0 = (CT)c.inv_rho0;
    uw = (CT)c.u_wall;
  }
};

// Pull the 18 populations streaming into row re (a lattice row) for the
// wave's columns.  colm / colc / colp are the source columns for
// c_x = +1 / 0 / -1.
template <typename ST, typename CT, bool WALLS>
__device__ __forceinline__ void pull_row(const StepArgs& a, const ST* __restrict__ src,
                                         const ST* __restrict__ wall_in, int re, int colm,
                                         int colc, int colp, CT (&f)[2][9]) {
  const Geometry& g = a.g;
  int rm, rp;  // source rows for c_y = +1 and c_y = -1
  if (WALLS) {
    rm = re > 0 ? re - 1 : 0;
    rp = re < g.ny - 1 ? re + 1 : g.ny - 1;
  } else {
    rm = re > 0 ? re - 1 : g.ny - 1;
    rp = re < g.ny - 1 ? re + 1 : 0;
  }
  const bool bottom = WALLS && re == 0;
  const bool top = WALLS && re == g.ny - 1;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int row = cy(i) > 0 ? rm : (cy(i) < 0 ? rp : re);
      const int col = cx(i) > 0 ? colm : (cx(i) < 0 ? colp : colc);
      const ST* plane = src + (long long)(s * 9 + i) * g.plane + (long long)row * g.pitch;
      f[s][i] = (CT)plane[col];
    }
    if (WALLS) {
      if (bottom) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
          f[s][wall_in_dir(0, j)] = (CT)wall_in[((0 * 2 + s) * 3 + j) * g.nx + colc];
      }
      if (top) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
          f[s][wall_in_dir(1, j)] = (CT)wall_in[((1 * 2 + s) * 3 + j) * g.nx + colc];
      }
    }
  }
}

template <typename CT, bool DEV>
__device__ __forceinline__ Fld<CT> make_fields(const Params<CT, DEV>& P, const CT (&f)[2][9]) {
  CT r[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    CT acc = f[s][0];
#pragma unroll
    for (int i = 1; i < 9; ++i) acc += f[s][i];
    r[s] = DEV ? P.rref[s] + acc : acc;
  }
  Fld<CT> o;
  o.ra = r[0];
  o.rb = r[1];
  o.pa = P.rho0 * (CT(1) - exp_ct(-r[0] * P.inv_rho0));
  o.pb = P.rho0 * (CT(1) - exp_ct(-r[1] * P.inv_rho0));
  return o;
}

template <typename CT, bool DEV, bool WALLS, int MODE, typename ST>
__device__ __forceinline__ void collide_row(const StepArgs& a, const Params<CT, DEV>& P,
                                            const Fld<CT>* __restrict__ ring, int lane,
                                            const int (&slot)[5], int y, int colc,
                                            const CT (&f)[2][9], double (&acc)[kNRed],
                                            double (&wacc)[2], bool& bad) {
  const Geometry& g = a.g;
  auto R = [&](int dy, int dx) -> const Fld<CT>& { return ring[slot[dy + 2] * kWave + lane + dx]; };
  const Fld<CT> c0 = R(0, 0);
  // first belt: full records
  const Fld<CT> e = R(0, 1), w = R(0, -1), n = R(1, 0), s = R(-1, 0);
  const Fld<CT> ne = R(1, 1), sw = R(-1, -1), nw = R(1, -1), se = R(-1, 1);
  // second belt: psi only.  Index order: (2,0) (-2,0) (0,2) (0,-2)
  // (2,1) (-2,-1) (2,-1) (-2,1) (1,2) (-1,-2) (1,-2) (-1,2) (2,2) (-2,-2) (2,-2) (-2,2)
  const int b2dx[16] = {2, -2, 0, 0, 2, -2, 2, -2, 1, -1, 1, -1, 2, -2, 2, -2};
  const int b2dy[16] = {0, 0, 2, -2, 1, -1, -1, 1, 2, -2, -2, 2, 2, -2, -2, 2};
  CT qa[16], qb[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const Fld<CT>& v = R(b2dy[m], b2dx[m]);
    qa[m] = v.pa;
    qb[m] = v.pb;
  }
  CT F[2][2];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    const CT* q = sp == 0 ? qa : qb;
    auto P1 = [&](const Fld<CT>& v) { return sp == 0 ? v.pa : v.pb; };
    auto Ro = [&](const Fld<CT>& v) { return sp == 0 ? v.rb : v.ra; };
    // belt 1, |c|^2 = 1 and 2
    const CT d1x = P1(e) - P1(w), d1y = P1(n) - P1(s);
    const CT da = P1(ne) - P1(sw), db = P1(se) - P1(nw);
    const CT d2x = da + db, d2y = da - db;
    // belt 2
    const CT d4x = CT(2) * (q[0] - q[1]), d4y = CT(2) * (q[2] - q[3]);
    const CT a1 = q[4] - q[5], a2 = q[6] - q[7], a3 = q[8] - q[9], a4 = q[10] - q[11];
    const CT d5x = CT(2) * (a1 + a2) + (a3 + a4), d5y = (a1 - a2) + CT(2) * (a3 - a4);
    const CT c1 = q[12] - q[13], c2 = q[14] - q[15];
    const CT d8x = CT(2) * (c1 + c2), d8y = CT(2) * (c1 - c2);
    const CT Sx = P.k[sp][0] * d1x + P.k[sp][1] * d2x + P.k[sp][2] * d4x + P.k[sp][3] * d5x +
                  P.k[sp][4] * d8x;
    const CT Sy = P.k[sp][0] * d1y + P.k[sp][1] * d2y + P.k[sp][2] * d4y + P.k[sp][3] * d5y +
                  P.k[sp][4] * d8y;
    // cross term on the other species' density
    const CT x1x = Ro(e) - Ro(w), x1y = Ro(n) - Ro(s);
    const CT xa = Ro(ne) - Ro(sw), xb = Ro(se) - Ro(nw);
    const CT Xx = P.kx[0] * x1x + P.kx[1] * (xa + xb);
    const CT Xy = P.kx[0] * x1y + P.kx[1] * (xa - xb);
    const CT psi0 = sp == 0 ? c0.pa : c0.pb;
    const CT rho0s = sp == 0 ? c0.ra : c0.rb;
    F[sp][0] = -psi0 * Sx - rho0s * Xx;
    F[sp][1] = -psi0 * Sy - rho0s * Xy;
  }
  // moments and velocities (Eq. (1) and the common velocity below it)
  const CT rho[2] = {c0.ra, c0.rb};
  CT jx[2], jy[2];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    jx[sp] = (f[sp][1] - f[sp][3]) + (f[sp][5] - f[sp][6]) + (f[sp][8] - f[sp][7]);
    jy[sp] = (f[sp][2] - f[sp][4]) + (f[sp][5] - f[sp][8]) + (f[sp][6] - f[sp][7]);
    if (!(rho[sp] > CT(0)) || !(rho[sp] < CT(1e30))) bad = true;
  }
  const CT inv_den = CT(1) / (rho[0] * P.om[0] + rho[1] * P.om[1]);
  const CT ux = (jx[0] * P.om[0] + jx[1] * P.om[1]) * inv_den;
  const CT uy = (jy[0] * P.om[0] + jy[1] * P.om[1]) * inv_den;

  if (MODE == kObserve) {
    const int x = colc;
    const long long site = (long long)y * g.nx + x;
    const long long n = (long long)g.nx * g.ny;
    const double rt = (double)rho[0] + (double)rho[1];
    const double jtx = (double)jx[0] + (double)jx[1], jty = (double)jy[0] + (double)jy[1];
    const double Ftx = (double)F[0][0] + (double)F[1][0], Fty = (double)F[0][1] + (double)F[1][1];
    if (a.fields) {
      a.fields[0 * n + site] = (double)rho[0];
      a.fields[1 * n + site] = (double)rho[1];
      a.fields[2 * n + site] = (double)ux;
      a.fields[3 * n + site] = (double)uy;
      a.fields[4 * n + site] = (jtx + 0.5 * Ftx) / rt;
      a.fields[5 * n + site] = (jty + 0.5 * Fty) / rt;
    }
    if (a.pops) {
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int i = 0; i < 9; ++i)
          a.pops[(long long)(sp * 9 + i) * n + site] =
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
    return;
  }

  // BGK relaxation towards the equilibrium at v_s = u' + tau_s F_s / rho_s
  CT post[2][9];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    const CT ir = CT(1) / rho[sp];
    const CT vx = ux + P.tau[sp] * F[sp][0] * ir;
    const CT vy = uy + P.tau[sp] * F[sp][1] * ir;
    const CT usq = CT(1.5) * (vx * vx + vy * vy);
    const CT drho = DEV ? rho[sp] - P.rref[sp] : CT(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const CT cu = (CT)cx(i) * vx + (CT)cy(i) * vy;
      const CT poly = cu * (CT(3) + CT(4.5) * cu) - usq;
      // f^eq_i = w_i rho (1 + poly); deviation form: f^eq_i - w_i rho_ref
      const CT feq = DEV ? wq<CT>(i) * (drho + rho[sp] * poly) : wq<CT>(i) * rho[sp] * (CT(1) + poly);
      post[sp][i] = f[sp][i] + P.om[sp] * (feq - f[sp][i]);
    }
  }
  ST* dst = (ST*)a.dst;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int i = 0; i < 9; ++i)
      dst[(long long)(sp * 9 + i) * g.plane + (long long)y * g.pitch + colc] = (ST)post[sp][i];

  if (WALLS) {
    const bool bottom = y == 0, top = y == g.ny - 1;
    if (bottom || top) {
      const int wl = top ? 1 : 0;
      const CT uwall = top ? P.uw : -P.uw;
      ST* wall_out = (ST*)a.wall_out;
      double mom = 0;
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          // the j-th link leaves along o = wall_out_dir and comes back as wall_in_dir:
          // f_back = f*_o - 2 w_o rho_w (c_o . u_w) / c_s^2, rho_w = rho_s(r, t)
          const int o = bottom ? wall_out_dir(0, j) : wall_out_dir(1, j);
          const CT corr = CT(6) * wq<CT>(o) * rho[sp] * ((CT)cx(o) * uwall);
          const CT back = post[sp][o] - corr;
          wall_out[((wl * 2 + sp) * 3 + j) * g.nx + colc] = (ST)back;
          const double full = (double)post[sp][o] + (DEV ? wq<double>(o) * (double)P.rref[sp] : 0.0);
          mom += (double)cx(o) * (2.0 * full - (double)corr);
        }
      wacc[wl] += mom;
    }
  }
}


template <typename ST, typename CT, bool DEV, bool WALLS, int MODE>
__global__ __launch_bounds__(kWave) void k_march(const StepArgs a) {
  __shared__ Fld<CT> ring[kRing * kWave];
  const Geometry& g = a.g;
  const int b = blockIdx.x;
  const int tile = (b & 7) * g.tiles_per_xcd + (b >> 3);
  if (tile >= g.ntiles) return;
  const int strip = tile % g.nstrips;
  const int seg = tile / g.nstrips;
  const int lane = threadIdx.x;
  const int nx = g.nx, ny = g.ny;
  const int x0 = (int)((long long)strip * nx / g.nstrips);
  const int x1 = (int)((long long)(strip + 1) * nx / g.nstrips);
  const int y0 = (int)((long long)seg * ny / g.nsegs);
  const int y1 = (int)((long long)(seg + 1) * ny / g.nsegs);
  const int nint = x1 - x0;
  const bool active = lane >= 2 && lane < 2 + nint;
  const int colc = wrap(x0 - 2 + lane, nx);
  const int colm = wrap(x0 - 3 + lane, nx);  // source column of c_x = +1
  const int colp = wrap(x0 - 1 + lane, nx);  // source column of c_x = -1
  const Params<CT, DEV> P(a.c);
  const ST* __restrict__ src = (const ST*)a.src;
  const ST* __restrict__ wall_in = (const ST*)a.wall_in;

  CT fr[3][2][9];
  double acc[kNRed];
#pragma unroll
  for (int m = 0; m < kNRed; ++m) acc[m] = 0.0;
  double wacc[2] = {0.0, 0.0};
  bool bad = false;
  const int K = (y1 - y0) + 4;  // rows y0-2 .. y1+1

  auto iter = [&](int k, auto cur_tag, auto old_tag) {
    constexpr int cur = decltype(cur_tag)::value;
    constexpr int old = decltype(old_tag)::value;
    const int r = y0 - 2 + k;
    int re;
    if (WALLS) {
      re = r < 0 ? -1 - r : (r >= ny ? 2 * ny - 1 - r : r);  // mirror ghost rows
    } else {
      re = r < 0 ? r + ny : (r >= ny ? r - ny : r);
      re = wrap(re, ny);  // lattices shorter than the ring
    }
    pull_row<ST, CT, WALLS>(a, src, wall_in, re, colm, colc, colp, fr[cur]);
    const Fld<CT> fl = make_fields<CT, DEV>(P, fr[cur]);
    lds_fence();
    ring[(k % kRing) * kWave + lane] = fl;
    lds_fence();
    if (k >= 4 && active) {
      int slot[5];
#pragma unroll
      for (int d = 0; d < 5; ++d) slot[d] = (k - 4 + d) % kRing;
      collide_row<CT, DEV, WALLS, MODE, ST>(a, P, ring, lane, slot, r - 2, colc, fr[old], acc,
                                            wacc, bad);
    }
  };

  for (int k0 = 0; k0 < K; k0 += 3) {
    iter(k0, std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
    if (k0 + 1 < K) iter(k0 + 1, std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{});
    if (k0 + 2 < K) iter(k0 + 2, std::integral_constant<int, 2>{}, std::integral_constant<int, 0>{});
  }

  if (__any(bad) && lane == 0) atomicOr(a.flag, 1);
  if (MODE == kObserve) {
#pragma unroll
    for (int m = 0; m < kNRed; ++m) {
      double v = acc[m];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) a.wave_red[(long long)tile * kNRed + m] = v;
    }
  } else if (WALLS && a.accumulate_wall && (y0 == 0 || y1 == ny)) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      double v = wacc[m];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) a.wave_wall[(long long)tile * 2 + m] += v;
    }
  }
}

// Fixed-order reduction of per-tile values: thread t sums tiles t, t + 256,
// ... in order, then a fixed binary tree.  One block; deterministic.
__global__ __launch_bounds__(256) void k_reduce_tiles(const double* __restrict__ in, int ntiles,
                                                      int width, double* __restrict__ out) {
  __shared__ double sh[256];
  for (int m = 0; m < width; ++m) {
    double v = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 256) v += in[(long long)t * width + m];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
      if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[m] = sh[0];
    __syncthreads();
  }
}

// Equilibrium (Sec. II, display below Eq. (1)) in FP64.
__device__ __forceinline__ double feq64(int i, double rho, double ux, double uy) {
  const double cu = cx(i) * ux + cy(i) * uy;
  return wq<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy));
}

// t = 0 state.  Thread per site q of the buffer: buf[s][i][q] holds what
// site q + c_i pulls, i.e. the population of that site.  FROM_POPS selects
// the source: equilibrium of rho/u, or explicit populations.
template <typename ST, bool DEV, bool WALLS, bool FROM_POPS>
__global__ __launch_bounds__(256) void k_init(Geometry g, Coefs c, const double* __restrict__ rho,
                                              const double* __restrict__ u,
                                              const double* __restrict__ pops, ST* __restrict__ buf,
                                              ST* __restrict__ wall) {
  const long long n = (long long)g.nx * g.ny;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int x = (int)(q % g.nx), y = (int)(q / g.nx);
  auto value = [&](int s, int i, int xs, int ys) -> double {
    const long long site = (long long)ys * g.nx + xs;
    double f;
    if (FROM_POPS) {
      f = pops[(long long)(s * 9 + i) * n + site];
    } else {
      const double ux = u ? u[site] : 0.0, uy = u ? u[n + site] : 0.0;
      f = feq64(i, rho[(long long)s * n + site], ux, uy);
    }
    return DEV ? f - wq<double>(i) * c.rho_ref[s] : f;
  };
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int xs = x + cx(i), ys = y + cy(i);
      xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
      if (WALLS) {
        if (ys < 0 || ys >= g.ny) ys = y;  // slot never pulled; keep it defined
      } else {
        ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
      }
      buf[(long long)(s * 9 + i) * g.plane + (long long)y * g.pitch + x] = (ST)value(s, i, xs, ys);
    }
  if (WALLS && (y == 0 || y == g.ny - 1)) {
    const int wl = y == 0 ? 0 : 1;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        wall[((wl * 2 + s) * 3 + j) * g.nx + x] = (ST)value(s, wall_in_dir(wl, j), x, y);
  }
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_noise(int nx, int ny, uint64_t seed, double ma, double mb,
                                               double amp, double* __restrict__ rho) {
  const long long n = (long long)nx * ny;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 2 * n) return;
  const int s = (int)(q / n);
  const double u01 = (double)(splitmix64(seed, (uint64_t)q + 1) >> 11) * 0x1.0p-53;
  rho[q] = (s == 0 ? ma : mb) + amp * (2.0 * u01 - 1.0);
}

template <int MODE>
hipError_t launch_march(const StepArgs& a, bool fp64, bool walls, hipStream_t st) {
  const dim3 grid(8 * a.g.tiles_per_xcd), block(kWave);
  if (fp64) {
    if (walls)
      hipLaunchKernelGGL((k_march<double, double, false, true, MODE>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_march<double, double, false, false, MODE>), grid, block, 0, st, a);
  } else if (MODE == kStep) {
    if (walls)
      hipLaunchKernelGGL((k_march<float, float, true, true, MODE>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_march<float, float, true, false, MODE>), grid, block, 0, st, a);
  } else {
    // observation of FP32 deviation storage is evaluated in FP64
    if (walls)
      hipLaunchKernelGGL((k_march<float, double, true, true, MODE>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_march<float, double, true, false, MODE>), grid, block, 0, st, a);
  }
  return hipGetLastError();
}

template <bool FROM_POPS>
hipError_t launch_init_any(const Geometry& g, const Coefs& c, bool fp64, bool walls,
                           const double* rho, const double* u, const double* pops, void* buf,
                           void* wall, hipStream_t st) {
  const long long n = (long long)g.nx * g.ny;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (fp64) {
    if (walls)
      hipLaunchKernelGGL((k_init<double, false, true, FROM_POPS>), grid, block, 0, st, g, c, rho, u,
                         pops, (double*)buf, (double*)wall);
    else
      hipLaunchKernelGGL((k_init<double, false, false, FROM_POPS>), grid, block, 0, st, g, c, rho,
                         u, pops, (double*)buf, (double*)wall);
  } else {
    if (walls)
      hipLaunchKernelGGL((k_init<float, true, true, FROM_POPS>), grid, block, 0, st, g, c, rho, u,
                         pops, (float*)buf, (float*)wall);
    else
      hipLaunchKernelGGL((k_init<float, true, false, FROM_POPS>), grid, block, 0, st, g, c, rho, u,
                         pops, (float*)buf, (float*)wall);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(const StepArgs& a, bool fp64, bool walls, hipStream_t st) {
  return launch_march<kStep>(a, fp64, walls, st);
}

hipError_t launch_observe(const StepArgs& a, bool fp64, bool walls, hipStream_t st) {
  return launch_march<kObserve>(a, fp64, walls, st);
}

hipError_t launch_reduce_tiles(const double* in, int ntiles, int width, double* out,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_tiles, dim3(1), dim3(256), 0, st, in, ntiles, width, out);
  return hipGetLastError();
}

hipError_t launch_init(const Geometry& g, const Coefs& c, bool fp64, bool walls, const double* rho,
                       const double* u, void* buf, void* wall, hipStream_t st) {
  return launch_init_any<false>(g, c, fp64, walls, rho, u, nullptr, buf, wall, st);
}

hipError_t launch_set_pops(const Geometry& g, const Coefs& c, bool fp64, bool walls,
                           const double* f, void* buf, void* wall, hipStream_t st) {
  return launch_init_any<true>(g, c, fp64, walls, nullptr, nullptr, f, buf, wall, st);
}

hipError_t launch_noise(int nx, int ny, uint64_t seed, double mean_a, double mean_b, double amp,
                        double* rho, hipStream_t st) {
  const long long n2 = 2LL * nx * ny;
  hipLaunchKernelGGL(k_noise, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, nx, ny, seed,
                     mean_a, mean_b, amp, rho);
  return hipGetLastError();
}

}  // namespace lbk
