// HIP kernels of the moment representation (LB_FP32_MOM), for
// tau_A = tau_B = 1.
//
// With tau_s = 1 the BGK collision of Eq. (1) replaces every population by
// its equilibrium, f*_is = f^eq_i(rho_s, v_s) (display below Eq. (1)), so
// after a collision the 18 populations of a site are fixed by the 6 numbers
// (rho_s, v_s).  The state is kept as those numbers, in pull form: the
// buffer for time t holds M_s(q) = (rho_s - rho_ref_s, v_s) of the collision
// at q in step t - 1, and the populations at t are
//     f_is(r, t) = f^eq_i(M_s(r - c_i)).
// A step forms rho_s and j_s of every site from the equilibria of its 9
// sources, the forces of Eq. (2), u' and v_s, and writes the site's own 6
// numbers: 48 B per site update in FP32 instead of 144 B.
// Right after an initialization the buffer is in "local" form (a flag per
// buffer): f_is(r, 0) = f^eq_i(M_s(r)), the zero-step equilibrium state of
// Sec. VI; the first step reads it that way and clears the flag of the
// buffer it writes.
//
// Layout: row y is pitch / 64 blocks of 64 sites, each block holding 6 runs
// of 64 FP32 values: rho_A - rho_ref_A, v_Ax, v_Ay, rho_B - rho_ref_B, v_Bx,
// v_By.
//
// Step kernel.  The equilibrium of direction i at a source with density
// A = rho_ref + r and velocity v is, minus w_i rho_ref,
//     w_i [ r + 3 A (c_i.v) + 4.5 A (c_i.v)^2 - 1.5 A v^2 ],
// which is linear in the source's r, A v_x, A v_y, A v_x^2, A v_y^2 and
// A v_x v_y.  Each source site is therefore turned once into seven stencil
// coefficients (struct Coef), after which every one of its nine outgoing
// equilibria costs one to three additions.  The nine sources of a site lie
// in three rows; each row, when it arrives, yields per column the
// contributions of its three "roles" -- as the row below the destination
// (populations moving up, U), the destination row itself (C) and the row
// above (D) -- and a destination row adds them as C + (U + D), the same
// association for either march direction, so results do not depend on the
// tiling.  Decomposition as in lb_kernels.hip: one wavefront per (64-column
// strip, row segment) tile marching along its rows, rho and psi of five
// finalized rows in an LDS ring, the row two behind collided.
//
// Observe kernel: FP64, from the 18 equilibria of each site (they are also
// the populations it reports).
#include "lb_device.h"

namespace lbk {
namespace {

constexpr int kPlanes = 6;
constexpr int kHalo = 3;                  // window columns beyond the strip, each side
constexpr int kWin = kWave + 2 * kHalo;  // window entries per row

// ---------------------------------------------------------------- step ----

// Stencil coefficients of one species at one source site.  Its deviation
// equilibria in the nine directions are
//   rest: b0;   E, W: bx +- 4 ax5;   N, S: by +- 4 ay5;
//   NE: bd + qxy + ax5 + ay5,  SE: bd - qxy + ax5 - ay5,
//   NW: bd - qxy - ax5 + ay5,  SW: bd + qxy - ax5 - ay5.
struct Coef {
  float bd, qxy, ax5, ay5;
  float bx, by, b0, r;  // r: the stored rho - rho_ref itself
};

__device__ __forceinline__ Coef coef_of(float rref, float r, float vx, float vy) {
#pragma clang fp contract(on)
  const float A = rref + r;
  const float ax = A * vx, ay = A * vy;
  const float qxx = ax * vx, qyy = ay * vy, qxy = ax * vy;
  const float sq = qxx + qyy;
  const float base = r - 1.5f * sq;  // r - 1.5 A v^2
  Coef c;
  c.bx = (1.f / 9.f) * (base + 4.5f * qxx);
  c.by = (1.f / 9.f) * (base + 4.5f * qyy);
  c.bd = (1.f / 36.f) * (r + 3.f * sq);  // base + 4.5 A v^2
  c.qxy = 0.25f * qxy;                   // 9 w_diag
  c.ax5 = (1.f / 12.f) * ax;             // 3 w_diag; 4 ax5 = 3 w_axis ax exactly
  c.ay5 = (1.f / 12.f) * ay;
  c.r = r;
  // The nine equilibria of a source sum to b0 + 2 bx + 2 by + 4 bd, which
  // is r in exact arithmetic (the equilibrium keeps the mass).  With FP32
  // weights (summing to 1 + 7.45e-9) b0 = (4/9) base would move the mass a
  // source sends out by that fraction, with the sign of its deviation, and
  // the total would drift; b0 is therefore what is left of r after the
  // eight moving equilibria, formed in FP64 (exactly (4/9) base otherwise).
  c.b0 = (float)((double)r - (2.0 * (double)c.bx + 2.0 * (double)c.by + 4.0 * (double)c.bd));
  return c;
}

// The LDS window of one row: each site's coefficients for both species, as
// two species-major planes of 16-byte entries, so that a wave's accesses of
// one species and one half are consecutive (no bank conflicts).
struct alignas(16) F4 {
  float x, y, z, w;
};
struct Window {
  F4 a[2][kWin];  // bd, qxy, ax5, ay5
  F4 b[2][kWin];  // bx, by, b0, r
  __device__ __forceinline__ void put(int s, int pos, const Coef& c) {
    a[s][pos] = F4{c.bd, c.qxy, c.ax5, c.ay5};
    b[s][pos] = F4{c.bx, c.by, c.b0, c.r};
  }
  __device__ __forceinline__ Coef get(int s, int pos) const {
    const F4 u = a[s][pos], v = b[s][pos];
    return Coef{u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
  }
};

// Contributions (density deviation and x momentum) of one source row to the
// column between sources L (x - 1), M (x) and R (x + 1) of that row, in its
// three roles.
struct Part {
  float u, ux, c, cx, d, dx;
};

__device__ __forceinline__ void partials(const Coef& L, const Coef& M, const Coef& R, Part& o) {
#pragma clang fp contract(on)
  const float ne = (L.bd + L.qxy) + (L.ax5 + L.ay5);
  const float se = (L.bd - L.qxy) + (L.ax5 - L.ay5);
  const float e = L.bx + 4.f * L.ax5;
  const float nw = (R.bd - R.qxy) - (R.ax5 - R.ay5);
  const float sw = (R.bd + R.qxy) - (R.ax5 + R.ay5);
  const float w = R.bx - 4.f * R.ax5;
  const float n = M.by + 4.f * M.ay5;
  const float s = M.by - 4.f * M.ay5;
  o.u = (n + ne) + nw;
  o.ux = ne - nw;
  o.c = (M.b0 + e) + w;
  o.cx = e - w;
  o.d = (s + se) + sw;
  o.dx = se - sw;
}

constexpr int kRingW = kWave + 4;  // ring entries per row

// One tile of the step; up: the tile marches towards increasing y; local:
// the source buffer is in local form (the first step after an
// initialization).  Both stay runtime selects: copies of the march per case
// measured slower (more registers, fewer waves per SIMD).
template <bool NT>
__device__ __forceinline__ void mstep_tile(const LaunchArgs& a, const LatticeDesc* __restrict__ D,
                                           int local_tile, int sel, bool up, bool local,
                                           Window& win, Pr<float>* ring_p, Pr<float>* ring_r) {
#pragma clang fp contract(on)
  constexpr int W = kRingW;
  const Geometry g = D->g;
  const int strip = local_tile % g.nstrips;
  const int seg = local_tile / g.nstrips;
  const int lane = threadIdx.x;
  const int nx = g.nx, ny = g.ny;
  const int x0 = strip * kWave;
  const int width = min(kWave, nx - x0);
  const int y0 = (int)((long long)seg * ny / g.nsegs);
  const int y1 = (int)((long long)(seg + 1) * ny / g.nsegs);
  const int dir = up ? 1 : -1;
  const bool active = lane < width;
  const int col = active ? x0 + lane : wrap(x0 + lane, nx);
  auto in_row = [&](int c) { return (uint32_t)((c >> 6) * (kPlanes * kWave) + (c & 63)) * 4u; };
  const uint32_t ob_c = in_row(col);
  constexpr uint32_t kPl = kWave * 4u;  // bytes between planes
  // halo items: lane t < 12 holds species t / 6 of halo column t % 6
  const bool hl = lane < 2 * 2 * kHalo;
  const int hc = lane % 6, hs = (lane / 6) & 1;
  const int hcol = wrap(hc < kHalo ? x0 - kHalo + hc : x0 + width + (hc - kHalo), nx);
  const int hpos = hc < kHalo ? hc : width + kHalo + (hc - kHalo);
  const uint32_t ob_h = in_row(hcol) + (uint32_t)(3 * hs) * kPl;
  // ring lanes 0..7: column rcl = lane & 3 of species lane >> 2
  const bool rl = lane < 8;
  const int rcl = lane & 3, rsp = (lane >> 2) & 1;
  const int rpos = rcl < 2 ? rcl : width + rcl;                 // ring position
  const int rwin = rcl < 2 ? 1 + rcl : width + kHalo + (rcl - 2);  // window position
  const int own = lane + kHalo;                                  // window position

  const Params<float, true> P(D->c);
  const float* __restrict__ src = (const float*)D->buf[sel];
  float* __restrict__ dst = (float*)D->buf[sel ^ 1];

  // march positions 0 .. NP-1 are rows y0-3 .. y1+2 (upward tiles)
  const int NP = (y1 - y0) + 6;
  const int rstart = up ? y0 - 3 : y1 + 2;
  auto lattice_row = [&](int p) {
    const int r = rstart + dir * p;
    return r < 0 ? r + ny : (r >= ny ? r - ny : r);
  };
  float ld[kPlanes], lh[3];
  auto issue = [&](int p) {
    const float* row = src + (long long)lattice_row(p) * g.row_elems;
#pragma unroll
    for (int q = 0; q < kPlanes; ++q) ld[q] = ld_at(row, ob_c + (uint32_t)q * kPl);
#pragma unroll
    for (int q = 0; q < 3; ++q) lh[q] = hl ? ld_at(row, ob_h + (uint32_t)q * kPl) : 0.f;
  };

  // Per row, both species: its contributions to the destination rows it
  // feeds, ordered by the march: C to itself, Fw to the next position, Bw
  // to the previous one.  In local form the sources of a site are the site
  // itself, so rho - rho_ref and j are its own numbers (the moments of an
  // equilibrium) and go into C, with Fw = Bw = 0.
  float qc[3][2], qcx[3][2], qcy[3][2], qf[3][2], qfx[3][2], qb[3][2], qbx[3][2];
  float rc[3], rf[3], rb[3];  // ring lanes: density contributions of their column
  float rdf[3][2], jxf[3][2], jyf[3][2];  // finalized rows
  const float fdir = (float)dir;
  bool bad = false;

  issue(0);
  for (int p0 = 0; p0 < NP; p0 += 3) {
    static_for<3>([&](auto J) {
      constexpr int j = decltype(J)::value;
      constexpr int j1 = (j + 2) % 3;  // slot of position p - 1
      constexpr int j2 = (j + 1) % 3;  // slot of position p - 2 (and p - 3)
      const int p = p0 + j;
      if (p >= NP) return;
      // row p: stencil coefficients into the window, then the next row's loads
      const Coef c0 = coef_of(P.rref[0], ld[0], ld[1], ld[2]);
      const Coef c1 = coef_of(P.rref[1], ld[3], ld[4], ld[5]);
      const Coef ch = coef_of(hs ? P.rref[1] : P.rref[0], lh[0], lh[1], lh[2]);
      // j of the own site (used in local form; same products as in coef_of)
      const float lj[2][2] = {{(P.rref[0] + ld[0]) * ld[1], (P.rref[0] + ld[0]) * ld[2]},
                              {(P.rref[1] + ld[3]) * ld[4], (P.rref[1] + ld[3]) * ld[5]}};
      if (p + 1 < NP) issue(p + 1);
      if (active) {
        win.put(0, own, c0);
        win.put(1, own, c1);
      }
      if (hl) win.put(hs, hpos, ch);
      lds_fence();
      {
        Part t[2];
        partials(win.get(0, own - 1), c0, win.get(0, own + 1), t[0]);
        partials(win.get(1, own - 1), c1, win.get(1, own + 1), t[1]);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          qc[j][s] = local ? (s ? c1.r : c0.r) : t[s].c;
          qcx[j][s] = local ? lj[s][0] : t[s].cx;
          qcy[j][s] = local ? lj[s][1] : 0.f;
          qf[j][s] = local ? 0.f : (up ? t[s].u : t[s].d);
          qfx[j][s] = local ? 0.f : (up ? t[s].ux : t[s].dx);
          qb[j][s] = local ? 0.f : (up ? t[s].d : t[s].u);
          qbx[j][s] = local ? 0.f : (up ? t[s].dx : t[s].ux);
        }
        if (rl) {
          Part tr;
          partials(win.get(rsp, rwin - 1), win.get(rsp, rwin), win.get(rsp, rwin + 1), tr);
          rc[j] = local ? win.b[rsp][rwin].w : tr.c;
          rf[j] = local ? 0.f : (up ? tr.u : tr.d);
          rb[j] = local ? 0.f : (up ? tr.d : tr.u);
        }
      }
      // finalize position f = p - 1: C of f plus the contributions of its
      // two neighbour rows, (U + D) in either march direction
      if (p >= 2) {
        const int f = p - 1;
        Pr<float>* rowp = ring_p + (f % kRing) * W;
        Pr<float>* rowr = ring_r + (f % kRing) * W;
        float psi[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          rdf[j1][s] = qc[j1][s] + (qf[j2][s] + qb[j][s]);
          jxf[j1][s] = qcx[j1][s] + (qfx[j2][s] + qbx[j][s]);
          jyf[j1][s] = qcy[j1][s] + (qf[j2][s] - qb[j][s]) * fdir;  // U - D
          psi[s] = psi_of<float, true>(P, s, rdf[j1][s]);
        }
        if (active) {
          rowp[lane + 2] = Pr<float>{psi[0], psi[1]};
          rowr[lane + 2] = Pr<float>{rdf[j1][0], rdf[j1][1]};
        }
        if (rl) {
          const float rr = rc[j1] + (rf[j2] + rb[j]);
          const float ps = psi_of<float, true>(P, rsp, rr);
          if (rsp) {
            rowp[rpos].b = ps;
            rowr[rpos].b = rr;
          } else {
            rowp[rpos].a = ps;
            rowr[rpos].a = rr;
          }
        }
      }
      lds_fence();

      // collide position c = p - 3 (rows y0 .. y1-1), finalized one step ago
      if (p >= 6 && active) {
        const int c = p - 3;
        int slot[5];
#pragma unroll
        for (int d = 0; d < 5; ++d) slot[d] = (c + dir * (d - 2)) % kRing;
        auto atp = [&](int dy, int dx) -> const Pr<float>& {
          return ring_p[slot[dy + 2] * W + lane + 2 + dx];
        };
        auto atr = [&](int dy, int dx) -> const Pr<float>& {
          return ring_r[slot[dy + 2] * W + lane + 2 + dx];
        };
        const int y = lattice_row(c);
        // forces (Eq. (2)) over the twelve +-c pairs
        float Sxa = 0, Sya = 0, Sxb = 0, Syb = 0, Xxa = 0, Xya = 0, Xxb = 0, Xyb = 0;
#pragma unroll
        for (int m = 0; m < 12; ++m) {
          const int px = pair_cx(m), py = pair_cy(m), kk = pair_class(m);
          const Pr<float>& hi = atp(py, px);
          const Pr<float>& lo = atp(-py, -px);
          const float da = hi.a - lo.a, db = hi.b - lo.b;
          if (px) {
            Sxa += (P.k[0][kk] * (float)px) * da;
            Sxb += (P.k[1][kk] * (float)px) * db;
          }
          if (py) {
            Sya += (P.k[0][kk] * (float)py) * da;
            Syb += (P.k[1][kk] * (float)py) * db;
          }
          if (m < 4) {
            const Pr<float>& rhi = atr(py, px);
            const Pr<float>& rlo = atr(-py, -px);
            const float ea = rhi.a - rlo.a, eb = rhi.b - rlo.b;
            if (px) {
              Xxa += (P.kx[kk] * (float)px) * eb;
              Xxb += (P.kx[kk] * (float)px) * ea;
            }
            if (py) {
              Xya += (P.kx[kk] * (float)py) * eb;
              Xyb += (P.kx[kk] * (float)py) * ea;
            }
          }
        }
        const Pr<float> c0p = atp(0, 0);
        const float rho[2] = {P.rref[0] + rdf[j][0], P.rref[1] + rdf[j][1]};
        const float psi[2] = {P.pref[0] + c0p.a, P.pref[1] + c0p.b};
        float F[2][2] = {{-psi[0] * Sxa - rho[0] * Xxa, -psi[0] * Sya - rho[0] * Xya},
                         {-psi[1] * Sxb - rho[1] * Xxb, -psi[1] * Syb - rho[1] * Xyb}};
        if (P.g != 0.f || P.g0 != 0.f) {
          const float gy = P.g * sinpi_ct<float>((float)y * P.iny2) + P.g0;
          F[0][0] += rho[0] * gy;
          F[1][0] += rho[1] * gy;
        }
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
          if (!(rho[sp] > 0.f) || !(rho[sp] < 1e30f)) bad = true;
        const float inv_den = rcp_ct(rho[0] * P.om[0] + rho[1] * P.om[1]);
        const float ux = (jxf[j][0] * P.om[0] + jxf[j][1] * P.om[1]) * inv_den;
        const float uy = (jyf[j][0] * P.om[0] + jyf[j][1] * P.om[1]) * inv_den;
        // post-collision numbers: rho unchanged, v_s = u' + tau_s F_s / rho_s
        float* row = dst + (long long)y * g.row_elems;
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
          const float ir = rcp_ct(rho[sp]);
          const float vx = ux + P.tau[sp] * F[sp][0] * ir;
          const float vy = uy + P.tau[sp] * F[sp][1] * ir;
          st_at<NT>(row, ob_c + (uint32_t)(3 * sp + 0) * kPl, rdf[j][sp]);
          st_at<NT>(row, ob_c + (uint32_t)(3 * sp + 1) * kPl, vx);
          st_at<NT>(row, ob_c + (uint32_t)(3 * sp + 2) * kPl, vy);
        }
      }
    });
  }
  if (__any(bad) && lane == 0) atomicOr(D->flag, 1);
}

template <bool NT>
__global__ __launch_bounds__(kWave) void k_mstep(const LaunchArgs a) {
  __shared__ Window win;
  __shared__ Pr<float> ring_p[kRing * kRingW];
  __shared__ Pr<float> ring_r[kRing * kRingW];
  const int b = blockIdx.x;
  const int tile = (b & 7) * a.tiles_per_xcd + (b >> 3);
  if (tile >= a.ntiles) return;
  const int li = a.tile_lattice ? a.tile_lattice[tile] : 0;
  const LatticeDesc* __restrict__ D = a.descs + li;
  const int local_tile = a.tile_lattice ? tile - D->tile_base : tile;
  const int sel = (a.parity ^ D->phase) & 1;
  const bool local = D->local[sel] != 0;  // sources are the site itself
  if (local_tile == 0 && threadIdx.x == 0)
    to_global(const_cast<LatticeDesc*>(D))->local[sel ^ 1] = 0;  // dst is in pull form
  const bool up = ((local_tile / D->g.nstrips) & 1) == 0;  // segments alternate
  mstep_tile<NT>(a, D, local_tile, sel, up, local, win, ring_p, ring_r);
}

// ------------------------------------------------------------- observe ----

// One species' numbers in the LDS window (padded to 32 B).
struct Mom {
  double r, vx, vy, pad;
};

// Equilibrium of direction i at (rho_ref + d, v), minus w_i rho_ref
// (display below Eq. (1), deviation form).
__device__ __forceinline__ double feq_dev(int i, double rref, const Mom& m) {
  const double cu = (double)cx(i) * m.vx + (double)cy(i) * m.vy;
  const double poly = cu * (3.0 + 4.5 * cu) - 1.5 * (m.vx * m.vx + m.vy * m.vy);
  return wq<double>(i) * (m.r + (rref + m.r) * poly);
}

// Observables and fields of the current state, in FP64: the 18 equilibria
// of every site from its sources, rho, j, the forces and u' (pre-collision
// quantities of the step that would follow).
__global__ __launch_bounds__(kWave) void k_mobserve(const LaunchArgs a) {
  using CT = double;
  constexpr int W = kWave + 4;  // ring entries per row
  __shared__ Mom win[3][kWin][2];
  __shared__ Pr<CT> ring_p[kRing * W];
  __shared__ Pr<CT> ring_r[kRing * W];
  const int b = blockIdx.x;
  const int tile = (b & 7) * a.tiles_per_xcd + (b >> 3);
  if (tile >= a.ntiles) return;
  const int li = a.tile_lattice ? a.tile_lattice[tile] : 0;
  const LatticeDesc* __restrict__ D = a.descs + li;
  const Geometry g = D->g;
  const int local_tile = a.tile_lattice ? tile - D->tile_base : tile;
  const int sel = (a.parity ^ D->phase) & 1;
  const int shift = D->local[sel] ? 0 : 1;  // 0: sources are the site itself
  const int strip = local_tile % g.nstrips;
  const int seg = local_tile / g.nstrips;
  const int lane = threadIdx.x;
  const int nx = g.nx, ny = g.ny;
  const int x0 = strip * kWave;
  const int width = min(kWave, nx - x0);
  const int y0 = (int)((long long)seg * ny / g.nsegs);
  const int y1 = (int)((long long)(seg + 1) * ny / g.nsegs);
  const int dir = (seg & 1) ? -1 : 1;
  const bool active = lane < width;
  const int col = active ? x0 + lane : wrap(x0 + lane, nx);
  auto in_row = [&](int c) { return (uint32_t)((c >> 6) * (kPlanes * kWave) + (c & 63)) * 4u; };
  const uint32_t ob_c = in_row(col);
  // halo items: lane t < 36 loads plane t / 6 of halo column t % 6
  const int hc = lane % 6, hp = lane / 6;
  const int hcol = wrap(hc < kHalo ? x0 - kHalo + hc : x0 + width + (hc - kHalo), nx);
  const int hpos = hc < kHalo ? hc : width + kHalo + (hc - kHalo);
  const uint32_t ob_h = in_row(hcol) + (uint32_t)hp * kWave * 4u;
  // ring lanes 0..7: column rc = lane & 3 of species lane >> 2
  const int rcl = lane & 3, rsp = (lane >> 2) & 1;
  const int rpos = rcl < 2 ? rcl : width + rcl;                 // ring position
  const int rwin = rcl < 2 ? 1 + rcl : width + kHalo + (rcl - 2);  // window position

  const Params<CT, true> P(D->c);
  const float* __restrict__ src = (const float*)D->buf[sel];

  const int K = (y1 - y0) + 4;
  const int rstart = dir > 0 ? y0 - 2 : y1 + 1;
  auto lattice_row = [&](int k) {
    const int r = rstart + dir * k;
    return r < 0 ? r + ny : (r >= ny ? r - ny : r);
  };
  // window slot q % 3 holds the row at march position q - 1
  float ld_own[kPlanes], ld_halo;
  auto issue = [&](int q) {
    const float* row = src + (long long)lattice_row(q - 1) * g.row_elems;
#pragma unroll
    for (int p = 0; p < kPlanes; ++p) ld_own[p] = ld_at(row, ob_c + (uint32_t)p * kWave * 4u);
    ld_halo = lane < 2 * kHalo * kPlanes ? ld_at(row, ob_h) : 0.f;
  };
  auto commit = [&](int q) {
    Mom(*w)[2] = win[q % 3];
    if (active) {
      w[lane + kHalo][0] = Mom{(CT)ld_own[0], (CT)ld_own[1], (CT)ld_own[2], CT(0)};
      w[lane + kHalo][1] = Mom{(CT)ld_own[3], (CT)ld_own[4], (CT)ld_own[5], CT(0)};
    }
    if (lane < 2 * kHalo * kPlanes) {
      Mom& m = w[hpos][hp / 3];
      const int cpt = hp % 3;
      if (cpt == 0) m.r = (CT)ld_halo;
      else if (cpt == 1) m.vx = (CT)ld_halo;
      else m.vy = (CT)ld_halo;
    }
  };
  // rho - rho_ref and j of species s at window position pos, pulled row at
  // march position k (sources in rows k-1..k+1 of the window)
  auto gather = [&](int k, int pos, int s, CT& rd, CT& jx, CT& jy, CT* fd) {
    const CT rref = s ? P.rref[1] : P.rref[0];
    rd = jx = jy = CT(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int dy = -cy(i) * shift, dx = -cx(i) * shift;  // source row offset, column offset
      const int slot = (k + 1 + dy * dir + 3) % 3;
      const CT d = feq_dev(i, rref, win[slot][pos + dx][s]);
      if (i == 0) rd = d;
      else rd += d;
      jx += (CT)cx(i) * d;
      jy += (CT)cy(i) * d;
      if (fd) fd[i] = d;
    }
  };

  // pulled moments of three rows and their 18 equilibria
  CT rd[3][2], jxs[3][2], jys[3][2];
  CT fo[3][2][9];
  double acc[kNRed];
#pragma unroll
  for (int m = 0; m < kNRed; ++m) acc[m] = 0.0;
  bool bad = false;

  issue(0);
  commit(0);
  issue(1);
  commit(1);
  issue(2);
  for (int k0 = 0; k0 < K; k0 += 3) {
    static_for<3>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int k = k0 + j;
      if (k >= K) return;
      commit(k + 2);
      lds_fence();
      // sources of row k are in the window: gather, then the next row's loads
      gather(k, lane + kHalo, 0, rd[j][0], jxs[j][0], jys[j][0], fo[j][0]);
      gather(k, lane + kHalo, 1, rd[j][1], jxs[j][1], jys[j][1], fo[j][1]);
      CT rring = CT(0), jdum0, jdum1;
      if (lane < 8) gather(k, rwin, rsp, rring, jdum0, jdum1, nullptr);
      if (k + 3 <= K + 1) issue(k + 3);
      Pr<CT>* rowp = ring_p + (k % kRing) * W;
      Pr<CT>* rowr = ring_r + (k % kRing) * W;
      if (active) {
        rowp[lane + 2] = Pr<CT>{psi_of<CT, true>(P, 0, rd[j][0]), psi_of<CT, true>(P, 1, rd[j][1])};
        rowr[lane + 2] = Pr<CT>{rd[j][0], rd[j][1]};
      }
      if (lane < 8) {
        const CT ps = psi_of<CT, true>(P, rsp, rring);
        if (rsp) {
          rowp[rpos].b = ps;
          rowr[rpos].b = rring;
        } else {
          rowp[rpos].a = ps;
          rowr[rpos].a = rring;
        }
      }
      lds_fence();
      if (k >= 4 && active) {
        constexpr int jc = (j + 1) % 3;  // set of march position k - 2
        int slot[5];
#pragma unroll
        for (int d = 0; d < 5; ++d) slot[d] = (k - 2 + dir * (d - 2)) % kRing;
        auto atp = [&](int dy, int dx) -> const Pr<CT>& {
          return ring_p[slot[dy + 2] * W + lane + 2 + dx];
        };
        auto atr = [&](int dy, int dx) -> const Pr<CT>& {
          return ring_r[slot[dy + 2] * W + lane + 2 + dx];
        };
        const int y = lattice_row(k - 2);
        // forces (Eq. (2)) over the twelve +-c pairs
        CT Sxa = 0, Sya = 0, Sxb = 0, Syb = 0, Xxa = 0, Xya = 0, Xxb = 0, Xyb = 0;
#pragma unroll
        for (int m = 0; m < 12; ++m) {
          const int px = pair_cx(m), py = pair_cy(m), kk = pair_class(m);
          const Pr<CT>& hi = atp(py, px);
          const Pr<CT>& lo = atp(-py, -px);
          const CT da = hi.a - lo.a, db = hi.b - lo.b;
          if (px) {
            Sxa += (P.k[0][kk] * (CT)px) * da;
            Sxb += (P.k[1][kk] * (CT)px) * db;
          }
          if (py) {
            Sya += (P.k[0][kk] * (CT)py) * da;
            Syb += (P.k[1][kk] * (CT)py) * db;
          }
          if (m < 4) {
            const Pr<CT>& rhi = atr(py, px);
            const Pr<CT>& rlo = atr(-py, -px);
            const CT ea = rhi.a - rlo.a, eb = rhi.b - rlo.b;
            if (px) {
              Xxa += (P.kx[kk] * (CT)px) * eb;
              Xxb += (P.kx[kk] * (CT)px) * ea;
            }
            if (py) {
              Xya += (P.kx[kk] * (CT)py) * eb;
              Xyb += (P.kx[kk] * (CT)py) * ea;
            }
          }
        }
        const Pr<CT> c0p = atp(0, 0);
        const CT rho[2] = {P.rref[0] + rd[jc][0], P.rref[1] + rd[jc][1]};
        const CT psi[2] = {P.pref[0] + c0p.a, P.pref[1] + c0p.b};
        CT F[2][2] = {{-psi[0] * Sxa - rho[0] * Xxa, -psi[0] * Sya - rho[0] * Xya},
                      {-psi[1] * Sxb - rho[1] * Xxb, -psi[1] * Syb - rho[1] * Xyb}};
        if (P.g != CT(0) || P.g0 != CT(0)) {
          const CT gy = P.g * sinpi_ct<CT>((CT)y * P.iny2) + P.g0;
          F[0][0] += rho[0] * gy;
          F[1][0] += rho[1] * gy;
        }
        const CT jx[2] = {jxs[jc][0], jxs[jc][1]}, jy[2] = {jys[jc][0], jys[jc][1]};
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
          if (!(rho[sp] > CT(0)) || !(rho[sp] < CT(1e30))) bad = true;
        const CT inv_den = rcp_ct(rho[0] * P.om[0] + rho[1] * P.om[1]);
        const CT ux = (jx[0] * P.om[0] + jx[1] * P.om[1]) * inv_den;
        const CT uy = (jy[0] * P.om[0] + jy[1] * P.om[1]) * inv_den;
        observe_site<CT, true>(a.fields, a.pops, g, P, y, col, rho, jx, jy, F, ux, uy, fo[jc], atr,
                               acc, (a.write_ref || D->has_ref) ? D->phi_ref : nullptr,
                               a.write_ref != 0);
      }
      if (k >= 4) {
        const long long rs = ((long long)lattice_row(k - 2) * g.nstrips + strip) * kNRed;
        wave_sums_store(acc, D->wave_red + rs, lane);
      }
    });
  }
  if (__any(bad) && lane == 0) atomicOr(D->flag, 1);
}

// ---------------------------------------------------------------- init ----

// t = 0 state in local form: rho_s - rho_ref_s and the initial velocity
// (both species) of every site.
__global__ __launch_bounds__(256) void k_moment_init(Geometry g, Coefs c,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ u,
                                                     float* __restrict__ buf) {
  const long long n = (long long)g.nx * g.ny;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int x = (int)(q % g.nx), y = (int)(q / g.nx);
  float* row = buf + (long long)y * g.row_elems + (long long)(x >> 6) * (kPlanes * kWave) + (x & 63);
  const double ux = u ? u[q] : 0.0, uy = u ? u[n + q] : 0.0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    row[(3 * s + 0) * kWave] = (float)(rho[s * n + q] - c.rho_ref[s]);
    row[(3 * s + 1) * kWave] = (float)ux;
    row[(3 * s + 2) * kWave] = (float)uy;
  }
}

}  // namespace

hipError_t launch_moment_step(const LaunchArgs& a, const StepVariant& v, hipStream_t st) {
  const dim3 grid(8 * a.tiles_per_xcd), block(kWave);
  if (v.stream_stores)
    hipLaunchKernelGGL(k_mstep<true>, grid, block, 0, st, a);
  else
    hipLaunchKernelGGL(k_mstep<false>, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_moment_observe(const LaunchArgs& a, hipStream_t st) {
  const dim3 grid(8 * a.tiles_per_xcd), block(kWave);
  hipLaunchKernelGGL(k_mobserve, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_moment_init(const Geometry& g, const Coefs& c, const double* rho,
                              const double* u, void* buf, hipStream_t st) {
  const long long n = (long long)g.nx * g.ny;
  hipLaunchKernelGGL(k_moment_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, c, rho,
                     u, (float*)buf);
  return hipGetLastError();
}

}  // namespace lbk
