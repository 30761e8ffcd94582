// HIP kernels for gfx950 of the two-species Shan-Chen lattice Boltzmann step
// (Benzi et al., arXiv:0906.3611, Sec. II).
//
// Layout.  Populations are stored in "pull" form: the buffer for time t
// holds, at site q and direction i, the post-collision value that site
// q + c_i pulls when it streams into time t.  Each lattice row is a run of
// 64-site blocks, each block holding its 18 populations as 18 runs of 64
// values (pop_index in lb_internal.h), so a wavefront reads and writes one
// contiguous block per row instead of 18 separate planes.
// A step reads one buffer and writes the other (ping-pong).  Under moving
// walls the three links of a wall-adjacent site that come back from the
// wall are kept in a small side buffer [wall][s][link][nx], written by the
// collision that sends them out.
//
// Decomposition.  One 64-lane wavefront owns a line-aligned strip of 64
// columns and marches along a segment of rows.  For every row it pulls the
// 18 populations (2 species x 9 directions) of its columns and of the two
// ring columns on each side, forms rho_s and psi_s into a 5-row LDS ring,
// and collides the row two behind, whose 25-point stencil is then complete.
// Pulled populations stay in registers until their collision, so every
// population is read from HBM once per step apart from the ring re-reads,
// which neighbouring strips and segments bring into L2 at the same time.
// This kernel steps FP64 lattices and observes every population-storage
// lattice; FP32 deviation storage steps with one wavefront per species
// (lb_split.hip).
#include "lb_device.h"

#include <algorithm>

namespace lbk {
namespace {

// Source rows of a pull into lattice row re: rm for c_y = +1, rp for c_y = -1.
template <bool WALLS>
__device__ __forceinline__ void source_rows(int re, int ny, int& rm, int& rp) {
  if (WALLS) {
    rm = re > 0 ? re - 1 : 0;  // row 0's c_y = +1 links come from the wall buffer
    rp = re < ny - 1 ? re + 1 : ny - 1;
  } else {
    rm = re > 0 ? re - 1 : ny - 1;
    rp = re < ny - 1 ? re + 1 : 0;
  }
}

// Pull the 18 populations streaming into row re at column col.  ob_m / ob_c
// / ob_p are the in-row byte offsets (block and lane, population 0) of the
// source columns col - 1, col, col + 1
// (sources of c_x = +1, 0, -1).
template <typename ST, typename CT, bool WALLS>
__device__ __forceinline__ void pull(const Geometry& g, const ST* __restrict__ src,
                                     const ST* __restrict__ wall_in, int re, uint32_t ob_m,
                                     uint32_t ob_c, uint32_t ob_p, int col, CT (&f)[2][9]) {
  int rm, rp;
  source_rows<WALLS>(re, g.ny, rm, rp);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int row = cy(i) > 0 ? rm : (cy(i) < 0 ? rp : re);
      const uint32_t ob = cx(i) > 0 ? ob_m : (cx(i) < 0 ? ob_p : ob_c);
      const ST* base = src + (long long)row * g.row_elems + (s * 9 + i) * kWave;
      f[s][i] = (CT)ld_at(base, ob);
    }
    if (WALLS) {
      if (re == 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
          f[s][wall_in_dir(0, j)] = (CT)to_global(wall_in)[((0 * 2 + s) * 3 + j) * g.nx + col];
      }
      if (re == g.ny - 1) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
          f[s][wall_in_dir(1, j)] = (CT)to_global(wall_in)[((1 * 2 + s) * 3 + j) * g.nx + col];
      }
    }
  }
}

// Density and pseudopotential of a pulled row (Sec. II; Eq. (5)).  With
// deviation storage the LDS record holds deviations from the reference,
// d_s = rho_s - rho_ref_s = sum_i delta_is and psi_s - psi(rho_ref_s), so
// that stencil differences lose no digits to the common background.
template <typename CT, bool DEV>
__device__ __forceinline__ Fld<CT> make_fields(const Params<CT, DEV>& P, const CT (&f)[2][9]) {
  CT r[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    CT acc = f[s][0];
#pragma unroll
    for (int i = 1; i < 9; ++i) acc += f[s][i];
    r[s] = acc;
  }
  Fld<CT> o;
  o.ra = r[0];
  o.rb = r[1];
  o.pa = psi_of<CT, DEV>(P, 0, r[0]);
  o.pb = psi_of<CT, DEV>(P, 1, r[1]);
  return o;
}

// Ring columns of a strip: x0 - 2, x0 - 1, x0 + w, x0 + w + 1 (w = strip
// width), wrapped periodically.
__device__ __forceinline__ int ring_col(int rc, int x0, int width, int nx) {
  return wrap(rc < 2 ? x0 - 2 + rc : x0 + width + (rc - 2), nx);
}

// Pull of the ring columns, shared by the whole wave: the 72 values
// (4 columns x 2 species x 9 directions) of lattice row re are items
// t = 4 (9 s + i) + rc, t = lane and t = 64 + lane (lanes 0..7).  The
// sources follow the same rules as pull().
template <typename ST, bool WALLS>
__device__ __forceinline__ void ring_pull(const Geometry& g, const ST* __restrict__ src,
                                          const ST* __restrict__ wall_in, int re, int x0,
                                          int width, int lane, ST (&v)[2]) {
  int rm, rp;
  source_rows<WALLS>(re, g.ny, rm, rp);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int t = lane + kWave * h;
    v[h] = ST(0);
    if (h == 1 && lane >= 8) continue;
    const int rc = t & 3, p = t >> 2;
    const int s = p >= 9 ? 1 : 0, i = p - 9 * s;
    const int c = ring_col(rc, x0, width, g.nx);
    const int dy = cy(i);
    if (WALLS && ((re == 0 && dy > 0) || (re == g.ny - 1 && dy < 0))) {
      const int wl = re == 0 ? 0 : 1;
      const int j = (i == 2 || i == 4) ? 0 : ((i == 5 || i == 7) ? 1 : 2);
      v[h] = to_global(wall_in)[((wl * 2 + s) * 3 + j) * g.nx + c];
    } else {
      int sc = c - cx(i);
      sc = sc < 0 ? sc + g.nx : (sc >= g.nx ? sc - g.nx : sc);
      const int row = dy > 0 ? rm : (dy < 0 ? rp : re);
      const long long off = (long long)row * g.row_elems + (long long)(sc >> 6) * (18 * kWave) +
                            (long long)(p * kWave + (sc & 63));
      v[h] = to_global(src)[off];
    }
  }
}

// Collide the sites of lattice row y whose stencil rows sit in LDS ring
// slots slot[0..4] (dy = -2..2).  Lane l owns LDS column l + 2.
// Per-wave output context of a collision.
template <typename ST>
struct Out {
  Geometry g;
  ST* dst;        // populations for t + 1
  ST* wall_out;   // wall links for t + 1
  double* fields;  // observe outputs (single-lattice launches)
  double* pops;
  double* phi_ref;  // observe: the reference order parameter, or null
  bool write_ref;   // observe: store phi as the reference first
};

template <typename CT, bool DEV, bool WALLS, int MODE, typename ST, bool NT>
__device__ __forceinline__ void collide_row(const Out<ST>& a, const Params<CT, DEV>& P,
                                            const Pr<CT>* __restrict__ ring_p,
                                            const Pr<CT>* __restrict__ ring_r, int lc,
                                            const int (&slot)[5], int y, int col, uint32_t ob_c,
                                            const CT (&f)[2][9], double (&acc)[kNRed],
                                            double (&wacc)[2], bool& bad) {
  const Geometry& g = a.g;
  constexpr int W = kWave + 4;
  auto atp = [&](int dy, int dx) -> const Pr<CT>& { return ring_p[slot[dy + 2] * W + lc + dx]; };
  auto atr = [&](int dy, int dx) -> const Pr<CT>& { return ring_r[slot[dy + 2] * W + lc + dx]; };
  // Shan-Chen sums over +-c pairs (Eq. (2)): S_s = sum_i k_s(i) psi_s(r + c_i) c_i,
  // X_s = sum_{belt 1} (G_AB / rho0^2) w_i rho_other(r + c_i) c_i.
  CT Sxa = 0, Sya = 0, Sxb = 0, Syb = 0, Xxa = 0, Xya = 0, Xxb = 0, Xyb = 0;
#pragma unroll
  for (int m = 0; m < 12; ++m) {
    const int px = pair_cx(m), py = pair_cy(m), k = pair_class(m);
    const Pr<CT>& hi = atp(py, px);
    const Pr<CT>& lo = atp(-py, -px);
    const CT da = hi.a - lo.a, db = hi.b - lo.b;
    if (px) {
      Sxa += (P.k[0][k] * (CT)px) * da;
      Sxb += (P.k[1][k] * (CT)px) * db;
    }
    if (py) {
      Sya += (P.k[0][k] * (CT)py) * da;
      Syb += (P.k[1][k] * (CT)py) * db;
    }
    if (m < 4) {
      const Pr<CT>& rhi = atr(py, px);
      const Pr<CT>& rlo = atr(-py, -px);
      const CT ea = rhi.a - rlo.a, eb = rhi.b - rlo.b;  // A's density acts on B and back
      if (px) {
        Xxa += (P.kx[k] * (CT)px) * eb;
        Xxb += (P.kx[k] * (CT)px) * ea;
      }
      if (py) {
        Xya += (P.kx[k] * (CT)py) * eb;
        Xyb += (P.kx[k] * (CT)py) * ea;
      }
    }
  }
  const Pr<CT> c0p = atp(0, 0), c0r = atr(0, 0);
  // centre values (deviation records add the references back)
  const CT rho[2] = {DEV ? P.rref[0] + c0r.a : c0r.a, DEV ? P.rref[1] + c0r.b : c0r.b};
  const CT psi[2] = {DEV ? P.pref[0] + c0p.a : c0p.a, DEV ? P.pref[1] + c0p.b : c0p.b};
  CT F[2][2] = {{-psi[0] * Sxa - rho[0] * Xxa, -psi[0] * Sya - rho[0] * Xya},
                {-psi[1] * Sxb - rho[1] * Xxb, -psi[1] * Syb - rho[1] * Xyb}};
  // body forces along x (row-uniform): the shear forcing of Sec. VIII,
  // rho_s g sin(2 pi y / ny), and a uniform rho_s g0
  if (P.g != CT(0) || P.g0 != CT(0)) {
    const CT gy = P.g * sinpi_ct<CT>((CT)y * P.iny2) + P.g0;
    F[0][0] += rho[0] * gy;
    F[1][0] += rho[1] * gy;
  }
  // moments and the common velocity (Eq. (1) and the definition of u below it)
  CT jx[2], jy[2];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    jx[sp] = (f[sp][1] - f[sp][3]) + (f[sp][5] - f[sp][6]) + (f[sp][8] - f[sp][7]);
    jy[sp] = (f[sp][2] - f[sp][4]) + (f[sp][5] - f[sp][8]) + (f[sp][6] - f[sp][7]);
    if (!(rho[sp] > CT(0)) || !(rho[sp] < CT(1e30))) bad = true;
  }
  const CT inv_den = rcp_ct(rho[0] * P.om[0] + rho[1] * P.om[1]);
  const CT ux = (jx[0] * P.om[0] + jx[1] * P.om[1]) * inv_den;
  const CT uy = (jy[0] * P.om[0] + jy[1] * P.om[1]) * inv_den;

  if (MODE == kObserve) {
    observe_site<CT, DEV>(a.fields, a.pops, g, P, y, col, rho, jx, jy, F, ux, uy, f, atr, acc,
                          a.phi_ref, a.write_ref);
    return;
  }

  ST* __restrict__ dst = a.dst;
  double mom = 0;
  const bool wall_row = WALLS && (y == 0 || y == g.ny - 1);
  const int wl = (WALLS && y == g.ny - 1) ? 1 : 0;
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    // BGK relaxation towards the equilibrium at v_s = u' + tau_s F_s / rho_s
    const CT ir = rcp_ct(rho[sp]);
    const CT vx = ux + P.tau[sp] * F[sp][0] * ir;
    const CT vy = uy + P.tau[sp] * F[sp][1] * ir;
    const CT usq = CT(1.5) * (vx * vx + vy * vy);
    const CT drho = DEV ? (sp == 0 ? c0r.a : c0r.b) : CT(0);  // sum of the deviations
    CT post[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const CT cu = (CT)cx(i) * vx + (CT)cy(i) * vy;
      const CT poly = cu * (CT(3) + CT(4.5) * cu) - usq;
      // f^eq_i = w_i rho (1 + poly); deviation form: f^eq_i - w_i rho_ref = w_i (d + rho poly)
      const CT feq = DEV ? wq<CT>(i) * (drho + rho[sp] * poly) : wq<CT>(i) * rho[sp] * (CT(1) + poly);
      post[i] = f[sp][i] + P.om[sp] * (feq - f[sp][i]);
      const ST* b = dst + (long long)y * g.row_elems + (sp * 9 + i) * kWave;
      st_at<NT>(const_cast<ST*>(b), ob_c, (ST)post[i]);
    }
    if (WALLS && wall_row) {
      const CT uwall = wl ? P.uw : -P.uw;
      ST* wall_out = a.wall_out;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        // the j-th link leaves along o and returns as wall_in_dir:
        // f_back = f*_o - 2 w_o rho_w (c_o . u_w) / c_s^2, rho_w = rho_s(r, t).
        // o is wall_out_dir(wl, j); both walls' o share the weight class.
        const int o0 = wall_out_dir(0, j), o1 = wall_out_dir(1, j);
        const CT po = wl ? post[o1] : post[o0];
        const int cxo = wl ? cx(o1) : cx(o0);
        const CT corr = CT(6) * wq<CT>(o0) * rho[sp] * ((CT)cxo * uwall);
        to_global(wall_out)[((wl * 2 + sp) * 3 + j) * g.nx + col] = (ST)(po - corr);
        const double full = (double)po + (DEV ? wq<double>(o0) * (double)P.rref[sp] : 0.0);
        mom += (double)cxo * (2.0 * full - (double)corr);
      }
    }
  }
  if (WALLS && wall_row) wacc[wl] += mom;
}

// One wavefront per (strip, segment) tile.  Lane l owns column x0 + l of a
// 64-column strip (line-aligned); lanes 0..3 also pull the four ring columns
// x0 - 2, x0 - 1, x0 + w, x0 + w + 1 (w = strip width).  Even segments
// march up the rows, odd ones down, so two neighbouring segments reach
// their shared ring rows at the same time and the second read hits L2.
// PF > 0 keeps the pulls of the next PF rows in flight during the current
// row's work (the loads of row k + PF are issued before the collision of
// row k - 2).
template <typename ST, typename CT, bool DEV, bool WALLS, int MODE, int PF, bool NT>
__global__ __launch_bounds__(kWave) void k_march(const LaunchArgs a) {
  constexpr int W = kWave + 4;
  constexpr int NSET = 3 + PF;
  __shared__ Pr<CT> ring_p[kRing * W];  // psi of the 5 stencil rows
  __shared__ Pr<CT> ring_r[kRing * W];  // rho of the 5 stencil rows
  __shared__ CT rstage[72];  // pulled ring-column values of the current row
  const int b = blockIdx.x;
  const int tile = (b & 7) * a.tiles_per_xcd + (b >> 3);
  if (tile >= a.ntiles) return;
  // the lattice of this tile and its record (uniform: scalar loads)
  const int li = a.tile_lattice ? a.tile_lattice[tile] : 0;
  const LatticeDesc* __restrict__ D = a.descs + li;
  const Geometry g = D->g;
  // batch launches number tiles across lattices; single-lattice launches
  // (tile_lattice null) number the lattice's own tiles from 0
  const int local = a.tile_lattice ? tile - D->tile_base : tile;
  const int sel = (a.parity ^ D->phase) & 1;
  const int strip = local % g.nstrips;
  const int seg = local / g.nstrips;
  const int lane = threadIdx.x;
  const int nx = g.nx, ny = g.ny;
  const int x0 = strip * kWave;
  const int width = min(kWave, nx - x0);
  const int y0 = (int)((long long)seg * ny / g.nsegs);
  const int y1 = (int)((long long)(seg + 1) * ny / g.nsegs);
  // Adjacent segments march towards each other, and every segment turns
  // round at each step (sel alternates), so a step first reads the rows the
  // previous step wrote last: with buffers a little larger than the 256 MB
  // Infinity Cache those are still there (with plain stores).  Each site's
  // arithmetic does not depend on the direction.
  const int dir = ((seg ^ sel) & 1) ? -1 : 1;
  const bool active = lane < width;
  // interior column (inactive lanes read a valid duplicate column)
  const int col = active ? x0 + lane : wrap(x0 + lane, nx);
  const uint32_t esz = sizeof(ST);
  auto in_row = [&](int c) { return (uint32_t)((c >> 6) * (18 * kWave) + (c & 63)) * esz; };
  const uint32_t ob_c = in_row(col);
  const uint32_t ob_m = in_row(col == 0 ? nx - 1 : col - 1);
  const uint32_t ob_p = in_row(col == nx - 1 ? 0 : col + 1);
  // ring lanes 0..7: column rc = lane & 3 of species lane >> 2, at LDS
  // position 0, 1 (left) or w + 2, w + 3 (right)
  const int rcl = lane & 3, rsp = (lane >> 2) & 1;
  const int rpos = rcl < 2 ? rcl : width + rcl;

  const Params<CT, DEV> P(D->c);
  const ST* __restrict__ src = (const ST*)D->buf[sel];
  const ST* __restrict__ wall_in = (const ST*)D->wall[sel];
  const bool ref_on = MODE == kObserve && (a.write_ref || D->has_ref);
  const Out<ST> out{g, (ST*)D->buf[sel ^ 1], (ST*)D->wall[sel ^ 1], a.fields, a.pops,
                    ref_on ? D->phi_ref : nullptr, a.write_ref != 0};

  CT fr[NSET][2][9];  // pulled rows, set k % NSET for march row k
  ST ri[NSET][2];     // this lane's ring items of those rows
  double acc[kNRed];
#pragma unroll
  for (int m = 0; m < kNRed; ++m) acc[m] = 0.0;
  double wacc[2] = {0.0, 0.0};
  bool bad = false;
  const int K = (y1 - y0) + 4;  // field rows pulled: the segment plus two ring rows each side
  const int rstart = dir > 0 ? y0 - 2 : y1 + 1;

  auto lattice_row = [&](int k) {
    const int r = rstart + dir * k;
    if (WALLS) return r < 0 ? -1 - r : (r >= ny ? 2 * ny - 1 - r : r);  // mirrored ghost rows
    return r < 0 ? r + ny : (r >= ny ? r - ny : r);
  };
  auto pull_row = [&](int k, CT (&dstf)[2][9], ST (&dri)[2]) {
    const int re = lattice_row(k);
    pull<ST, CT, WALLS>(g, src, wall_in, re, ob_m, ob_c, ob_p, col, dstf);
    ring_pull<ST, WALLS>(g, src, wall_in, re, x0, width, lane, dri);
  };

  // PF rows are in flight ahead of the row whose fields are being formed
  static_for<PF>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    if (q < K) pull_row(q, fr[q], ri[q]);
  });
  for (int k0 = 0; k0 < K; k0 += NSET) {
    static_for<NSET>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int k = k0 + j;
      if (k >= K) return;
      if (!PF) pull_row(k, fr[j], ri[j]);
      // fields of the pulled row into LDS slot k % 5; the ring columns'
      // values go through LDS to lanes 0..7, one (column, species) each,
      // which sum them in the order make_fields uses
      const Fld<CT> fl = make_fields<CT, DEV>(P, fr[j]);
      rstage[lane] = (CT)ri[j][0];
      if (lane < 8) rstage[kWave + lane] = (CT)ri[j][1];
      lds_fence();
      Pr<CT>* rowp = ring_p + (k % kRing) * W;
      Pr<CT>* rowr = ring_r + (k % kRing) * W;
      if (active) {
        rowp[lane + 2] = Pr<CT>{fl.pa, fl.pb};
        rowr[lane + 2] = Pr<CT>{fl.ra, fl.rb};
      }
      if (lane < 8) {
        CT acc = rstage[(rsp * 9) * 4 + rcl];
#pragma unroll
        for (int i = 1; i < 9; ++i) acc += rstage[(rsp * 9 + i) * 4 + rcl];
        const CT ps = psi_of<CT, DEV>(P, rsp, acc);
        if (rsp) {
          rowp[rpos].b = ps;
          rowr[rpos].b = acc;
        } else {
          rowp[rpos].a = ps;
          rowr[rpos].a = acc;
        }
      }
      lds_fence();
      if (PF && k + PF < K) pull_row(k + PF, fr[(j + PF) % NSET], ri[(j + PF) % NSET]);
      if (k >= 4 && active) {
        int slot[5];
#pragma unroll
        for (int d = 0; d < 5; ++d) slot[d] = (k - 2 + dir * (d - 2)) % kRing;
        const int y = lattice_row(k - 2);
        collide_row<CT, DEV, WALLS, MODE, ST, NT>(out, P, ring_p, ring_r, lane + 2, slot, y, col, ob_c,
                                              fr[(j + NSET - 2) % NSET], acc, wacc, bad);
      }
      if (MODE == kObserve && k >= 4) {
        // partials of this strip row (fixed lane tree), stored by (row,
        // strip): the totals do not depend on how rows are cut into segments
        const long long rs = ((long long)lattice_row(k - 2) * g.nstrips + strip) * kNRed;
        wave_sums_store(acc, D->wave_red + rs, lane);
      }
    });
  }

  if (__any(bad) && lane == 0) atomicOr(D->flag, 1);
  if (MODE == kStep && WALLS && a.accumulate_wall) {
    // wall momentum of this strip: slot (strip, wall), added to only by the
    // tile holding that wall's row
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (m == 0 ? y0 != 0 : y1 != ny) continue;
      double v = wacc[m];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) D->wave_wall[(long long)strip * 2 + m] += v;
    }
  }
}

// Fixed-order reduction of a lattice's partials, in two passes.  Slots are
// (row, strip) for observables (kNRed values each) and strips for the wall
// momentum (2 values), so the order below depends only on the lattice's
// size: the result is the same bit for bit alone or in a batch, and for any
// segment height.
// Pass 1: workgroup (c, lattice) takes chunk c of kRedChunk slots; thread t
// sums slots t, t + kRedT, ... of the chunk in order, all WIDTH values of a
// slot at once (a wave reads contiguous runs), then a fixed binary tree per
// value.  A lattice of one chunk is done; otherwise the chunk's sums go to
// the chunk's own first slot, which no other workgroup reads (the observe
// partials are rewritten by every observe pass).  The wall accumulators
// carry on across steps, so they are never overwritten: they form one
// chunk whatever their number.
// Pass 2: one workgroup per lattice of several chunks sums the chunk sums
// the same way (thread t: chunks t, t + kRedT, ...; then the tree).
constexpr int kRedT = 1024;
constexpr long long kRedChunk = 8LL * kRedT;

__device__ __forceinline__ long long red_slots(const LatticeDesc* D, int width) {
  return width == kNRed ? (long long)D->g.ny * D->g.nstrips : (long long)D->g.nstrips;
}

// Sum of v over the workgroup's threads by a fixed tree; the result in sh[0].
__device__ __forceinline__ void red_tree(double* sh, double v) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int h = kRedT / 2; h >= 1; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
}

template <int WIDTH>
__global__ __launch_bounds__(kRedT) void k_reduce_chunks(const LatticeDesc* __restrict__ descs,
                                                         double* __restrict__ out, int out_stride) {
  __shared__ double sh[kRedT];
  const LatticeDesc* D = descs + blockIdx.y;
  const long long nslots = red_slots(D, WIDTH);
  const long long nchunks = WIDTH == kNRed ? (nslots + kRedChunk - 1) / kRedChunk : 1;
  if (blockIdx.x > 0 && (long long)blockIdx.x >= nchunks) return;  // uniform
  double* in = WIDTH == kNRed ? D->wave_red : D->wave_wall;
  const long long lo = (long long)blockIdx.x * kRedChunk;
  const long long hi = WIDTH == kNRed ? min(nslots, lo + kRedChunk) : nslots;
  double v[WIDTH];
#pragma unroll
  for (int m = 0; m < WIDTH; ++m) v[m] = 0.0;
#pragma unroll 4
  for (long long t = lo + threadIdx.x; t < hi; t += kRedT) {
#pragma unroll
    for (int m = 0; m < WIDTH; ++m) v[m] += in[t * WIDTH + m];
  }
  double r[WIDTH];
#pragma unroll
  for (int m = 0; m < WIDTH; ++m) {
    red_tree(sh, v[m]);  // every read of the chunk precedes its first barrier
    r[m] = sh[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < WIDTH; ++m) {
      if (nchunks <= 1) out[(long long)blockIdx.y * out_stride + m] = r[m];
      else in[lo * WIDTH + m] = r[m];
    }
  }
}

template <int WIDTH>
__global__ __launch_bounds__(kRedT) void k_reduce_sums(const LatticeDesc* __restrict__ descs,
                                                       double* __restrict__ out, int out_stride) {
  __shared__ double sh[kRedT];
  static_assert(WIDTH == kNRed, "only the observe partials are reduced in two passes");
  const LatticeDesc* D = descs + blockIdx.x;
  const long long nchunks = (red_slots(D, WIDTH) + kRedChunk - 1) / kRedChunk;
  if (nchunks <= 1) return;
  const double* __restrict__ in = D->wave_red;
  double v[WIDTH];
#pragma unroll
  for (int m = 0; m < WIDTH; ++m) v[m] = 0.0;
  for (long long c = threadIdx.x; c < nchunks; c += kRedT) {
#pragma unroll
    for (int m = 0; m < WIDTH; ++m) v[m] += in[c * kRedChunk * WIDTH + m];
  }
#pragma unroll 1
  for (int m = 0; m < WIDTH; ++m) {
    red_tree(sh, v[m]);
    if (threadIdx.x == 0) out[(long long)blockIdx.x * out_stride + m] = sh[0];
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
      buf[pop_index(g.row_elems, s, i, y, x)] = (ST)value(s, i, xs, ys);
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

template <int MODE, int PF, bool NT>
hipError_t launch_march(const LaunchArgs& a, bool fp64, bool walls, hipStream_t st) {
  const dim3 grid(8 * a.tiles_per_xcd), block(kWave);
  if (fp64) {
    if (walls)
      hipLaunchKernelGGL((k_march<double, double, false, true, MODE, PF, NT>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_march<double, double, false, false, MODE, PF, NT>), grid, block, 0, st, a);
  } else if constexpr (MODE == kStep) {
    return hipErrorInvalidValue;  // FP32 deviation storage steps in k_split (lb_split.hip)
  } else {
    // observation of FP32 deviation storage is evaluated in FP64
    if (walls)
      hipLaunchKernelGGL((k_march<float, double, true, true, MODE, PF, NT>), grid, block, 0, st, a);
    else
      hipLaunchKernelGGL((k_march<float, double, true, false, MODE, PF, NT>), grid, block, 0, st, a);
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

hipError_t launch_step(const LaunchArgs& a, bool fp64, bool walls, const StepVariant& v,
                       hipStream_t st) {
  if (v.prefetch >= 2)
    return v.stream_stores ? launch_march<kStep, 2, true>(a, fp64, walls, st)
                           : launch_march<kStep, 2, false>(a, fp64, walls, st);
  if (v.prefetch == 1)
    return v.stream_stores ? launch_march<kStep, 1, true>(a, fp64, walls, st)
                           : launch_march<kStep, 1, false>(a, fp64, walls, st);
  return v.stream_stores ? launch_march<kStep, 0, true>(a, fp64, walls, st)
                         : launch_march<kStep, 0, false>(a, fp64, walls, st);
}

hipError_t launch_observe(const LaunchArgs& a, bool fp64, bool walls, hipStream_t st) {
  return launch_march<kObserve, 0, false>(a, fp64, walls, st);
}

hipError_t launch_reduce_lattices(const LatticeDesc* descs, int n, int which, double* out,
                                  int out_stride, long long max_slots, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long chunks = which ? 1 : std::max(1LL, (max_slots + kRedChunk - 1) / kRedChunk);
  if (n > 65535 || chunks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g1((unsigned)chunks, (unsigned)n);
  if (which)
    hipLaunchKernelGGL(k_reduce_chunks<2>, g1, dim3(kRedT), 0, st, descs, out, out_stride);
  else
    hipLaunchKernelGGL(k_reduce_chunks<kNRed>, g1, dim3(kRedT), 0, st, descs, out, out_stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || chunks == 1) return e;
  hipLaunchKernelGGL(k_reduce_sums<kNRed>, dim3(n), dim3(kRedT), 0, st, descs, out, out_stride);
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
