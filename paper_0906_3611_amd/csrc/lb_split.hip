// Step kernel with one wavefront per species (population storage, FP32
// deviations, periodic or with moving walls; FP64 measured no faster than
// k_march and is not built here).
//
// The tiles, memory layout and march are those of k_march (lb_kernels.hip):
// a workgroup owns a 64-column strip and a segment of rows and marches
// along it, keeping rho and psi of five rows in an LDS ring.  Here the
// workgroup has two wavefronts, wave s handling species s for all 64
// columns: it pulls the 9 populations of its species (Eq. (1) LHS), forms
// rho_s and psi_s (Eq. (5)), and, for the row two behind, the force on its
// species (Eq. (2); the cross term reads the other species' density from
// the ring) and the BGK update of its 9 populations.  The common velocity
// u' couples the species: each wave puts the j_s of every row it pulls in
// LDS and both evaluate u' by the same expression in the same order.  Per wave this halves the
// registers and the instruction stream of a row, so twice as many waves
// share the work and hide each other's latency; the HBM traffic is the
// same.
#include "lb_device.h"

namespace lbk {
namespace {

// NSUB tiles of adjacent strips of one segment share a workgroup (2 NSUB
// waves, one barrier per row across all of them) and one set of LDS ring
// rows spanning their columns: a tile's ring columns are then its
// neighbours' own columns, and only the group's first and last tile load
// ring items (its outer columns); on periodic lattices larger than the
// Infinity Cache the remaining side loads hit lines the same CU has just
// fetched.  Grouped launches need every lattice of the launch to
// have a multiple of NSUB strips, so that a group's tiles lie in one
// segment and march equally far.  Each wave checks that once its first
// loads are in flight; a group that does not satisfy it leaves as a whole,
// before any barrier, and raises flag bit 2 (reported by the host as a
// launch error).
template <typename ST, typename CT, bool DEV, bool WALLS, int PF, bool NT, int NSUB>
__global__ __launch_bounds__(2 * kWave * NSUB) void k_split(const LaunchArgs a) {
  // Multiply-adds are fused only within one source expression, so every
  // unrolled copy of the march rounds a site alike.
#pragma clang fp contract(on)
  constexpr int W = kWave * NSUB + 4;  // ring entries per row: the group's columns and 2 each side
  constexpr int NSET = 3 + PF;     // pulled rows held in registers
  constexpr int kItems = 4 * 9;    // ring items of one species: 4 columns x 9 directions
  // One barrier per row (after both waves have written it), so a wave can
  // run one row ahead of the other: the ring keeps 6 rows (5 are read) and
  // the momenta 4 (row k - 2 is read while row k + 1 may be written).
  constexpr int kSRing = 6, kJRing = 4;
  // psi and rho of the stencil rows, [species][slot][pos]: species-major so
  // that a wave reading one species hits consecutive banks
  __shared__ CT ring_p[2][kSRing * W];
  __shared__ CT ring_r[2][kSRing * W];
  __shared__ CT rstage_[NSUB][2][kItems];       // pulled ring items of the current row, per species
  __shared__ CT xj_[NSUB][kJRing][2][2][kWave];  // j_x, j_y of a pulled row, per species
  __shared__ double wmom_[NSUB][2][2][kWave];   // walls: x momentum to [species][wall] per lane
  const int sub = NSUB > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 7) : 0;
  auto& rstage = rstage_[sub];
  auto& xj = xj_[sub];
  auto& wmom = wmom_[sub];
  const int b = blockIdx.x;
  const int ngroups = a.ntiles / NSUB;
  const int gpx = NSUB > 1 ? (ngroups + 7) / 8 : a.tiles_per_xcd;  // groups per XCD
  const int group = (b & 7) * gpx + (b >> 3);
  if (group >= ngroups) return;  // the whole workgroup leaves together
  const int tile = group * NSUB + sub;
  const int li = a.tile_lattice ? a.tile_lattice[tile] : 0;
  const LatticeDesc* __restrict__ D = a.descs + li;
  const Geometry g = D->g;
  const int local = a.tile_lattice ? tile - D->tile_base : tile;
  const int sel = (a.parity ^ D->phase) & 1;
  const int strip = local % g.nstrips;
  const int seg = local / g.nstrips;
  const int s = __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) & 1);  // species of this wave
  // (readfirstlane: provably uniform, so per-species values live in scalar registers)
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = g.nx, ny = g.ny;
  const int x0 = strip * kWave;
  const int width = min(kWave, nx - x0);
  const int y0 = (int)((long long)seg * ny / g.nsegs);
  const int y1 = (int)((long long)(seg + 1) * ny / g.nsegs);
  const int dir = (seg & 1) ? -1 : 1;
  const bool active = lane < width;
  const int col = active ? x0 + lane : wrap(x0 + lane, nx);
  constexpr uint32_t esz = sizeof(ST);
  auto in_row = [&](int c) { return (uint32_t)((c >> 6) * (18 * kWave) + (c & 63)) * esz; };
  const uint32_t ob_c = in_row(col);
  // ring item of this lane (lanes 0..35): column rc of x0 - 2, x0 - 1,
  // x0 + w, x0 + w + 1, direction ri; its source column and in-row offset
  const int rc = lane & 3;
  // ring columns are loaded only at the group's outer edges: the left ones by
  // its first tile, the right ones by its last; the others are the
  // neighbouring tiles' own columns in the shared ring rows
  const bool need_l = sub == 0, need_r = sub == NSUB - 1;
  const bool rl = lane < kItems && (rc < 2 ? need_l : need_r);
  const int ri = lane < kItems ? lane >> 2 : 0;
  const int rcol = wrap(rc < 2 ? x0 - 2 + rc : x0 + width + (rc - 2), nx);
  const int rsrc = wrap(rcol - cx(ri), nx);
  const int rdy = cy(ri);
  // walls: the wall-buffer link of a ring item whose source is the wall
  const int rj = (ri == 2 || ri == 4) ? 0 : ((ri == 5 || ri == 7) ? 1 : 2);
  const uint32_t rob =
      (uint32_t)((rsrc >> 6) * (18 * kWave) + (s * 9 + ri) * kWave + (rsrc & 63)) * esz;
  // lanes 0..3 sum the ring column rc = lane; its ring position
  const int gpos = kWave * sub;  // this tile's first column in the ring rows, less 2
  const int rpos = gpos + (lane < 2 ? lane : width + lane);
  const bool rsum = lane < 4 && (lane < 2 ? need_l : need_r);  // lanes that sum a ring column
  // The own pulls load each direction's run aligned (lane = column, one
  // 256-byte run of the 64-site block) and move the c_x = +-1 directions by
  // one lane in registers: loads shifted by a column straddle two blocks and
  // cost the cache hierarchy far more.  Lanes 0 and 63 take their missing
  // neighbour (columns x0 - 1 and x0 + 64) from edge items loaded by lanes
  // 36..41 with the ring items: directions 1, 5, 8 at x0 - 1 and 3, 6, 7 at
  // x0 + 64.  (In a ragged strip the first lane past the strip already holds
  // the right neighbour column, wrapped.)
  const bool el = lane >= kItems && lane < kItems + 6;
  const int ee = lane - kItems;
  const int edir = ee < 3 ? (ee == 0 ? 1 : (ee == 1 ? 5 : 8)) : (ee == 3 ? 3 : (ee == 4 ? 6 : 7));
  const int ecol = wrap(ee < 3 ? x0 - 1 : x0 + kWave, nx);
  // this lane's side load (ring item or edge item): source row offset and in-row offset
  const int sdy = el ? cy(edir) : rdy;
  const uint32_t sob =
      el ? (uint32_t)((ecol >> 6) * (18 * kWave) + (s * 9 + edir) * kWave + (ecol & 63)) * esz : rob;
  const bool sl = rl || el;
  const bool lane0 = lane == 0, lane63 = lane == kWave - 1;

  const Params<CT, DEV> P(D->c);
  const ST* __restrict__ src = (const ST*)D->buf[sel];
  ST* __restrict__ dst = (ST*)D->buf[sel ^ 1];
  const ST* __restrict__ wall_in = (const ST*)D->wall[sel];
  ST* __restrict__ wall_out = (ST*)D->wall[sel ^ 1];
  if (WALLS) {  // a tile reaches each wall row at most once; lanes off the lattice add 0
    wmom[s][0][lane] = 0.0;
    wmom[s][1][lane] = 0.0;
  }
  // per-species constants (selects: a uniform index into P would move it to memory)
  const CT rref = s ? P.rref[1] : P.rref[0];
  const CT pref = s ? P.pref[1] : P.pref[0];
  const CT tau = s ? P.tau[1] : P.tau[0];
  const CT om = s ? P.om[1] : P.om[0];
  CT ks[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) ks[c] = s ? P.k[1][c] : P.k[0][c];

  CT fr[NSET][9];  // pulled rows of this species, set k % NSET for march row k
  ST rv[NSET];     // this lane's ring item of those rows
  bool bad = false;
  const int K = (y1 - y0) + 4;
  const int rstart = dir > 0 ? y0 - 2 : y1 + 1;
  auto lattice_row = [&](int k) {
    const int r = rstart + dir * k;
    if (WALLS) return r < 0 ? -1 - r : (r >= ny ? 2 * ny - 1 - r : r);  // mirrored ghost rows
    return r < 0 ? r + ny : (r >= ny ? r - ny : r);
  };
  auto pull_row = [&](int k, CT (&f)[9], ST& v) {
    const int re = lattice_row(k);
    int rm, rp;
    if (WALLS) {
      rm = re > 0 ? re - 1 : 0;  // row 0's c_y = +1 links come from the wall buffer
      rp = re < ny - 1 ? re + 1 : ny - 1;
    } else {
      rm = re > 0 ? re - 1 : ny - 1;
      rp = re < ny - 1 ? re + 1 : 0;
    }
    {
      const int row = sdy > 0 ? rm : (sdy < 0 ? rp : re);
      v = sl ? ld_at(src + (long long)row * g.row_elems, sob) : ST(0);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int row = cy(i) > 0 ? rm : (cy(i) < 0 ? rp : re);
      const ST* base = src + (long long)row * g.row_elems + (s * 9 + i) * kWave;
      f[i] = (CT)ld_at(base, ob_c);
    }
    // c_x = +1 comes from the column to the left, c_x = -1 from the right
    static_for<9>([&](auto I) {
      constexpr int i = decltype(I)::value;
      if constexpr (cx(i) != 0) {
        constexpr int e = cx(i) > 0 ? (i == 1 ? 0 : (i == 5 ? 1 : 2)) : (i == 3 ? 3 : (i == 6 ? 4 : 5));
        constexpr int ctrl = cx(i) > 0 ? 0x138 : 0x130;  // DPP wave_shr:1 / wave_shl:1
        const float edge = __builtin_bit_cast(
            float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, (float)v), kItems + e));
        const int moved =
            __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, (float)f[i]), ctrl, 0xF, 0xF, false);
        f[i] = (CT)((cx(i) > 0 ? lane0 : lane63) ? edge : __builtin_bit_cast(float, moved));
      }
    });
    if (WALLS && (re == 0 || re == ny - 1)) {  // a wall row (uniform): links from the wall buffer
      const int wl = re == 0 ? 0 : 1;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const CT w = (CT)to_global(wall_in)[((wl * 2 + s) * 3 + j) * nx + col];
        if (wl) f[wall_in_dir(1, j)] = w;
        else f[wall_in_dir(0, j)] = w;
      }
      if (rl && (wl ? rdy < 0 : rdy > 0)) v = to_global(wall_in)[((wl * 2 + s) * 3 + rj) * nx + rcol];
    }
  };

  static_for<PF>([&](auto Q) {
    constexpr int q = decltype(Q)::value;
    if (q < K) pull_row(q, fr[q], rv[q]);
  });
  if (NSUB > 1) {
    // the group's tiles are consecutive: its first and last tile in one
    // lattice and one segment put all of them there (the same for every wave)
    const int t0 = group * NSUB, t1 = t0 + NSUB - 1;
    const int l0 = a.tile_lattice ? a.tile_lattice[t0] : 0;
    const int l1 = a.tile_lattice ? a.tile_lattice[t1] : 0;
    bool same = l0 == l1;
    if (same) {
      const LatticeDesc* __restrict__ D0 = a.descs + l0;
      const int base = a.tile_lattice ? D0->tile_base : 0;
      same = (t0 - base) / D0->g.nstrips == (t1 - base) / D0->g.nstrips;
    }
    if (!__builtin_amdgcn_readfirstlane(same)) {
      if (threadIdx.x == 0) atomicOr(D->flag, 2);
      return;  // every wave of the group
    }
  }
  for (int k0 = 0; k0 < K; k0 += NSET) {
    static_for<NSET>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const int k = k0 + j;
      if (k >= K) return;
      // From the row's start to the row barrier (and, with prefetch, to the
      // issue of row k + PF's loads just after it) the wave runs at a
      // raised priority: the workgroup's waves meet at that barrier, so the
      // slowest one's way to it paces them all, while the collision after it
      // can give way to the SIMD's other waves.
      __builtin_amdgcn_s_setprio(3);
      if (!PF) pull_row(k, fr[j], rv[j]);
      // rho_s and psi_s of the pulled row into ring slot k % kSRing; the ring
      // items go through LDS to lanes 0..3, which sum them in the same order
      CT rho = fr[j][0];
#pragma unroll
      for (int i = 1; i < 9; ++i) rho += fr[j][i];
      const CT psi = psi_of<CT, DEV>(P, s, rho);
      if (rl) rstage[s][lane] = (CT)rv[j];
      {
        const CT(&f)[9] = fr[j];
        xj[k % kJRing][s][0][lane] = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
        xj[k % kJRing][s][1][lane] = (f[2] - f[4]) + (f[5] - f[8]) + (f[6] - f[7]);
      }
      lds_fence();
      const int slot = k % kSRing;
      if (active) {
        ring_p[s][slot * W + gpos + lane + 2] = psi;
        ring_r[s][slot * W + gpos + lane + 2] = rho;
      }
      if (rsum) {
        CT acc = rstage[s][lane];
#pragma unroll
        for (int i = 1; i < 9; ++i) acc += rstage[s][4 * i + lane];
        ring_p[s][slot * W + rpos] = psi_of<CT, DEV>(P, s, acc);
        ring_r[s][slot * W + rpos] = acc;
      }
      __syncthreads();  // both species' row k is in the ring
      if (PF && k + PF < K) pull_row(k + PF, fr[(j + PF) % NSET], rv[(j + PF) % NSET]);
      __builtin_amdgcn_s_setprio(0);
      if (k >= 4) {
        constexpr int jc = (j + NSET - 2) % NSET;  // set of march row k - 2
        const CT(&f)[9] = fr[jc];
        int rows[5];
#pragma unroll
        for (int d = 0; d < 5; ++d) rows[d] = ((k - 2 + dir * (d - 2)) % kSRing) * W + gpos + lane + 2;
        auto psi_at = [&](int dy, int dx, int sp) { return ring_p[sp][rows[dy + 2] + dx]; };
        auto rho_at = [&](int dy, int dx, int sp) { return ring_r[sp][rows[dy + 2] + dx]; };
        const int y = lattice_row(k - 2);
        const int so = s ^ 1;
        // forces (Eq. (2)) on species s over the twelve +-c pairs
        CT Sx = 0, Sy = 0, Xx = 0, Xy = 0;
        if (active) {
#pragma unroll
          for (int m = 0; m < 12; ++m) {
            const int px = pair_cx(m), py = pair_cy(m), kk = pair_class(m);
            const CT d = psi_at(py, px, s) - psi_at(-py, -px, s);
            if (px) Sx += (ks[kk] * (CT)px) * d;
            if (py) Sy += (ks[kk] * (CT)py) * d;
            if (m < 4) {
              const CT e = rho_at(py, px, so) - rho_at(-py, -px, so);  // the other species acts
              if (px) Xx += (P.kx[kk] * (CT)px) * e;
              if (py) Xy += (P.kx[kk] * (CT)py) * e;
            }
          }
          const int jr = (k - 2) % kJRing;
          const CT J0x = xj[jr][0][0][lane], J1x = xj[jr][1][0][lane];
          const CT J0y = xj[jr][0][1][lane], J1y = xj[jr][1][1][lane];
          const CT c0a = rho_at(0, 0, 0), c0b = rho_at(0, 0, 1);
          const CT rho0 = DEV ? P.rref[0] + c0a : c0a, rho1 = DEV ? P.rref[1] + c0b : c0b;
          const CT drho = s ? c0b : c0a;  // deviation (DEV) or density of species s
          const CT rho_s = s ? rho1 : rho0;
          const CT psi_s = DEV ? pref + psi_at(0, 0, s) : psi_at(0, 0, s);
          CT Fx = -psi_s * Sx - rho_s * Xx, Fy = -psi_s * Sy - rho_s * Xy;
          if (P.g != CT(0) || P.g0 != CT(0))
            Fx += rho_s * (P.g * sinpi_ct<CT>((CT)y * P.iny2) + P.g0);
          if (!(rho_s > CT(0)) || !(rho_s < CT(1e30))) bad = true;
          // common velocity (Eq. (1) and the definition of u below it)
          const CT inv_den = rcp_ct(rho0 * P.om[0] + rho1 * P.om[1]);
          const CT ux = (J0x * P.om[0] + J1x * P.om[1]) * inv_den;
          const CT uy = (J0y * P.om[0] + J1y * P.om[1]) * inv_den;
          // BGK relaxation towards the equilibrium at v_s = u' + tau_s F_s / rho_s
          const CT ir = rcp_ct(rho_s);
          const CT vx = ux + tau * Fx * ir;
          const CT vy = uy + tau * Fy * ir;
          const CT usq = CT(1.5) * (vx * vx + vy * vy);
          ST* row = dst + (long long)y * g.row_elems + (s * 9) * kWave;
          CT post[9];
#pragma unroll
          for (int i = 1; i < 9; ++i) {
            const CT cu = (CT)cx(i) * vx + (CT)cy(i) * vy;
            const CT poly = cu * (CT(3) + CT(4.5) * cu) - usq;
            const CT feq = DEV ? wq<CT>(i) * (drho + rho_s * poly) : wq<CT>(i) * rho_s * (CT(1) + poly);
            post[i] = f[i] + om * (feq - f[i]);
          }
          // The collision keeps each species' mass (the equilibrium's zeroth
          // moment is rho_s).  In FP32 the weights 4/9, 1/9, 1/36 round to
          // values summing to 1 + 7.45e-9, so an FP32 equilibrium moved a
          // site's deviation mass by that fraction every step: down in the
          // phase where the deviation is negative, up in the other, which
          // left a drift in the total.  The rest population therefore takes
          // what the site held before the collision minus its eight moving
          // populations, summed in FP64 (exact for the spans met here): the
          // site's mass then changes by the final rounding alone.
          {
            double before = (double)f[0], moved = 0.0;
#pragma unroll
            for (int i = 1; i < 9; ++i) {
              before += (double)f[i];
              moved += (double)post[i];
            }
            post[0] = (CT)(before - moved);
          }
#pragma unroll
          for (int i = 0; i < 9; ++i) st_at<NT>(row + i * kWave, ob_c, (ST)post[i]);
          if (WALLS && (y == 0 || y == ny - 1)) {
            // the links leaving towards a wall return with the moving-wall
            // term (halfway bounce-back); their x momentum goes to the wall
            const int wl = y == ny - 1 ? 1 : 0;
            const CT uwall = wl ? P.uw : -P.uw;
            double mom = 0.0;
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
              const int o0 = wall_out_dir(0, jj), o1 = wall_out_dir(1, jj);
              const CT po = wl ? post[o1] : post[o0];
              const int cxo = wl ? cx(o1) : cx(o0);
              const CT corr = CT(6) * wq<CT>(o0) * rho_s * ((CT)cxo * uwall);
              to_global(wall_out)[((wl * 2 + s) * 3 + jj) * nx + col] = (ST)(po - corr);
              const double full = (double)po + (DEV ? wq<double>(o0) * (double)rref : 0.0);
              mom += (double)cxo * (2.0 * full - (double)corr);
            }
            wmom[s][wl][lane] = mom;
          }
        }
      }
    });
  }
  if (__any(bad) && lane == 0) atomicOr(D->flag, 1);
  if (WALLS && a.accumulate_wall && (y0 == 0 || y1 == ny)) {  // uniform over the workgroup
    // wall momentum of this strip: per lane species A + species B, then a
    // fixed lane tree; slot (strip, wall), added to only by the tile holding
    // that wall's row
    __syncthreads();
    if (s == 0) {
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        if (m == 0 ? y0 != 0 : y1 != ny) continue;
        double v = wmom[0][m][lane] + wmom[1][m][lane];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) D->wave_wall[(long long)strip * 2 + m] += v;
      }
    }
  }
}

template <bool WALLS, int PF, bool NT, int NSUB>
hipError_t launch_split_t(const LaunchArgs& a, hipStream_t st) {
  if (a.ntiles % NSUB) return hipErrorInvalidValue;
  const int gpx = NSUB > 1 ? (a.ntiles / NSUB + 7) / 8 : a.tiles_per_xcd;
  hipLaunchKernelGGL((k_split<float, float, true, WALLS, PF, NT, NSUB>), dim3(8 * gpx),
                     dim3(2 * kWave * NSUB), 0, st, a);
  return hipGetLastError();
}

template <bool WALLS, int NSUB>
hipError_t launch_split_w(const LaunchArgs& a, const StepVariant& v, hipStream_t st) {
  if (v.prefetch >= 2)
    return v.stream_stores ? launch_split_t<WALLS, 2, true, NSUB>(a, st)
                           : launch_split_t<WALLS, 2, false, NSUB>(a, st);
  if (v.prefetch == 1)
    return v.stream_stores ? launch_split_t<WALLS, 1, true, NSUB>(a, st)
                           : launch_split_t<WALLS, 1, false, NSUB>(a, st);
  return v.stream_stores ? launch_split_t<WALLS, 0, true, NSUB>(a, st)
                         : launch_split_t<WALLS, 0, false, NSUB>(a, st);
}

}  // namespace

hipError_t launch_split_step(const LaunchArgs& a, bool fp64, bool walls, const StepVariant& v,
                             hipStream_t st) {
  if (fp64) return hipErrorInvalidValue;  // FP32 deviation storage only
  if (v.group == kGroupTiles)
    return walls ? launch_split_w<true, kGroupTiles>(a, v, st) : launch_split_w<false, kGroupTiles>(a, v, st);
  if (v.group > 1) return hipErrorInvalidValue;
  return walls ? launch_split_w<true, 1>(a, v, st) : launch_split_w<false, 1>(a, v, st);
}

}  // namespace lbk
