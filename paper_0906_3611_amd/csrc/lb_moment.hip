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
// A step gathers the 6 numbers of each site's 9 sources, forms rho_s and
// j_s from their equilibria, the forces of Eq. (2), u' and v_s, and writes
// the site's own 6 numbers: 48 B per site update in FP32 instead of 144 B.
// Right after an initialization the buffer is in "local" form (a flag per
// buffer): f_is(r, 0) = f^eq_i(M_s(r)), the zero-step equilibrium state of
// Sec. VI; the first step reads it that way and clears the flag of the
// buffer it writes.
//
// Layout: row y is pitch / 64 blocks of 64 sites, each block holding 6 runs
// of 64 FP32 values: rho_A - rho_ref_A, v_Ax, v_Ay, rho_B - rho_ref_B, v_Bx,
// v_By.
//
// Decomposition as in lb_kernels.hip: one wavefront per (64-column strip,
// row segment) tile marching along its rows; the 6 numbers of three source
// rows (with 3 halo columns on each side) sit in an LDS window, rho and psi
// of five rows in the LDS ring, and the row two behind is collided.
#include "lb_device.h"

namespace lbk {
namespace {

constexpr int kPlanes = 6;
constexpr int kHalo = 3;                  // window columns beyond the strip, each side
constexpr int kWin = kWave + 2 * kHalo;  // window entries per row

// One species' numbers in the LDS window (padded to 16 B for FP32).
template <typename CT>
struct Mom {
  CT r, vx, vy, pad;
};

// Equilibrium of direction i at (rho_ref + d, v), minus w_i rho_ref
// (display below Eq. (1), deviation form).
template <typename CT>
__device__ __forceinline__ CT feq_dev(int i, CT rref, const Mom<CT>& m) {
#pragma clang fp contract(on)
  const CT cu = (CT)cx(i) * m.vx + (CT)cy(i) * m.vy;
  const CT poly = cu * (CT(3) + CT(4.5) * cu) - CT(1.5) * (m.vx * m.vx + m.vy * m.vy);
  return wq<CT>(i) * (m.r + (rref + m.r) * poly);
}

template <typename CT, int MODE, bool NT>
__global__ __launch_bounds__(kWave) void k_moment(const LaunchArgs a) {
  // Multiply-adds are fused only within one source expression: the march
  // loop is unrolled three times, and free fusion could round a site
  // differently depending on which copy (row position) processes it.
#pragma clang fp contract(on)
  constexpr int W = kWave + 4;  // ring entries per row
  __shared__ Mom<CT> win[3][kWin][2];
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
  float* __restrict__ dst = (float*)D->buf[sel ^ 1];
  if (MODE == kStep && local_tile == 0 && lane == 0)
    to_global(const_cast<LatticeDesc*>(D))->local[sel ^ 1] = 0;  // dst is in pull form

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
    Mom<CT>(*w)[2] = win[q % 3];
    if (active) {
      w[lane + kHalo][0] = Mom<CT>{(CT)ld_own[0], (CT)ld_own[1], (CT)ld_own[2], CT(0)};
      w[lane + kHalo][1] = Mom<CT>{(CT)ld_own[3], (CT)ld_own[4], (CT)ld_own[5], CT(0)};
    }
    if (lane < 2 * kHalo * kPlanes) {
      Mom<CT>& m = w[hpos][hp / 3];
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
      const CT d = feq_dev<CT>(i, rref, win[slot][pos + dx][s]);
      if (i == 0) rd = d;
      else rd += d;
      jx += (CT)cx(i) * d;
      jy += (CT)cy(i) * d;
      if (fd) fd[i] = d;
    }
  };

  // pulled moments of three rows (and, observing, the 18 equilibria)
  CT rd[3][2], jxs[3][2], jys[3][2];
  CT fo[MODE == kObserve ? 3 : 1][2][9];
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
      CT* fdo = MODE == kObserve ? fo[j % (MODE == kObserve ? 3 : 1)][0] : nullptr;
      gather(k, lane + kHalo, 0, rd[j][0], jxs[j][0], jys[j][0], fdo);
      gather(k, lane + kHalo, 1, rd[j][1], jxs[j][1], jys[j][1],
             MODE == kObserve ? fo[j % (MODE == kObserve ? 3 : 1)][1] : nullptr);
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
        if (P.g != CT(0)) {
          const CT gy = P.g * sinpi_ct<CT>((CT)y * P.iny2);
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
        if (MODE == kObserve) {
          observe_site<CT, true>(a.fields, a.pops, g, P, y, col, rho, jx, jy, F, ux, uy,
                                 fo[jc % (MODE == kObserve ? 3 : 1)], atr, acc);
        } else {
          // post-collision numbers: rho unchanged, v_s = u' + tau_s F_s / rho_s
          float* row = dst + (long long)y * g.row_elems;
#pragma unroll
          for (int sp = 0; sp < 2; ++sp) {
            const CT ir = rcp_ct(rho[sp]);
            const CT vx = ux + P.tau[sp] * F[sp][0] * ir;
            const CT vy = uy + P.tau[sp] * F[sp][1] * ir;
            st_at<NT>(row, ob_c + (uint32_t)(3 * sp + 0) * kWave * 4u, (float)rd[jc][sp]);
            st_at<NT>(row, ob_c + (uint32_t)(3 * sp + 1) * kWave * 4u, (float)vx);
            st_at<NT>(row, ob_c + (uint32_t)(3 * sp + 2) * kWave * 4u, (float)vy);
          }
        }
      }
      if (MODE == kObserve && k >= 4) {
        const long long rs = ((long long)lattice_row(k - 2) * g.nstrips + strip) * kNRed;
#pragma unroll
        for (int m = 0; m < kNRed; ++m) {
          double v = acc[m];
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
          if (lane == 0) D->wave_red[rs + m] = v;
          acc[m] = 0.0;
        }
      }
    });
  }
  if (__any(bad) && lane == 0) atomicOr(D->flag, 1);
}

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
    hipLaunchKernelGGL((k_moment<float, kStep, true>), grid, block, 0, st, a);
  else
    hipLaunchKernelGGL((k_moment<float, kStep, false>), grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_moment_observe(const LaunchArgs& a, hipStream_t st) {
  const dim3 grid(8 * a.tiles_per_xcd), block(kWave);
  hipLaunchKernelGGL((k_moment<double, kObserve, false>), grid, block, 0, st, a);
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
