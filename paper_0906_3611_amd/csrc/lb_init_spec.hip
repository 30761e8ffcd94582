// Initial conditions from a compact specification (host side): the
// disc-emulsion state, and the C ABI entry points that use it.
//
// Random numbers: counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA
// 2014): output k (k = 1, 2, ...) of a generator seeded with `seed` is the
// finalizer applied to seed + k * 0x9E3779B97F4A7C15 (mod 2^64); a uniform
// double in [0, 1) is its top 53 bits times 2^-53.
#include "lb.h"
#include "lb_engine.h"

#include <cfenv>
#include <algorithm>
#include <cmath>
#include <vector>

namespace {

constexpr uint64_t kDiscCounterBase = 1ull << 48;

uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t seed, uint64_t k) { return (double)(splitmix64(seed, k) >> 11) * 0x1.0p-53; }

}  // namespace

namespace lbe {

// Union of random discs covering at least a fraction phi of an nx x ny
// periodic lattice.  Disc k has centre (nx U0, ny U1) and radius
// rmin + (rmax - rmin) U2, U_j = draw kDiscCounterBase + 3k + j + 1; a site
// is inside when its minimum-image distance to the centre is <= the radius;
// discs are added until the covered count reaches phi nx ny.
int disc_mask(int nx, int ny, uint64_t seed, double phi, double rmin, double rmax,
              std::vector<unsigned char>& mask) {
#pragma clang fp contract(off)
  if (!(phi >= 0.0 && phi <= 1.0) || !(rmin > 0.0) || !(rmax >= rmin) || !std::isfinite(rmax))
    return LB_E_INVAL;
  mask.assign((size_t)nx * ny, 0);
  const double target = phi * (double)nx * (double)ny;
  long long covered = 0;
  const int saved = std::fegetround();
  std::fesetround(FE_TONEAREST);  // nearbyint rounds half to even
  for (uint64_t k = 0; (double)covered < target; ++k) {
    if (k >= 10000000ull) {
      std::fesetround(saved);
      return LB_E_INVAL;
    }
    const uint64_t c = kDiscCounterBase + 3 * k;
    const double cx = nx * uniform01(seed, c + 1);
    const double cy = ny * uniform01(seed, c + 2);
    const double r = rmin + (rmax - rmin) * uniform01(seed, c + 3);
    const long long ri = (long long)std::ceil(r) + 1;
    const long long x0 = (long long)std::floor(cx) - ri, x1 = (long long)std::floor(cx) + ri + 2;
    const long long y0 = (long long)std::floor(cy) - ri, y1 = (long long)std::floor(cy) + ri + 2;
    const bool no_dup = (x1 - x0) <= nx && (y1 - y0) <= ny;
    const double r2 = r * r;
    for (long long ys = y0; ys < y1; ++ys) {
      double dy = (double)ys - cy;
      dy = dy - ny * std::nearbyint(dy / ny);
      const int yi = (int)(((ys % ny) + ny) % ny);
      for (long long xs = x0; xs < x1; ++xs) {
        double dx = (double)xs - cx;
        dx = dx - nx * std::nearbyint(dx / nx);
        if (dy * dy + dx * dx <= r2) {
          const int xi = (int)(((xs % nx) + nx) % nx);
          unsigned char& m = mask[(size_t)yi * nx + xi];
          if (!m) {
            m = 1;
            if (no_dup) ++covered;
          }
        }
      }
    }
    if (!no_dup) {
      covered = 0;
      for (unsigned char v : mask) covered += v;
    }
  }
  std::fesetround(saved);
  return LB_OK;
}

int disc_fields(int nx, int ny, uint64_t seed, double phi, double rmin, double rmax, double in_a,
                double in_b, double out_a, double out_b, std::vector<double>& ra,
                std::vector<double>& rb) {
  std::vector<unsigned char> m;
  const int rc = disc_mask(nx, ny, seed, phi, rmin, rmax, m);
  if (rc != LB_OK) return rc;
  ra.resize(m.size());
  rb.resize(m.size());
  for (size_t k = 0; k < m.size(); ++k) {
    ra[k] = m[k] ? in_a : out_a;
    rb[k] = m[k] ? in_b : out_b;
  }
  return LB_OK;
}

}  // namespace lbe

extern "C" {

int lb_disc_fields(int32_t nx, int32_t ny, uint64_t seed, double phi, double rmin, double rmax,
                   double in_a, double in_b, double out_a, double out_b, double* rho_a,
                   double* rho_b) {
  if (nx < 1 || ny < 1 || !rho_a || !rho_b) return LB_E_INVAL;
  std::vector<double> ra, rb;
  const int rc = lbe::disc_fields(nx, ny, seed, phi, rmin, rmax, in_a, in_b, out_a, out_b, ra, rb);
  if (rc != LB_OK) return rc;
  std::copy(ra.begin(), ra.end(), rho_a);
  std::copy(rb.begin(), rb.end(), rho_b);
  return LB_OK;
}

int lb_init_discs(lb_lattice* L, uint64_t seed, double phi, double rmin, double rmax, double in_a,
                  double in_b, double out_a, double out_b) {
  if (!L) return LB_E_INVAL;
  const auto& g = L->e.m[0].d.g;
  std::vector<double> ra, rb;
  const int rc = lbe::disc_fields(g.nx, g.ny, seed, phi, rmin, rmax, in_a, in_b, out_a, out_b, ra, rb);
  if (rc != LB_OK) return L->e.fail(rc, "invalid disc specification");
  return lbe::engine_init(L->e, 0, ra.data(), rb.data(), nullptr, nullptr);
}

int lb_batch_init_discs(lb_batch* B, int32_t i, uint64_t seed, double phi, double rmin,
                        double rmax, double in_a, double in_b, double out_a, double out_b) {
  if (!B) return LB_E_INVAL;
  if (i < 0 || i >= (int)B->e.m.size()) return B->e.fail(LB_E_INVAL, "lattice index out of range");
  const auto& g = B->e.m[i].d.g;
  std::vector<double> ra, rb;
  const int rc = lbe::disc_fields(g.nx, g.ny, seed, phi, rmin, rmax, in_a, in_b, out_a, out_b, ra, rb);
  if (rc != LB_OK) return B->e.fail(rc, "invalid disc specification");
  return lbe::engine_init(B->e, i, ra.data(), rb.data(), nullptr, nullptr);
}

}  // extern "C"
