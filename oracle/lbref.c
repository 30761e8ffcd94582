/*
 * lbref.c -- plain FP64 CPU oracle for one time step of the two-species
 * Shan-Chen lattice Boltzmann model of Benzi, Sbragaglia, Succi, Bernaschi
 * and Chibbaro, "Mesoscopic lattice Boltzmann modeling of soft-glassy
 * systems: theory and simulations" (arXiv:0906.3611).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  It is deliberately slow and direct: every step of the
 * method is its own loop over the lattice, in the order the paper states it,
 * with no blocking, fusion or pair-summing.  It shares no source, header,
 * table or helper with the GPU library, and only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.
 *
 * Build: gcc -O2 -std=c11 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * (no FMA contraction: every product and sum is rounded as written).
 *
 * State layout: f[s][i][y][x], s in {0=A, 1=B}, i the D2Q9 direction, x fastest.
 * f holds the pre-collision populations at integer time t.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NS 2   /* species A, B */
#define NQ 9   /* D2Q9 kinetic velocities */
#define NE 25  /* interaction speeds: rest + belt 1 (8) + belt 2 (16) */

/* ------------------------------------------------------------------------ */
/* Lattice constants.                                                        */
/* ------------------------------------------------------------------------ */

/* D2Q9 kinetic set, sound speed c_s^2 = 1/3 (Sec. II, Eq. (4)).  The
 * equilibrium weights are the D2Q9 ones of Table I (w_0 = 4/9, 1/9 on the
 * axes, 1/36 on the diagonals).  Order: rest, +x, +y, -x, -y, then the four
 * diagonals counter-clockwise from (1,1). */
static const int    CX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int    CY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WQ[NQ] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                              1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

/* 25-speed interaction lattice (Sec. II, Table I and Fig. 2).  Index 0 is the
 * rest speed, 1..8 the first belt (the same vectors as the D2Q9 set above),
 * 9..24 the second belt: 9..12 the (+-2,0),(0,+-2) speeds, 13..20 the
 * (+-2,+-1),(+-1,+-2) speeds and 21..24 the (+-2,+-2) speeds.  PE holds the
 * repulsion weights p_i of Table I; WE holds the attraction / cross weights
 * w_i of Table I, which exist on the first belt only. */
static const int EX[NE] = {0, 1, 0, -1, 0, 1, -1, -1, 1,
                           2, 0, -2, 0,
                           2, 1, -1, -2, -2, -1, 1, 2,
                           2, -2, -2, 2};
static const int EY[NE] = {0, 0, 1, 0, -1, 1, 1, -1, -1,
                           0, 2, 0, -2,
                           1, 2, 2, 1, -1, -2, -2, -1,
                           2, 2, -2, -2};
static const double PE[NE] = {
    247.0 / 420.0,
    4.0 / 63.0,  4.0 / 63.0,  4.0 / 63.0,  4.0 / 63.0,
    4.0 / 135.0, 4.0 / 135.0, 4.0 / 135.0, 4.0 / 135.0,
    1.0 / 180.0, 1.0 / 180.0, 1.0 / 180.0, 1.0 / 180.0,
    2.0 / 945.0, 2.0 / 945.0, 2.0 / 945.0, 2.0 / 945.0,
    2.0 / 945.0, 2.0 / 945.0, 2.0 / 945.0, 2.0 / 945.0,
    1.0 / 15120.0, 1.0 / 15120.0, 1.0 / 15120.0, 1.0 / 15120.0};
static const double WE[NE] = {
    4.0 / 9.0,
    1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

static int opposite(int i) {
  for (int k = 0; k < NQ; ++k)
    if (CX[k] == -CX[i] && CY[k] == -CY[i]) return k;
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Parameters.                                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t nx, ny;
  int32_t walls;    /* 0: periodic in y.  1: halfway bounce-back walls at
                       y = -1/2 (moving with x-velocity -u_wall) and at
                       y = ny - 1/2 (moving with +u_wall).  x is periodic. */
  int32_t pad_;
  double tau[NS];   /* relaxation times tau_s (Eq. (1)) */
  double rho0;      /* pseudopotential density scale (Eq. (5)) */
  double Ga[NS];    /* G^a_s, belt-1 intra-species coupling (Eq. (2)) */
  double Gr[NS];    /* G^r_s, belt-1+2 intra-species coupling (Eq. (2)) */
  double Gab;       /* G_AB = G_BA, belt-1 cross coupling (Eq. (2)) */
  double u_wall;    /* wall speed for walls == 1 */
  double g_body;    /* amplitude of the volumetric shear forcing of Sec. VIII:
                       each species feels rho_s g(y) along x with
                       g(y) = g_body sin(2 pi y / ny), the force that drives
                       U_x = U0 sin(k y), k = 2 pi / ny (first mode) */
  double g_uniform; /* uniform body force per unit mass along x: each species
                       feels rho_s g_uniform (the same kind of volumetric force
                       as the shear forcing, constant in space; between the
                       walls it drives plane Poiseuille flow) */
} lbref_params;

static const double TWO_PI = 6.283185307179586476925286766559;

#define IDX(p, y, x) ((size_t)(y) * (size_t)(p)->nx + (size_t)(x))
#define FI(p, f, s, i, y, x) \
  (f)[(((size_t)(s) * NQ + (size_t)(i)) * (size_t)(p)->ny + (size_t)(y)) * (size_t)(p)->nx + (size_t)(x)]

static size_t nsites(const lbref_params* p) { return (size_t)p->nx * (size_t)p->ny; }

/* Neighbour row for the force stencil.  Periodic: wrap.  Walls: the density
 * and pseudopotential fields are mirrored across the wall plane, so the ghost
 * row at y = -1 repeats row 0, y = -2 repeats row 1, and likewise at the top. */
static int stencil_row(const lbref_params* p, int y) {
  if (!p->walls) return ((y % p->ny) + p->ny) % p->ny;
  if (y < 0) return -1 - y;
  if (y >= p->ny) return 2 * p->ny - 1 - y;
  return y;
}
static int wrap_x(const lbref_params* p, int x) { return ((x % p->nx) + p->nx) % p->nx; }

/* ------------------------------------------------------------------------ */
/* The steps of one time step, each its own pass.                            */
/* ------------------------------------------------------------------------ */

/* Species density rho_s = sum_i f_is (Sec. II, below Eq. (1)). */
void lbref_density(const lbref_params* p, const double* f, double* rho) {
  const size_t n = nsites(p);
  for (int s = 0; s < NS; ++s)
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        double r = 0.0;
        for (int i = 0; i < NQ; ++i) r += FI(p, f, s, i, y, x);
        rho[s * n + IDX(p, y, x)] = r;
      }
}

/* Pseudopotential psi(rho) = rho0 (1 - exp(-rho/rho0)) with a common rho0
 * for both species (Sec. II, Eq. (5)). */
void lbref_psi(const lbref_params* p, const double* rho, double* psi) {
  const size_t n = nsites(p);
  for (size_t k = 0; k < NS * n; ++k) psi[k] = p->rho0 * (1.0 - exp(-rho[k] / p->rho0));
}

/* Force on each species (Sec. II, Eq. (2)):
 *   F^a_s = -G^a_s psi_s(r) sum_{belt 1} w_i psi_s(r + c_i) c_i
 *   F^r_s = -G^r_s psi_s(r) sum_{belt 1} p_i psi_s(r + c_i) c_i
 *           -G^r_s psi_s(r) sum_{belt 2} p_i psi_s(r + c_i) c_i
 *   F^X_s = -(1/rho0^2) rho_s(r) sum_{s' != s} sum_{belt 1} G_ss' w_i rho_s'(r + c_i) c_i
 * F[s][a][y][x], a = 0 (x) or 1 (y).  Each of the three terms is summed on
 * its own, over its neighbours in table order, then the three are added. */
void lbref_force(const lbref_params* p, const double* rho, const double* psi, double* F) {
  const size_t n = nsites(p);
  for (int s = 0; s < NS; ++s) {
    const int so = 1 - s;
    const double* ps = psi + (size_t)s * n;
    const double* rs = rho + (size_t)s * n;
    const double* ro = rho + (size_t)so * n;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        double att[2] = {0, 0}, rep1[2] = {0, 0}, rep2[2] = {0, 0}, crs[2] = {0, 0};
        for (int i = 1; i < NE; ++i) {
          const size_t nb = IDX(p, stencil_row(p, y + EY[i]), wrap_x(p, x + EX[i]));
          const double c[2] = {(double)EX[i], (double)EY[i]};
          for (int a = 0; a < 2; ++a) {
            if (i <= 8) {
              att[a] += WE[i] * ps[nb] * c[a];
              rep1[a] += PE[i] * ps[nb] * c[a];
              crs[a] += p->Gab * WE[i] * ro[nb] * c[a];
            } else {
              rep2[a] += PE[i] * ps[nb] * c[a];
            }
          }
        }
        const size_t k = IDX(p, y, x);
        const double gy = p->g_body * sin(TWO_PI * (double)y / (double)p->ny) + p->g_uniform;
        for (int a = 0; a < 2; ++a) {
          const double Fa = -p->Ga[s] * ps[k] * att[a];
          const double Fr = -p->Gr[s] * ps[k] * rep1[a] - p->Gr[s] * ps[k] * rep2[a];
          const double FX = -(1.0 / (p->rho0 * p->rho0)) * rs[k] * crs[a];
          const double Fb = a == 0 ? rs[k] * gy : 0.0; /* body forces (Sec. VIII) */
          F[((size_t)s * 2 + a) * n + k] = Fa + Fr + FX + Fb;
        }
      }
  }
}

/* Second-order equilibrium (Sec. II, display below Eq. (1)):
 *   f^eq_i(rho, v) = w_i rho [1 + (v.c_i)/c_s^2 + (c_ia c_ib - c_s^2 delta_ab) v_a v_b / (2 c_s^4)]. */
static double feq(int i, double rho, double vx, double vy) {
  const double cu = CX[i] * vx + CY[i] * vy;
  const double quad = ((CX[i] * CX[i] - CS2) * vx * vx + 2.0 * CX[i] * CY[i] * vx * vy +
                       (CY[i] * CY[i] - CS2) * vy * vy) / (2.0 * CS2 * CS2);
  return WQ[i] * rho * (1.0 + cu / CS2 + quad);
}

/* Common velocity u' = sum_s (1/tau_s) sum_i f_is c_i / sum_s rho_s / tau_s
 * (Sec. II, below Eq. (1)).  u[a][y][x]. */
void lbref_common_velocity(const lbref_params* p, const double* f, const double* rho, double* u) {
  const size_t n = nsites(p);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      const size_t k = IDX(p, y, x);
      double num[2] = {0, 0}, den = 0;
      for (int s = 0; s < NS; ++s) {
        double j[2] = {0, 0};
        for (int i = 0; i < NQ; ++i) {
          j[0] += FI(p, f, s, i, y, x) * CX[i];
          j[1] += FI(p, f, s, i, y, x) * CY[i];
        }
        num[0] += j[0] / p->tau[s];
        num[1] += j[1] / p->tau[s];
        den += rho[(size_t)s * n + k] / p->tau[s];
      }
      u[k] = num[0] / den;
      u[n + k] = num[1] / den;
    }
}

/* BGK collision (Sec. II, Eq. (1), right-hand side): each species relaxes
 * towards the equilibrium evaluated at its shifted velocity
 * v_s = u' + tau_s F_s / rho_s:
 *   f*_is = f_is - (f_is - f^eq_i(rho_s, v_s)) / tau_s. */
void lbref_collide(const lbref_params* p, const double* f, const double* rho, const double* u,
                   const double* F, double* fpost) {
  const size_t n = nsites(p);
  for (int s = 0; s < NS; ++s)
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        const size_t k = IDX(p, y, x);
        const double r = rho[(size_t)s * n + k];
        const double vx = u[k] + p->tau[s] * F[((size_t)s * 2 + 0) * n + k] / r;
        const double vy = u[n + k] + p->tau[s] * F[((size_t)s * 2 + 1) * n + k] / r;
        for (int i = 0; i < NQ; ++i) {
          const double fi = FI(p, f, s, i, y, x);
          FI(p, fpost, s, i, y, x) = fi - (fi - feq(i, r, vx, vy)) / p->tau[s];
        }
      }
}

/* Free streaming (Sec. II, Eq. (1), left-hand side): f_is(r + c_i, t + 1) =
 * f*_is(r, t).  x is periodic.  y is periodic, or, with walls, a population
 * whose destination lies beyond a wall returns to its own site in the
 * opposite direction (halfway bounce-back) with the moving-wall correction
 *   f_{-i}(r, t+1) = f*_i(r, t) - 2 w_i rho_w (c_i . u_w) / c_s^2,
 * rho_w = rho_s(r, t), the density of that fluid site at time t.
 * wall_mom[0] (bottom) and wall_mom[1] (top) accumulate, summed over both
 * species and all wall links, the x-momentum handed to each wall:
 *   c_ix (f*_i + f_{-i}) = c_ix (2 f*_i - 2 w_i rho_w (c_i . u_w) / c_s^2). */
void lbref_stream(const lbref_params* p, const double* fpost, const double* rho, double* fnew,
                  double* wall_mom) {
  const size_t n = nsites(p);
  double mom[2] = {0, 0};
  for (int s = 0; s < NS; ++s)
    for (int i = 0; i < NQ; ++i)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          const double v = FI(p, fpost, s, i, y, x);
          const int yd = y + CY[i];
          if (!p->walls) {
            FI(p, fnew, s, i, ((yd % p->ny) + p->ny) % p->ny, wrap_x(p, x + CX[i])) = v;
          } else if (yd >= 0 && yd < p->ny) {
            FI(p, fnew, s, i, yd, wrap_x(p, x + CX[i])) = v;
          } else {
            const int top = yd >= p->ny;
            const double uw = top ? p->u_wall : -p->u_wall;
            const double rw = rho[(size_t)s * n + IDX(p, y, x)];
            const double corr = 2.0 * WQ[i] * rw * (CX[i] * uw) / CS2;
            FI(p, fnew, s, opposite(i), y, x) = v - corr;
            mom[top] += CX[i] * (2.0 * v - corr);
          }
        }
  if (wall_mom) {
    wall_mom[0] += mom[0];
    wall_mom[1] += mom[1];
  }
}

/* ------------------------------------------------------------------------ */
/* One full step and the drivers built on it.                                */
/* ------------------------------------------------------------------------ */

static size_t work_doubles(const lbref_params* p) {
  /* rho (2n), psi (2n), F (4n), u (2n), fpost (18n) */
  return 28 * nsites(p);
}

/* One time step t -> t+1 (Sec. II, Eq. (1) with the forces of Eq. (2)): all
 * forces come from the densities at time t; then every site collides; then
 * everything streams.  f_in and f_out must not alias.  work: scratch of
 * lbref_work_doubles() doubles, or NULL to allocate. */
int lbref_step(const lbref_params* p, const double* f_in, double* f_out, double* work,
               double* wall_mom) {
  const size_t n = nsites(p);
  double* own = NULL;
  if (!work) {
    own = (double*)malloc(work_doubles(p) * sizeof(double));
    if (!own) return -1;
    work = own;
  }
  double* rho = work;
  double* psi = rho + 2 * n;
  double* F = psi + 2 * n;
  double* u = F + 4 * n;
  double* fpost = u + 2 * n;
  lbref_density(p, f_in, rho);
  lbref_psi(p, rho, psi);
  lbref_force(p, rho, psi, F);
  lbref_common_velocity(p, f_in, rho, u);
  lbref_collide(p, f_in, rho, u, F, fpost);
  lbref_stream(p, fpost, rho, f_out, wall_mom);
  free(own);
  return 0;
}

size_t lbref_work_doubles(const lbref_params* p) { return work_doubles(p); }

/* Advance nsteps steps in place.  f must hold 18 n doubles.  wall_mom, when
 * not NULL, accumulates (see lbref_stream) over the steps whose index k
 * (0-based within this call) satisfies k >= avg_from. */
int lbref_run(const lbref_params* p, double* f, int64_t nsteps, int64_t avg_from,
              double* wall_mom) {
  const size_t n = nsites(p);
  double* tmp = (double*)malloc((18 * n + work_doubles(p)) * sizeof(double));
  if (!tmp) return -1;
  double* other = tmp;
  double* work = tmp + 18 * n;
  for (int64_t k = 0; k < nsteps; ++k) {
    lbref_step(p, f, other, work, (wall_mom && k >= avg_from) ? wall_mom : NULL);
    memcpy(f, other, 18 * n * sizeof(double));
  }
  free(tmp);
  return 0;
}

/* Populations at equilibrium with density rho_s and velocity (ux, uy) at
 * every site (ux, uy may be NULL for zero velocity, the paper's initial
 * state in Sec. VI). */
void lbref_init_equilibrium(const lbref_params* p, const double* rhoA, const double* rhoB,
                            const double* ux, const double* uy, double* f) {
  for (int s = 0; s < NS; ++s) {
    const double* r = s ? rhoB : rhoA;
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        const size_t k = IDX(p, y, x);
        const double vx = ux ? ux[k] : 0.0, vy = uy ? uy[k] : 0.0;
        for (int i = 0; i < NQ; ++i) FI(p, f, s, i, y, x) = feq(i, r[k], vx, vy);
      }
  }
}

/* Macroscopic fields of the state f at time t:
 *   rho[2][n]   species densities,
 *   u[2][n]     common velocity u',
 *   uphys[2][n] (sum_s j_s + F/2) / rho with F the total force at time t,
 *   F[2][2][n]  species forces at time t. */
int lbref_fields(const lbref_params* p, const double* f, double* rho, double* u, double* uphys,
                 double* F) {
  const size_t n = nsites(p);
  double* psi = (double*)malloc(2 * n * sizeof(double));
  if (!psi) return -1;
  lbref_density(p, f, rho);
  lbref_psi(p, rho, psi);
  lbref_force(p, rho, psi, F);
  lbref_common_velocity(p, f, rho, u);
  for (size_t k = 0; k < n; ++k) {
    const int y = (int)(k / (size_t)p->nx), x = (int)(k % (size_t)p->nx);
    double jx = 0, jy = 0;
    for (int s = 0; s < NS; ++s)
      for (int i = 0; i < NQ; ++i) {
        jx += FI(p, f, s, i, y, x) * CX[i];
        jy += FI(p, f, s, i, y, x) * CY[i];
      }
    const double rt = rho[k] + rho[n + k];
    uphys[k] = (jx + 0.5 * (F[0 * n + k] + F[2 * n + k])) / rt;
    uphys[n + k] = (jy + 0.5 * (F[1 * n + k] + F[3 * n + k])) / rt;
  }
  free(psi);
  return 0;
}

/* Global sums of the state f at time t, each a plain double accumulation in
 * site order:
 *   out[0..1] species masses sum_r rho_s,
 *   out[2..3] total momentum sum_r sum_s j_s,
 *   out[4..5] total momentum with half the force, sum_r (sum_s j_s + F/2),
 *   out[6]    kinetic stress sum_r sum_s sum_i f_is c_ix c_iy (Sec. III, Eq. (10)),
 *   out[7]    first sine mode of the line-averaged x-velocity (Sec. VIII,
 *             Eq. (66)): (2 / ny) sum_y sin(2 pi y / ny) Ubar(y), Ubar(y) =
 *             sum_x uphys_x / nx; divided by U0 it is the response R(t),
 *   out[8]    interface indicator I_AB = - sum_r grad rho_A . grad rho_B
 *             (Sec. VIII, Eq. (67)), with the lattice gradient
 *             grad phi(r) = (1 / c_s^2) sum_{i=1..8} w_i phi(r + c_i) c_i over
 *             the force stencil's neighbours (wrapped, or mirrored at walls). */
int lbref_totals(const lbref_params* p, const double* f, double* out) {
  const size_t n = nsites(p);
  double* rho = (double*)malloc(10 * n * sizeof(double));
  if (!rho) return -1;
  double* u = rho + 2 * n;
  double* uphys = u + 2 * n;
  double* F = uphys + 2 * n;
  lbref_fields(p, f, rho, u, uphys, F);
  for (int k = 0; k < 7; ++k) out[k] = 0;
  for (int s = 0; s < NS; ++s)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        double r = 0, jx = 0, jy = 0, pxy = 0;
        for (int i = 0; i < NQ; ++i) {
          const double v = FI(p, f, s, i, y, x);
          r += v;
          jx += v * CX[i];
          jy += v * CY[i];
          pxy += v * CX[i] * CY[i];
        }
        const size_t k = IDX(p, y, x);
        out[s] += r;
        out[2] += jx;
        out[3] += jy;
        out[4] += jx + 0.5 * F[((size_t)s * 2 + 0) * n + k];
        out[5] += jy + 0.5 * F[((size_t)s * 2 + 1) * n + k];
        out[6] += pxy;
      }
  out[7] = 0.0;
  for (int y = 0; y < p->ny; ++y) {
    double ubar = 0.0;
    for (int x = 0; x < p->nx; ++x) ubar += uphys[IDX(p, y, x)];
    ubar /= (double)p->nx;
    out[7] += sin(TWO_PI * (double)y / (double)p->ny) * ubar;
  }
  out[7] *= 2.0 / (double)p->ny;
  out[8] = 0.0;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      double g[NS][2] = {{0, 0}, {0, 0}};
      for (int i = 1; i <= 8; ++i) {
        const size_t nb = IDX(p, stencil_row(p, y + EY[i]), wrap_x(p, x + EX[i]));
        for (int s = 0; s < NS; ++s) {
          g[s][0] += WE[i] * rho[(size_t)s * n + nb] * EX[i] / CS2;
          g[s][1] += WE[i] * rho[(size_t)s * n + nb] * EY[i] / CS2;
        }
      }
      out[8] -= g[0][0] * g[1][0] + g[0][1] * g[1][1];
    }
  free(rho);
  return 0;
}

/* Tables, exported so the tests can check them against Table I. */
void lbref_tables(int* cx, int* cy, double* wq, int* ex, int* ey, double* pe, double* we) {
  for (int i = 0; i < NQ; ++i) {
    cx[i] = CX[i];
    cy[i] = CY[i];
    wq[i] = WQ[i];
  }
  for (int i = 0; i < NE; ++i) {
    ex[i] = EX[i];
    ey[i] = EY[i];
    pe[i] = PE[i];
    we[i] = WE[i];
  }
}

int lbref_abi_version(void) { return 1; }

/* Threads of the OpenMP loops (for timing the oracle as a baseline). */
int lbref_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void lbref_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
