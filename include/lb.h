/*
 * lb.h -- C ABI of liblbsoft, an MI355X (gfx950) implementation of the time
 * step of the two-species lattice Boltzmann model for soft-glassy fluids of
 * Benzi, Sbragaglia, Succi, Bernaschi and Chibbaro (arXiv:0906.3611).
 *
 * One step (Sec. II) advances the populations f_is of species s in {A, B}
 * on the D2Q9 lattice:
 *   1. rho_s = sum_i f_is and psi_s = rho0 (1 - exp(-rho_s / rho0))   (Eq. (5))
 *   2. Shan-Chen forces F_s (Eq. (2), weights of Table I): intra-species
 *      attraction G^a_s on the first belt, repulsion G^r_s on both belts
 *      (24 neighbours), A-B repulsion G_AB / rho0^2 on the first belt
 *   3. common velocity u' = sum_s j_s / tau_s / sum_s rho_s / tau_s and
 *      shifted velocities v_s = u' + tau_s F_s / rho_s                 (Eq. (1))
 *   4. BGK relaxation of each species to the second-order equilibrium at
 *      (rho_s, v_s), then free streaming                              (Eq. (1))
 * on a periodic lattice, or with halfway bounce-back walls moving at -u_wall
 * (below row 0) and +u_wall (above row ny-1) and x periodic.
 *
 * Conventions for every function below:
 *  - Return value: LB_OK (0) or a negative LB_E_* status.  No function
 *    aborts, exits or throws; the text of the last failure on a handle is
 *    available from lb_last_error() (lb_batch_last_error, lb_pool_last_error).
 *    A create call that fails leaves its reason for the calling thread:
 *    the same functions return it when given a null handle ("null handle"
 *    when no create call of this thread has failed since its last success).
 *  - Host arrays are FP64, row-major [ny][nx] with x fastest, whatever the
 *    storage precision, and are only borrowed for the duration of the call.
 *  - Work is enqueued on the HIP stream given at creation (NULL: the null
 *    stream).  lb_step() is asynchronous; a numerical instability detected on
 *    the device (a non-finite or non-positive density) is reported as
 *    LB_E_UNSTABLE by the next synchronizing call (lb_observables,
 *    lb_get_fields, lb_get_populations, lb_sync).
 *  - A handle is not thread-safe; distinct handles may be used from
 *    different threads.
 */
#ifndef LBSOFT_LB_H
#define LBSOFT_LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_ABI_VERSION 4

enum {
  LB_OK = 0,
  LB_E_INVAL = -1,    /* invalid argument or parameter */
  LB_E_NOMEM = -2,    /* device allocation failed / workspace too small / not admitted */
  LB_E_DEVICE = -3,   /* HIP runtime error */
  LB_E_UNSTABLE = -4, /* non-finite or non-positive density met on the device */
  LB_E_STATE = -5     /* call out of order (e.g. lb_step before lb_init) */
};

enum { LB_PERIODIC = 0, LB_COUETTE_Y = 1 };
enum { LB_FP64 = 0, LB_FP32_DEV = 1, LB_FP32_MOM = 2 };

/* Model and storage parameters.  Constraints checked by lb_create():
 * nx, ny >= 5 (the +-2 stencil must reach distinct sites); tau_s > 1/2;
 * rho0 > 0; all couplings finite.  G_a / G_r / G_AB are G^a_s, G^r_s and
 * G_AB of Sec. II, Eq. (2) (positive repels, negative attracts). */
typedef struct {
  int32_t nx, ny;
  int32_t boundary;   /* LB_PERIODIC or LB_COUETTE_Y */
  int32_t precision;  /* LB_FP64: populations stored and updated in FP64.
                         LB_FP32_DEV: stored and updated in FP32 as deviations
                         f_is - w_i rho_ref_s; reductions stay FP64.
                         LB_FP32_MOM: for tau_A = tau_B = 1 only, where the
                         collision sets every population to its equilibrium
                         (Eq. (1)): the state is the post-collision rho_s - rho_ref_s
                         and v_s of each site in FP32 (6 numbers instead of 18;
                         the populations at t are the equilibria of the
                         sources r - c_i).  Periodic boundaries only;
                         lb_set_populations is not available.  Same model,
                         different rounding from LB_FP32_DEV. */
  double tau[2];
  double rho0;
  double G_a[2];
  double G_r[2];
  double G_AB;
  double u_wall;      /* wall x-speed for LB_COUETTE_Y (top +u_wall, bottom -u_wall) */
  double body_force;  /* amplitude g of the shear forcing of Sec. VIII: each
                         species feels rho_s g sin(2 pi y / ny) along x (the
                         drive of U_x = U0 sin(k y), k = 2 pi / ny; a
                         non-interacting fluid reaches U0 = g / (nu k^2)).
                         0: no body force.  Must be finite. */
  double body_force_x; /* uniform body force per unit mass along x: each
                         species feels rho_s body_force_x (the same kind of
                         volumetric force as body_force, constant in space;
                         between LB_COUETTE_Y walls at rest it drives plane
                         Poiseuille flow).  0: none.  Must be finite. */
  double rho_ref[2];  /* LB_FP32_DEV reference densities; <= 0 selects the
                         lattice mean of the fields given to lb_init() */
  void* device_buffer;   /* optional caller-owned device workspace (e.g. the
                            storage of a torch uint8 tensor); NULL: the library
                            allocates.  Must stay alive until lb_destroy(). */
  size_t device_bytes;   /* size of device_buffer; >= lb_workspace_bytes() */
} lb_params;

/* Observables of the state at the current time t (FP64 device reductions in
 * a fixed order, so they are reproducible bit for bit). */
typedef struct {
  int64_t step;          /* t */
  double mass[2];        /* sum_r rho_s */
  double mom[2];         /* sum_r sum_s j_s, j_s = sum_i f_is c_i */
  double mom_phys[2];    /* sum_r (sum_s j_s + F/2), F = F_A + F_B at time t */
  double pxy_kin;        /* sum_r sum_s sum_i f_is c_ix c_iy (Sec. III, Eq. (10)) */
  double wall_stress[2]; /* x-momentum handed to the (bottom, top) wall per step
                            and per unit wall length, averaged over the steps
                            since the last lb_reset_averages() */
  int64_t avg_count;     /* number of steps in that average */
  int32_t flags;         /* bit 0: instability seen */
  int32_t pad_;
  double u_mode;         /* first sine mode of the line-averaged x-velocity,
                            (2 / (nx ny)) sum_r u_phys,x sin(2 pi y / ny);
                            divided by U0 it is the response R(t) of
                            Sec. VIII, Eq. (66) */
  double i_ab;           /* interface indicator -sum_r grad rho_A . grad rho_B
                            (Sec. VIII, Eq. (67)); grad phi = (1 / c_s^2)
                            sum_{i=1..8} w_i phi(r + c_i) c_i over the force
                            stencil's neighbours (mirrored at walls) */
  double phi_overlap;    /* sum_r phi(r, t_w) phi(r, t), phi = rho_A - rho_B,
                            against the reference stored at t_w by
                            lb_set_overlap_reference (0 without one) */
  double phi_ref_sq;     /* sum_r phi(r, t_w)^2 (0 without a reference).  The
                            ageing correlation of Sec. VIII B, Eq. (68), over an
                            ensemble of lattices is sum phi_overlap over the
                            realizations / sum phi_ref_sq */
  int64_t ref_step;      /* t_w, the step of the reference; -1 if none */
} lb_obs;

typedef struct lb_lattice lb_lattice;

/* Device bytes one lattice needs for these parameters (two population
 * buffers plus reduction and wall scratch).  out must not be NULL. */
int lb_workspace_bytes(const lb_params* p, size_t* out);

/* Validate p, take (or allocate) the device workspace and bind the HIP
 * stream (a hipStream_t, borrowed; NULL = null stream).  The current HIP
 * device at this call owns the lattice.  *out is NULL on failure. */
int lb_create(const lb_params* p, void* hip_stream, lb_lattice** out);

/* Set the state at t = 0 to the equilibrium populations f_is = f^eq_i(rho_s, u)
 * (the paper's initial state, Sec. VI, has u = 0).  rho_a, rho_b: host
 * [ny][nx], finite and > 0 (else LB_E_INVAL).  ux, uy: host [ny][nx] or NULL
 * for zero.  Resets t, the averages and the instability flag.  Synchronous. */
int lb_init(lb_lattice* lat, const double* rho_a, const double* rho_b, const double* ux,
            const double* uy);

/* Same as lb_init with rho_s = mean_s + amp (2U - 1), U uniform in [0, 1)
 * drawn on the device: U = (z >> 11) 2^-53 with z output number
 * (s ny + y) nx + x + 1 of SplitMix64 seeded with seed.  Requires
 * |amp| < min(mean_a, mean_b).  With LB_FP32_DEV and rho_ref <= 0 the
 * reference densities are mean_a and mean_b. */
int lb_init_noise(lb_lattice* lat, uint64_t seed, double mean_a, double mean_b, double amp);

/* Sharp two-phase emulsion (the mixed initial state of Sec. VI, in disc
 * form): a union of random discs covering at least a fraction phi of the
 * lattice holds (in_a, in_b), the rest (out_a, out_b).  Disc k has centre
 * (nx U0, ny U1) and radius rmin + (rmax - rmin) U2 with U_j = (z >> 11)
 * 2^-53, z output number 2^48 + 3k + j + 1 of SplitMix64 seeded with seed;
 * a site is inside when its minimum-image periodic distance to a centre is
 * <= that radius; discs are added until the covered count reaches
 * phi nx ny.  Built on the host, then as lb_init with u = 0.  LB_E_INVAL for
 * phi outside [0, 1], rmin <= 0 or rmax < rmin.  Synchronous. */
int lb_init_discs(lb_lattice* lat, uint64_t seed, double phi, double rmin, double rmax,
                  double in_a, double in_b, double out_a, double out_b);

/* The densities lb_init_discs uses, into host rho_a, rho_b [ny][nx]
 * (no lattice or device involved). */
int lb_disc_fields(int32_t nx, int32_t ny, uint64_t seed, double phi, double rmin, double rmax,
                   double in_a, double in_b, double out_a, double out_b, double* rho_a,
                   double* rho_b);

/* The shear-forcing amplitude (lb_params.body_force) that drives
 * U_x = U0 sin(2 pi y / ny) in a fluid of relaxation time tau (Sec. VIII):
 * the steady Stokes balance nu U'' + g sin(k y) = 0 gives g = nu k^2 U0 with
 * nu = c_s^2 (tau - 1/2) = (tau - 1/2) / 3 and k = 2 pi / ny.  Host only, no
 * device involved.  LB_E_INVAL for ny < 5, tau <= 1/2, a non-finite u0 or a
 * NULL g. */
int lb_kolmogorov_force(double u0, int32_t ny, double tau, double* g);

/* Enqueue n >= 0 time steps (Sec. II, Eq. (1)).  Asynchronous. */
int lb_step(lb_lattice* lat, int64_t n);

/* Observables of the current state (synchronizes). */
int lb_observables(lb_lattice* lat, lb_obs* out);

/* Fields of the current state into host arrays (each may be NULL):
 * rho_a, rho_b [ny][nx]; u [2][ny][nx] the common velocity u'; u_phys
 * [2][ny][nx] = (sum_s j_s + F/2) / (rho_A + rho_B).  Synchronizes. */
int lb_get_fields(lb_lattice* lat, double* rho_a, double* rho_b, double* u, double* u_phys);

/* lb_get_fields without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, outputs and errors as lb_get_fields,
 * except: the fields are staged in a static device array of 48 MiB per GPU
 * (held until the process ends), so the lattice may have at most 2^20 sites
 * (LB_E_INVAL otherwise, with the reason in lb_last_error); calls that
 * overlap in time on one GPU share that array and race, so the caller must
 * serialize them.  Synchronizes. */
int lb_get_fields_noalloc(lb_lattice* lat, double* rho_a, double* rho_b, double* u,
                          double* u_phys);

/* Pre-collision populations f_is(r, t) of the current state into host
 * f[2][9][ny][nx] (FP64, D2Q9 order rest, +x, +y, -x, -y, (1,1), (-1,1),
 * (-1,-1), (1,-1)).  Synchronizes. */
int lb_get_populations(lb_lattice* lat, double* f);

/* Replace the current state by host populations f[2][9][ny][nx] (same
 * layout) at time t = step (checkpoint restore).  For LB_FP32_DEV the
 * deviations f - w_i rho_ref_s are rounded to FP32.  Resets the averages. */
int lb_set_populations(lb_lattice* lat, const double* f, int64_t step);

/* Restart the wall-stress average at the current step. */
int lb_reset_averages(lb_lattice* lat);

/* Store the order parameter phi = rho_A - rho_B of the current state (FP64,
 * on the device, in the lattice's workspace) as the reference of the ageing
 * overlap (Sec. VIII B, Eq. (68)): from now on lb_observables also reports
 * sum_r phi_ref phi and sum_r phi_ref^2, reduced in FP64 in a fixed order.
 * lb_init / lb_set_populations drop the reference.  Synchronizes. */
int lb_set_overlap_reference(lb_lattice* lat);

/* Wait for all enqueued work; reports LB_E_UNSTABLE if flagged. */
int lb_sync(lb_lattice* lat);

/* Current time step t (host counter; no synchronization). */
int64_t lb_current_step(const lb_lattice* lat);

/* How a step is launched: each lattice is cut into nstrips column strips of
 * 64 columns (the last may be narrower) and nsegs row segments of about
 * seg_h rows; each (strip, segment) tile is one workgroup of block_threads
 * lanes (128 for FP32 deviation storage, one 64-lane wavefront per species;
 * 64 for the FP64 and moment storages, one wavefront for both species), or
 * tiles_per_group tiles share one, grid_blocks workgroups per step.  prefetch / stream_stores / use_graph
 * report the code variant in use (1 = on); tiles_per_group the tiles that
 * share a workgroup in a step launch (1, or 4 where grouping applies: see
 * lb_set_launch), block_threads and grid_blocks counting them. */
typedef struct {
  int32_t nstrips, nsegs, ntiles, grid_blocks, block_threads, pitch;
  size_t workspace_bytes;
  size_t population_bytes;   /* one population buffer of every lattice, summed */
  int32_t seg_h, prefetch, stream_stores, use_graph;
  int32_t tiles_per_group;
} lb_launch_info;
int lb_get_launch_info(const lb_lattice* lat, lb_launch_info* out);

/* Tuning knobs that leave the arithmetic unchanged: fields and observables
 * stay bit for bit the same (the FP64 reductions run over (row, strip) and
 * strip partials, not over tiles).  Any argument < 0 keeps the current choice.
 *   seg_h: row-segment height, >= 4 (0 to 3 = default policy); wall
 *     averages carry on.
 *   prefetch: rows whose loads are in flight ahead of the current one
 *     (0, 1 or 2; larger values mean 2; the moment storage ignores it).
 *     Default 1 (FP64: 2), and 0 where tiles are grouped or the moment
 *     storage exceeds the Infinity Cache.
 *   stream_stores: nontemporal population stores.  Default on where both
 *     population buffers exceed the 256 MB Infinity Cache (FP64: twice it,
 *     since its march reads back what plain stores left there).
 *   use_graph: replay lb_step as captured two-step HIP graphs (default 0:
 *     on MI355X under ROCm 7 a replayed step measured 2.3-2.5 us longer than
 *     a plain launch of the same kernel, so graphs only pay where the caller's
 *     host-side launch rate is the limit).
 *   tiles_per_group: 1 or 4 tiles of adjacent strips per workgroup of the
 *     FP32 deviation step; 4 applies only where the strip counts
 *     (ceil(nx / 64)) of all lattices of the launch are multiples of 4,
 *     elsewhere launches use 1.  Default 4 where it applies and the
 *     population buffers exceed the 256 MB Infinity Cache (1-5% faster
 *     there; slower on cache-resident lattices).  Other values: LB_E_INVAL,
 *     nothing changed. */
int lb_set_launch(lb_lattice* lat, int32_t seg_h, int32_t prefetch, int32_t stream_stores,
                  int32_t use_graph, int32_t tiles_per_group);

/* Autotuner: time candidate launch shapes on the lattice's current state and
 * keep the fastest.  The current shape first steps untimed for about 30 ms
 * (a streaming kernel runs slower for its first tens of milliseconds after
 * idle or copies).  Candidates are the default policy and forced segment
 * heights of 4 to 256 rows with the current code variant, then the six
 * prefetch (0..2) / stream_stores variants at the best height, each with
 * the current tiles_per_group (the moment
 * storage has no prefetch variants: only its two stream_stores variants are
 * timed there), then, where grouping applies, the other tiles_per_group;
 * each runs 2 untimed steps and then `steps` (>= 2, rounded up
 * to even) timed with HIP events on the lattice's stream, twice (two passes;
 * the better time counts).  The default height and the current variant are
 * kept unless another candidate is more than 1% faster, and the chosen shape
 * steps untimed for about 20 ms before the state is restored.  Results are kept
 * for the life of the process, by library ABI, GPU architecture, precision,
 * boundary type, graph use and lattice shapes;
 * steps = 0 applies a kept result without timing anything (and tunes with 16
 * steps when there is none; lb_set_tune_cache keeps results across
 * processes).  The device state (populations, wall links, flags)
 * and the step count are copied aside first and restored, so the evolution
 * and the wall-stress averages are unchanged.  Needs temporary device memory of the lattice's workspace size
 * (LB_E_NOMEM otherwise).  out (may be NULL) receives the chosen shape,
 * us_per_step (may be NULL) its time per step.  Synchronous. */
int lb_autotune(lb_lattice* lat, int32_t steps, lb_launch_info* out, double* us_per_step);

/* Keep the autotuner's results (lb_autotune, lb_batch_autotune) in the text
 * file `path` as well: results already in it are loaded now (lines that do
 * not parse are skipped), and the whole table is written back, through a
 * temporary file renamed into place, after every new result, so a later
 * process can apply them with steps = 0.  Keys carry the ABI version, GPU
 * architecture, storage, boundary type, graph use and lattice shapes; a
 * result only picks among launch shapes that give bit-identical numbers.
 * NULL or "" stops writing.  LB_E_INVAL if the file cannot be written.
 * Thread-safe; host only. */
int lb_set_tune_cache(const char* path);

void lb_destroy(lb_lattice* lat);
const char* lb_strerror(int status);
const char* lb_last_error(const lb_lattice* lat);
int lb_abi_version(void);

/* ------------------------------------------------------------------------
 * Batches: n independent lattices (any sizes and couplings, one precision
 * and boundary type) advanced together, one kernel launch per time step over
 * the tiles of all of them.  Each lattice evolves exactly as it would alone:
 * its fields are bit-for-bit those of an lb_lattice with the same parameters
 * and initial state, and so are its observables.
 * ------------------------------------------------------------------------ */
typedef struct lb_batch lb_batch;

/* Device bytes for the batch (all lattices plus shared scratch). */
int lb_batch_workspace_bytes(const lb_params* p /*[n]*/, int32_t n, size_t* out);
/* p[i].device_buffer is ignored; device_buffer/device_bytes (optional, as in
 * lb_params) cover the whole batch.  LB_E_INVAL if precisions or boundary
 * types differ. */
int lb_batch_create(const lb_params* p /*[n]*/, int32_t n, void* device_buffer,
                    size_t device_bytes, void* hip_stream, lb_batch** out);
int32_t lb_batch_size(const lb_batch* b);
/* Per-lattice initial state (as lb_init / lb_init_noise), i in [0, n). */
int lb_batch_init(lb_batch* b, int32_t i, const double* rho_a, const double* rho_b,
                  const double* ux, const double* uy);
int lb_batch_init_noise(lb_batch* b, int32_t i, uint64_t seed, double mean_a, double mean_b,
                        double amp);
int lb_batch_init_discs(lb_batch* b, int32_t i, uint64_t seed, double phi, double rmin,
                        double rmax, double in_a, double in_b, double out_a, double out_b);
/* Enqueue n steps of every lattice (LB_E_STATE until all are initialized). */
int lb_batch_step(lb_batch* b, int64_t n);
/* Observables of every lattice into out[0 .. n) (synchronizes). */
int lb_batch_observables(lb_batch* b, lb_obs* out);
int lb_batch_get_fields(lb_batch* b, int32_t i, double* rho_a, double* rho_b, double* u,
                        double* u_phys);
int lb_batch_get_populations(lb_batch* b, int32_t i, double* f);
int lb_batch_sync(lb_batch* b);
/* Restart the wall-stress averages of every lattice (as lb_reset_averages). */
int lb_batch_reset_averages(lb_batch* b);
/* As lb_set_overlap_reference, for every lattice of the batch. */
int lb_batch_set_overlap_reference(lb_batch* b);
int lb_batch_get_launch_info(const lb_batch* b, lb_launch_info* out);
/* As lb_set_launch; seg_h applies to every lattice of the batch (equal
 * tile heights balance the work of uneven lattices). */
int lb_batch_set_launch(lb_batch* b, int32_t seg_h, int32_t prefetch, int32_t stream_stores,
                        int32_t use_graph, int32_t tiles_per_group);
/* As lb_autotune, over the whole batch (one common segment height). */
int lb_batch_autotune(lb_batch* b, int32_t steps, lb_launch_info* out, double* us_per_step);
void lb_batch_destroy(lb_batch* b);
const char* lb_batch_last_error(const lb_batch* b);

/* ------------------------------------------------------------------------
 * Serving pool: simulation jobs (one lattice each) are admitted while their
 * device footprint fits an HBM budget (first fit: a job that does not fit
 * yet does not block later, smaller ones), kept resident, and advanced in
 * launches of one class of (precision, boundary type) each, over the
 * advancing jobs of that class (see lb_pool_set_schedule for which jobs
 * advance).  A job stops exactly at its own step count; it is then retired:
 * its observables (and, unless switched off, its density fields) are copied
 * to the host and its device memory is released.  Whatever the schedule, a
 * job's results are bit for bit those of the same lattice run alone.  Times
 * are seconds since lb_pool_create on a monotonic host clock.  Not
 * thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct lb_pool lb_pool;
enum { LB_JOB_QUEUED = 0, LB_JOB_RUNNING = 1, LB_JOB_DONE = 2, LB_JOB_FAILED = 3 };

typedef struct {
  int64_t submitted, queued, running, done, failed;
  size_t resident_bytes, budget_bytes;
  int64_t site_updates;  /* completed site updates, summed over jobs */
  int64_t ticks;         /* launch rounds (steps between membership changes) */
  int64_t steps;         /* pool steps run */
  double clock;          /* seconds since creation */
} lb_pool_stats;

/* hbm_budget_bytes: ceiling on the summed device footprint of resident jobs. */
int lb_pool_create(size_t hbm_budget_bytes, void* hip_stream, lb_pool** out);
void lb_pool_destroy(lb_pool* pool);
const char* lb_pool_last_error(const lb_pool* pool);
/* keep_fields: copy final densities at retirement (default 1); use_graph:
 * replay step pairs as HIP graphs (default 0, see lb_set_launch).  < 0 keeps
 * the setting. */
int lb_pool_set_options(lb_pool* pool, int32_t keep_fields, int32_t use_graph);
/* Which resident jobs advance, and in which order queued jobs are admitted.
 * policy 1 (default), least remaining work: queued jobs are admitted in
 * increasing order of sites x steps (ties in arrival order), and each pool
 * step advances only the resident jobs of least remaining sites x steps,
 * taken in that order until their sites reach fill_sites (at least one job;
 * default 2^23); the others wait, buffers untouched, and their step count,
 * time and wall averages do not move.  Finished jobs leave sooner, so mean
 * and median turnaround fall; a large job can wait while smaller ones keep
 * arriving.  A smaller fill_sites trades throughput for turnaround: fewer
 * sites per launch fill the device less (on a 60-job trace with sides 64 to
 * 2048, fill 2^21 gave 0.86x the lock-step throughput at 0.27x its median
 * turnaround, 2^23 0.97x at 0.53x, 2^24 0.99x at 0.83x).  max_hold > 0
 * bounds the wait: a resident job held back for max_hold pool steps in a
 * row advances in the next chunk, ahead of the order of remaining work
 * (longest held first; every job at the bound advances, past fill_sites if
 * need be), and a chunk ends early when a waiting job reaches the bound, so
 * no resident job waits more than max_hold pool steps in a row; 0
 * (default): no bound.  policy 0, lock-step: arrival-order admission, every resident job
 * advances every step.  policy < 0, fill_sites <= 0 or max_hold < 0 keeps
 * that setting; policy > 1 is LB_E_INVAL. */
int lb_pool_set_schedule(lb_pool* pool, int32_t policy, int64_t fill_sites, int64_t max_hold);
/* Device footprint of one job with these parameters (0 if invalid). */
size_t lb_pool_job_bytes(const lb_params* p);
/* Queue a job of `steps` steps (p->device_buffer ignored), started from the
 * lb_init_noise state or from host densities (copied at submission).
 * LB_E_NOMEM if its footprint alone exceeds the budget; LB_E_INVAL for
 * LB_FP32_MOM (the pool runs population storage). */
int lb_pool_submit_noise(lb_pool* pool, const lb_params* p, uint64_t seed, double mean_a,
                         double mean_b, double amp, int64_t steps, int64_t* job_id);
int lb_pool_submit(lb_pool* pool, const lb_params* p, const double* rho_a, const double* rho_b,
                   int64_t steps, int64_t* job_id);
/* Admit what fits, run n pool steps (jobs finish at their own counts),
 * retire finished jobs, admit again as memory frees.  Synchronizes. */
int lb_pool_advance(lb_pool* pool, int64_t n);
int lb_pool_job_state(const lb_pool* pool, int64_t job_id, int32_t* state);
/* Steps a job has run so far (0 while queued, its step count once done);
 * no synchronization: the count of enqueued steps. */
int lb_pool_job_progress(const lb_pool* pool, int64_t job_id, int64_t* steps_done);
/* Result of a finished job: observables, densities [ny][nx] (each may be
 * NULL) and times[3] = {submitted, admitted, done} (may be NULL; filled for
 * any job).  LB_E_STATE if not finished; the failure status if it failed. */
int lb_pool_job_result(lb_pool* pool, int64_t job_id, lb_obs* obs, double* rho_a, double* rho_b,
                       double* times);
/* Forget a finished job (frees its host copies). */
int lb_pool_release(lb_pool* pool, int64_t job_id);
int lb_pool_get_stats(const lb_pool* pool, lb_pool_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* LBSOFT_LB_H */
