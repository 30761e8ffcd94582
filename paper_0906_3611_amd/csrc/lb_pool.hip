// Serving pool (C ABI lb_pool_*): simulation jobs are admitted while their
// device footprint fits an HBM budget, kept resident, advanced in launches
// of one precision/boundary class each (over every resident job of the
// class, or over those of least remaining work), and retired when they
// reach their step count: observables and density fields are copied to the
// host and the device memory is released.
#include "lb.h"
#include "lb_engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

using lbe::DeviceGuard;
using lbe::Engine;

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  int64_t id = 0;
  lb_params p{};
  int64_t steps = 0;
  // initial state: host fields, or a noise spec
  bool noise = false;
  uint64_t seed = 0;
  double mean_a = 0, mean_b = 0, amp = 0;
  std::vector<double> rho_a, rho_b;
  int32_t state = LB_JOB_QUEUED;
  int engine = -1;  // engine class while running
  size_t bytes = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  lb_obs result{};
  std::vector<double> out_a, out_b;  // final densities (done)
  int status = LB_OK;               // failure status
  int64_t held = 0;                 // pool steps resident without advancing
};

int engine_class(const lb_params* p) {
  return (p->precision == LB_FP64 ? 1 : 0) + (p->boundary == LB_COUETTE_Y ? 2 : 0);
}

}  // namespace

struct lb_pool {
  size_t budget = 0, resident = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  Engine eng[4];
  bool eng_ready[4] = {false, false, false, false};
  std::map<int64_t, Job> jobs;
  std::deque<int64_t> queue;
  int64_t next_id = 1;
  int64_t site_updates = 0, ticks = 0, steps_run = 0;
  int keep_fields = 1;
  int use_graph = 0;
  // scheduling: 0 = every resident job advances every step; 1 = the jobs
  // of least remaining work (sites x steps), up to fill_sites sites, advance
  // and the others wait (admission in the same order)
  int schedule = 1;
  // 2^23 sites: on a 60-job trace (sides 64-2048) 0.97x the lock-step
  // throughput at 0.53x its median turnaround; 2^21 gives 0.86x at 0.27x
  int64_t fill_sites = 1 << 23;
  // a resident job held back this many pool steps advances next, ahead of
  // the order of remaining work (0: no bound)
  int64_t max_hold = 0;
  Clock::time_point t0 = Clock::now();
  std::string err;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
};

namespace {

int ensure_engine(lb_pool* P, int cls) {
  if (P->eng_ready[cls]) return LB_OK;
  Engine& E = P->eng[cls];
  const int rc = lbe::engine_create_dynamic(E, (cls & 1) != 0, (cls & 2) != 0, P->stream);
  if (rc != LB_OK) return P->fail(rc, E.err);
  lbe::engine_set_variant(E, -1, -1, P->use_graph, -1);
  P->eng_ready[cls] = true;
  return LB_OK;
}

double job_work(const Job& j) { return (double)j.p.nx * (double)j.p.ny * (double)j.steps; }

// Admit queued jobs while they fit the budget (first fit: a job that does
// not fit yet does not block later, smaller ones), in arrival order or, when
// scheduling by remaining work, least work first (ties in arrival order).
int admit(lb_pool* P) {
  if (P->schedule == 1)
    std::stable_sort(P->queue.begin(), P->queue.end(), [&](int64_t x, int64_t y) {
      return job_work(P->jobs[x]) < job_work(P->jobs[y]);
    });
  for (auto it = P->queue.begin(); it != P->queue.end();) {
    Job& j = P->jobs[*it];
    if (P->resident + j.bytes > P->budget) {
      ++it;
      continue;
    }
    const int cls = engine_class(&j.p);
    int rc = ensure_engine(P, cls);
    if (rc != LB_OK) return rc;
    Engine& E = P->eng[cls];
    int idx = -1;
    rc = lbe::engine_add(E, &j.p, j.id, &idx);
    if (rc == LB_E_NOMEM) {  // device allocation failed: leave it queued
      ++it;
      continue;
    }
    if (rc == LB_OK)
      rc = j.noise ? lbe::engine_init_noise(E, idx, j.seed, j.mean_a, j.mean_b, j.amp)
                   : lbe::engine_init(E, idx, j.rho_a.data(), j.rho_b.data(), nullptr, nullptr);
    if (rc != LB_OK) {
      j.state = LB_JOB_FAILED;
      j.status = rc;
      j.t_done = P->now();
      if (idx >= 0) lbe::engine_remove(E, idx);
      it = P->queue.erase(it);
      continue;
    }
    j.rho_a.clear();
    j.rho_a.shrink_to_fit();
    j.rho_b.clear();
    j.rho_b.shrink_to_fit();
    j.state = LB_JOB_RUNNING;
    j.engine = cls;
    j.t_admit = P->now();
    P->resident += j.bytes;
    it = P->queue.erase(it);
  }
  return LB_OK;
}

// Observables and (optionally) densities of member i, then release it.
int retire(lb_pool* P, int cls, int i) {
  Engine& E = P->eng[cls];
  const int64_t id = E.m[i].tag;
  Job& j = P->jobs[id];
  int rc = lbe::engine_member_observables(E, i, &j.result);
  if (rc == LB_OK && P->keep_fields) {
    const size_t n = (size_t)j.p.nx * j.p.ny;
    j.out_a.resize(n);
    j.out_b.resize(n);
    rc = lbe::engine_fields(E, i, j.out_a.data(), j.out_b.data(), nullptr, nullptr);
  }
  j.state = rc == LB_OK ? LB_JOB_DONE : LB_JOB_FAILED;
  j.status = rc;
  const int rr = lbe::engine_remove(E, i);
  P->resident -= j.bytes;
  j.t_done = P->now();
  return rr != LB_OK ? rr : LB_OK;
}

int64_t remaining(const lb_pool* P, int cls, int i) {
  const Engine& E = P->eng[cls];
  const Job& j = P->jobs.at(E.m[i].tag);
  return j.steps - lbe::member_time(E, i);
}

}  // namespace

extern "C" {

int lb_pool_create(size_t hbm_budget_bytes, void* hip_stream, lb_pool** out) {
  if (!out || hbm_budget_bytes == 0) return LB_E_INVAL;
  *out = nullptr;
  lb_pool* P = new (std::nothrow) lb_pool();
  if (!P) return LB_E_NOMEM;
  P->budget = hbm_budget_bytes;
  P->stream = (hipStream_t)hip_stream;
  const hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) {
    lbe::create_error() = std::string("hipGetDevice: ") + hipGetErrorString(e);
    delete P;
    return LB_E_DEVICE;
  }
  lbe::create_error().clear();
  *out = P;
  return LB_OK;
}

void lb_pool_destroy(lb_pool* P) {
  if (!P) return;
  for (int c = 0; c < 4; ++c)
    if (P->eng_ready[c]) lbe::engine_destroy(P->eng[c]);
  delete P;
}

const char* lb_pool_last_error(const lb_pool* P) { return lbe::handle_error(P ? &P->err : nullptr); }

int lb_pool_set_options(lb_pool* P, int32_t keep_fields, int32_t use_graph) {
  if (!P) return LB_E_INVAL;
  if (keep_fields >= 0) P->keep_fields = keep_fields ? 1 : 0;
  if (use_graph >= 0) {
    P->use_graph = use_graph ? 1 : 0;
    for (int c = 0; c < 4; ++c)
      if (P->eng_ready[c]) lbe::engine_set_variant(P->eng[c], -1, -1, P->use_graph, -1);
  }
  return LB_OK;
}

int lb_pool_set_schedule(lb_pool* P, int32_t policy, int64_t fill_sites, int64_t max_hold) {
  if (!P) return LB_E_INVAL;
  if (policy > 1) return P->fail(LB_E_INVAL, "schedule policy must be 0 or 1");
  if (policy >= 0) P->schedule = policy;
  if (fill_sites > 0) P->fill_sites = fill_sites;
  if (max_hold >= 0) P->max_hold = max_hold;
  return LB_OK;
}

size_t lb_pool_job_bytes(const lb_params* p) {
  return lbe::validate(p, nullptr) == LB_OK ? lbe::member_region_bytes(p) : 0;
}

static int submit_common(lb_pool* P, const lb_params* p, int64_t steps, Job& j, int64_t* job_id) {
  std::string why;
  if (lbe::validate(p, &why) != LB_OK) return P->fail(LB_E_INVAL, why);
  if (p->precision == LB_FP32_MOM) return P->fail(LB_E_INVAL, "the pool runs population storage only");
  if (steps < 0) return P->fail(LB_E_INVAL, "steps must be >= 0");
  j.p = *p;
  j.p.device_buffer = nullptr;
  j.p.device_bytes = 0;
  j.steps = steps;
  j.bytes = lbe::member_region_bytes(p);
  if (j.bytes > P->budget) return P->fail(LB_E_NOMEM, "job footprint exceeds the pool budget");
  j.id = P->next_id++;
  j.t_submit = P->now();
  P->jobs[j.id] = std::move(j);
  P->queue.push_back(P->jobs.rbegin()->first);
  if (job_id) *job_id = P->jobs.rbegin()->first;
  return LB_OK;
}

int lb_pool_submit_noise(lb_pool* P, const lb_params* p, uint64_t seed, double mean_a,
                         double mean_b, double amp, int64_t steps, int64_t* job_id) {
  if (!P || !p) return LB_E_INVAL;
  if (!(std::fabs(amp) < std::min(mean_a, mean_b))) return P->fail(LB_E_INVAL, "need |amp| < means");
  Job j;
  j.noise = true;
  j.seed = seed;
  j.mean_a = mean_a;
  j.mean_b = mean_b;
  j.amp = amp;
  return submit_common(P, p, steps, j, job_id);
}

int lb_pool_submit(lb_pool* P, const lb_params* p, const double* rho_a, const double* rho_b,
                   int64_t steps, int64_t* job_id) {
  if (!P || !p || !rho_a || !rho_b) return LB_E_INVAL;
  std::string why;  // the sizes must be valid before the arrays are read
  if (lbe::validate(p, &why) != LB_OK) return P->fail(LB_E_INVAL, why);
  const size_t n = (size_t)p->nx * p->ny;
  for (size_t k = 0; k < n; ++k)
    if (!(rho_a[k] > 0) || !(rho_b[k] > 0) || !std::isfinite(rho_a[k]) || !std::isfinite(rho_b[k]))
      return P->fail(LB_E_INVAL, "densities must be finite and > 0");
  Job j;
  j.rho_a.assign(rho_a, rho_a + n);
  j.rho_b.assign(rho_b, rho_b + n);
  return submit_common(P, p, steps, j, job_id);
}

int lb_pool_advance(lb_pool* P, int64_t n) {
  if (!P || n < 0) return LB_E_INVAL;
  DeviceGuard dg(P->device);
  int rc = admit(P);
  if (rc != LB_OK) return rc;
  int64_t left = n;
  while (true) {
    // retire finished jobs (also those admitted with 0 steps)
    for (int c = 0; c < 4; ++c) {
      if (!P->eng_ready[c]) continue;
      for (int i = (int)P->eng[c].m.size() - 1; i >= 0; --i)
        if (remaining(P, c, i) <= 0) {
          rc = retire(P, c, i);
          if (rc != LB_OK) return P->fail(rc, P->eng[c].err);
        }
    }
    rc = admit(P);
    if (rc != LB_OK) return rc;
    if (left <= 0) break;
    // resident jobs: (class, member, remaining steps, sites)
    struct Res {
      int c, i;
      int64_t rem;
      size_t sites;
    };
    std::vector<Res> rs;
    for (int c = 0; c < 4; ++c) {
      if (!P->eng_ready[c]) continue;
      for (int i = 0; i < (int)P->eng[c].m.size(); ++i)
        rs.push_back({c, i, remaining(P, c, i),
                      (size_t)P->eng[c].m[i].p.nx * P->eng[c].m[i].p.ny});
    }
    if (rs.empty()) break;
    auto held = [&](const Res& r) -> int64_t& { return P->jobs[P->eng[r.c].m[r.i].tag].held; };
    if (P->schedule == 1) {
      // jobs held back to the bound first (longest held first), then least
      // remaining work (stable: ties by class, member)
      const int64_t H = P->max_hold;
      std::stable_sort(rs.begin(), rs.end(), [&](const Res& x, const Res& y) {
        const bool ox = H > 0 && held(x) >= H, oy = H > 0 && held(y) >= H;
        if (ox != oy) return ox;
        if (ox) return held(x) > held(y);
        return (double)x.rem * (double)x.sites < (double)y.rem * (double)y.sites;
      });
    }
    // the advancing set: everyone (schedule 0), or in that order until
    // fill_sites sites; it runs until its first job finishes
    std::vector<int> sel[4];
    std::vector<char> adv(rs.size(), 0);
    int64_t m = left;
    size_t sites = 0;
    // every job held back to the bound advances, even past fill_sites (they
    // come first in the order), so none waits longer than max_hold
    for (size_t k = 0; k < rs.size(); ++k) {
      const bool due = P->schedule == 1 && P->max_hold > 0 && held(rs[k]) >= P->max_hold;
      if (P->schedule == 1 && sites >= (size_t)P->fill_sites && !due) break;
      sel[rs[k].c].push_back(rs[k].i);
      adv[k] = 1;
      sites += rs[k].sites;
      m = std::min(m, rs[k].rem);
    }
    // with a hold bound, a chunk also ends when a waiting job reaches it
    if (P->schedule == 1 && P->max_hold > 0)
      for (size_t k = 0; k < rs.size(); ++k)
        if (!adv[k]) m = std::min(m, std::max<int64_t>(1, P->max_hold - held(rs[k])));
    for (size_t k = 0; k < rs.size(); ++k) held(rs[k]) = adv[k] ? 0 : held(rs[k]) + m;
    for (int c = 0; c < 4; ++c) {
      if (sel[c].empty()) continue;
      rc = lbe::engine_step_subset(P->eng[c], sel[c], m);
      if (rc != LB_OK) return P->fail(rc, P->eng[c].err);
    }
    P->site_updates += (int64_t)sites * m;
    P->steps_run += m;
    left -= m;
    ++P->ticks;
  }
  if (hipStreamSynchronize(P->stream) != hipSuccess) return P->fail(LB_E_DEVICE, "synchronize failed");
  return LB_OK;
}

int lb_pool_job_progress(const lb_pool* P, int64_t job_id, int64_t* steps_done) {
  if (!P || !steps_done) return LB_E_INVAL;
  auto it = P->jobs.find(job_id);
  if (it == P->jobs.end()) return LB_E_INVAL;
  const Job& j = it->second;
  if (j.state == LB_JOB_RUNNING) {
    const Engine& E = P->eng[j.engine];
    const int i = lbe::member_index(E, j.id);
    *steps_done = i >= 0 ? lbe::member_time(E, i) : 0;
  } else {
    *steps_done = j.state == LB_JOB_DONE ? j.steps : 0;
  }
  return LB_OK;
}

int lb_pool_job_state(const lb_pool* P, int64_t job_id, int32_t* state) {
  if (!P || !state) return LB_E_INVAL;
  auto it = P->jobs.find(job_id);
  if (it == P->jobs.end()) return LB_E_INVAL;
  *state = it->second.state;
  return LB_OK;
}

int lb_pool_job_result(lb_pool* P, int64_t job_id, lb_obs* obs, double* rho_a, double* rho_b,
                       double* times) {
  if (!P) return LB_E_INVAL;
  auto it = P->jobs.find(job_id);
  if (it == P->jobs.end()) return P->fail(LB_E_INVAL, "unknown job");
  Job& j = it->second;
  if (times) {
    times[0] = j.t_submit;
    times[1] = j.t_admit;
    times[2] = j.t_done;
  }
  if (j.state == LB_JOB_FAILED) return j.status != LB_OK ? j.status : LB_E_STATE;
  if (j.state != LB_JOB_DONE) return P->fail(LB_E_STATE, "job not finished");
  if (obs) *obs = j.result;
  const size_t n = (size_t)j.p.nx * j.p.ny;
  if (rho_a || rho_b) {
    if (j.out_a.size() != n) return P->fail(LB_E_STATE, "fields were not kept");
    if (rho_a) std::copy(j.out_a.begin(), j.out_a.end(), rho_a);
    if (rho_b) std::copy(j.out_b.begin(), j.out_b.end(), rho_b);
  }
  return LB_OK;
}

int lb_pool_release(lb_pool* P, int64_t job_id) {
  if (!P) return LB_E_INVAL;
  auto it = P->jobs.find(job_id);
  if (it == P->jobs.end()) return LB_E_INVAL;
  if (it->second.state == LB_JOB_QUEUED || it->second.state == LB_JOB_RUNNING)
    return P->fail(LB_E_STATE, "job still active");
  P->jobs.erase(it);
  return LB_OK;
}

int lb_pool_get_stats(const lb_pool* P, lb_pool_stats* out) {
  if (!P || !out) return LB_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  for (const auto& kv : P->jobs) {
    switch (kv.second.state) {
      case LB_JOB_QUEUED: ++out->queued; break;
      case LB_JOB_RUNNING: ++out->running; break;
      case LB_JOB_DONE: ++out->done; break;
      default: ++out->failed; break;
    }
  }
  out->submitted = P->next_id - 1;
  out->resident_bytes = P->resident;
  out->budget_bytes = P->budget;
  out->site_updates = P->site_updates;
  out->ticks = P->ticks;
  out->steps = P->steps_run;
  out->clock = P->now();
  return LB_OK;
}

}  // extern "C"
