// Serving layer: continuous batching of steady solves on one GPU.
//
// A dispatcher admits queued requests while a slot is free and the estimated
// device footprint fits the budget; each admitted request gets its own
// context and stream (default priority) and is driven by its own host thread
// through implicit steps (Algorithm 1) until the residual has dropped by the
// requested factor.  When it finishes its device memory is freed and the
// dispatcher admits the next request.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "hgks.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Job {
  int64_t ticket = 0;
  // copied request
  std::vector<double> xyz;
  std::vector<int32_t> tets, bfaces, btags, bc_tag, bc_kind;
  double prim[5];
  hgks_options opts;
  double drop = 1e-8;
  int32_t max_steps = 1000;
  size_t footprint = 0;
  // lifecycle
  Clock::time_point t_submit, t_admit, t_done;
  bool admitted = false, done = false;
  hgks_result result{};
  std::vector<double> Q;  // final state
  std::thread worker;
  hgks_ctx* ctx = nullptr;  // while the request runs (set and cleared under the server lock)
};

}  // namespace

struct hgks_server {
  std::mutex mu;
  std::condition_variable cv;  // signals state changes (admission, completion)
  size_t budget = 0, in_use = 0;
  int max_slots = 1, active = 0;
  int64_t next_ticket = 1;
  std::deque<int64_t> queue;
  std::map<int64_t, std::unique_ptr<Job>> jobs;
  std::vector<std::thread> finished_workers;
  int64_t cell_evals = 0;
  int64_t steps_finished = 0;  // implicit steps of finished requests
  int32_t n_done = 0;
  bool stopping = false;
  int device = 0;
  std::thread dispatcher;
};

namespace {

void run_job(hgks_server* S, Job* J) {
  (void)hipSetDevice(S->device);
  hgks_result r{};
  r.n_cells = (int64_t)(J->tets.size() / 4);
  r.footprint_bytes = J->footprint;
  hgks_options o = J->opts;
  o.stream = nullptr;  // the context creates its own stream
  hgks_ctx* ctx = nullptr;
  hgks_status st = hgks_create(&o, &ctx);
  if (st == HGKS_OK) {
    std::lock_guard<std::mutex> lk(S->mu);
    J->ctx = ctx;
  }
  std::vector<double> Q;
  if (st == HGKS_OK)
    st = hgks_load_mesh(ctx, (int64_t)(J->xyz.size() / 3), J->xyz.data(), r.n_cells, J->tets.data(),
                        (int64_t)(J->btags.size()), J->bfaces.data(), J->btags.data());
  if (st == HGKS_OK) st = hgks_set_freestream(ctx, J->prim);
  for (size_t k = 0; st == HGKS_OK && k < J->bc_tag.size(); ++k)
    st = hgks_set_bc(ctx, J->bc_tag[k], J->bc_kind[k], nullptr);
  if (st == HGKS_OK) {
    // initial state: the free stream (gradients zero)
    double g = o.gamma;
    double rho = J->prim[0], u = J->prim[1], v = J->prim[2], w = J->prim[3], p = J->prim[4];
    double q[5] = {rho, rho * u, rho * v, rho * w, p / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w)};
    Q.assign((size_t)5 * r.n_cells, 0.0);
    for (int k = 0; k < 5; ++k)
      for (int64_t i = 0; i < r.n_cells; ++i) Q[(size_t)k * r.n_cells + i] = q[k];
    st = hgks_set_state(ctx, Q.data(), nullptr);
  }
  if (st == HGKS_OK) {
    hgks_solve_info si{};
    st = hgks_solve_steady(ctx, J->drop, J->max_steps, &si);
    r.steps = si.steps;
    r.res0 = si.res0;
    r.res_final = si.res_final;
    r.n_resid_evals = si.n_resid_evals;
    hgks_get_state(ctx, Q.data(), nullptr);
  }
  if (ctx) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      J->ctx = nullptr;
      S->steps_finished += hgks_steps_done(ctx);
    }
    hgks_destroy(ctx);
  }
  r.status = st;
  std::lock_guard<std::mutex> lk(S->mu);
  J->t_done = Clock::now();
  r.t_queue_ms = ms_between(J->t_submit, J->t_admit);
  r.t_solve_ms = ms_between(J->t_admit, J->t_done);
  r.t_total_ms = ms_between(J->t_submit, J->t_done);
  J->result = r;
  J->Q.swap(Q);
  J->done = true;
  S->in_use -= J->footprint;
  S->active -= 1;
  S->n_done += 1;
  S->cell_evals += r.n_cells * r.n_resid_evals;
  S->finished_workers.push_back(std::move(J->worker));
  S->cv.notify_all();
}

// admission: of the queued requests that fit, the one with the smallest
// footprint (the estimate of its size, so of its work per step) goes first,
// ties in arrival order; once the oldest request has waited more than
// STARVE_MS it goes next and no other request passes it
constexpr double STARVE_MS = 60000.0;
void dispatch_loop(hgks_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    for (auto& t : S->finished_workers)
      if (t.joinable()) t.join();
    S->finished_workers.clear();
    if (S->stopping && S->active == 0) break;
    bool admitted = false;
    if (!S->stopping && S->active < S->max_slots && !S->queue.empty()) {
      Job* head = S->jobs[S->queue.front()].get();
      const bool head_starving = ms_between(head->t_submit, Clock::now()) > STARVE_MS;
      auto best = S->queue.end();
      for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
        Job* J = S->jobs[*it].get();
        const bool fits = S->in_use + J->footprint <= S->budget || S->active == 0;
        if (fits && (best == S->queue.end() || J->footprint < S->jobs[*best]->footprint)) best = it;
        if (head_starving) break;  // only the head may go
      }
      if (best != S->queue.end()) {
        Job* J = S->jobs[*best].get();
        S->queue.erase(best);
        J->admitted = true;
        J->t_admit = Clock::now();
        S->in_use += J->footprint;
        S->active += 1;
        J->worker = std::thread(run_job, S, J);
        admitted = true;
      }
    }
    if (!admitted) S->cv.wait_for(lk, std::chrono::milliseconds(50));
  }
}

}  // namespace

extern "C" {

size_t hgks_estimate_bytes(int64_t n_tets, int64_t n_bfaces, const hgks_options* o) {
  // mirrors the allocations of hgks_load_mesh and the first use of the inner
  // precision (faces: F = (4N + Nb)/2 exactly for a conforming tet mesh)
  double N = (double)n_tets, Nb = (double)n_bfaces, F = 0.5 * (4.0 * N + Nb), NX = N + Nb;
  int m = o ? o->krylov_dim : 10;
  bool hw = o && o->scheme == HGKS_HWENO;
  bool ko = o && o->scheme == HGKS_KFVS1;  // no stencils, operators or side values
  bool f32 = o && o->precision == HGKS_FP32_INNER;
  // faces (L, R, kind), cell faces, neighbours, ghosts; WENO stencils
  double ints = F * 3 + N * 4 + N * 4 + Nb * 2 + (ko || hw ? 0 : (16 + 24) * N);
  double bytes = 4.0 * ints + (hw || ko ? 0 : N);
  double fp = N * (1 + 1 + 1 + 6) + F * (3 + 1 + 9 + 9) + (ko ? 0 : (hw ? N * (171 + 24) : N * (144 + 72)));
  double work = 5 * NX + (ko ? 0 : 105 * N + 120 * F) + 5 * F + 5 * F + N + (hw ? 15 * NX : 0);
  bytes += 8.0 * (fp + work);
  // state, base residuals, gradients, diagonal, Krylov basis, work vectors
  bytes += 8.0 * (5 * N + 5 * NX + (hw ? 15 * NX : 0) + N + 10 * N + 15 * N + F + N + (m + 1) * 5 * N + 6 * 5 * N +
                  2 * 1024 + 128);
  if (f32) bytes += 4.0 * (fp + work + 5 * NX);
  if (o && o->solver == HGKS_SOLVER_LUSGS) bytes += 4.0 * 2 * N;  // colours and colour order
  return (size_t)(bytes * 1.05) + ((size_t)16 << 20);
}

hgks_status hgks_server_create(size_t hbm_budget_bytes, int32_t max_slots, hgks_server** out) {
  if (!out || max_slots < 1 || hbm_budget_bytes == 0) return HGKS_EINVAL;
  hgks_server* S = new (std::nothrow) hgks_server;
  if (!S) return HGKS_ENOMEM;
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  if (hipGetDevice(&S->device) != hipSuccess) S->device = 0;
  S->dispatcher = std::thread(dispatch_loop, S);
  *out = S;
  return HGKS_OK;
}

hgks_status hgks_server_submit(hgks_server* S, const hgks_request* q, int64_t* ticket) {
  if (!S || !q || !ticket || q->n_tets <= 0 || q->n_nodes <= 0 || !q->xyz || !q->tet2node) return HGKS_EINVAL;
  if (q->n_bc < 0 || (q->n_bc > 0 && (!q->bc_tag || !q->bc_kind))) return HGKS_EINVAL;
  auto J = std::make_unique<Job>();
  J->xyz.assign(q->xyz, q->xyz + 3 * q->n_nodes);
  J->tets.assign(q->tet2node, q->tet2node + 4 * q->n_tets);
  if (q->n_bfaces > 0) {
    J->bfaces.assign(q->bface2node, q->bface2node + 3 * q->n_bfaces);
    J->btags.assign(q->bface_tag, q->bface_tag + q->n_bfaces);
  }
  for (int k = 0; k < q->n_bc; ++k) {
    J->bc_tag.push_back(q->bc_tag[k]);
    J->bc_kind.push_back(q->bc_kind[k]);
  }
  std::memcpy(J->prim, q->prim_inf, sizeof(J->prim));
  J->opts = q->opts;
  J->drop = q->drop;
  J->max_steps = q->max_steps;
  J->footprint = hgks_estimate_bytes(q->n_tets, q->n_bfaces, &q->opts);
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopping) return HGKS_EINVAL;
  J->ticket = S->next_ticket++;
  J->t_submit = Clock::now();
  *ticket = J->ticket;
  S->queue.push_back(J->ticket);
  S->jobs[J->ticket] = std::move(J);
  S->cv.notify_all();
  return HGKS_OK;
}

hgks_status hgks_server_poll(hgks_server* S, int64_t ticket, int32_t* done, hgks_result* out) {
  if (!S || !done) return HGKS_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return HGKS_EINVAL;
  *done = it->second->done ? 1 : 0;
  if (it->second->done && out) *out = it->second->result;
  return HGKS_OK;
}

hgks_status hgks_server_wait(hgks_server* S, int64_t ticket, hgks_result* out) {
  if (!S) return HGKS_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) return HGKS_EINVAL;
  Job* J = it->second.get();
  S->cv.wait(lk, [&] { return J->done; });
  if (out) *out = J->result;
  return HGKS_OK;
}

hgks_status hgks_server_get_state(hgks_server* S, int64_t ticket, double* Q) {
  if (!S || !Q) return HGKS_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end() || !it->second->done || it->second->Q.empty()) return HGKS_EINVAL;
  std::memcpy(Q, it->second->Q.data(), it->second->Q.size() * sizeof(double));
  return HGKS_OK;
}

hgks_status hgks_server_release(hgks_server* S, int64_t ticket) {
  if (!S) return HGKS_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end() || !it->second->done) return HGKS_EINVAL;
  S->jobs.erase(it);
  return HGKS_OK;
}

hgks_status hgks_server_stats(hgks_server* S, hgks_server_info* out) {
  if (!S || !out) return HGKS_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  out->queued = (int32_t)S->queue.size();
  out->active = S->active;
  out->done = S->n_done;
  out->bytes_in_use = S->in_use;
  out->budget = S->budget;
  out->cell_resid_evals = S->cell_evals;
  out->steps_done = S->steps_finished;
  for (const auto& kv : S->jobs)
    if (kv.second->ctx) out->steps_done += hgks_steps_done(kv.second->ctx);
  return HGKS_OK;
}

void hgks_server_destroy(hgks_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
    S->queue.clear();
    S->cv.notify_all();
  }
  if (S->dispatcher.joinable()) S->dispatcher.join();
  for (auto& t : S->finished_workers)
    if (t.joinable()) t.join();
  delete S;
}

}  // extern "C"
