// Request server: continuous batching of single-core-state solves over
// device-resident systems.
//
// Each request (one core state of a resident molecule) is the whole path:
// gwc_sigma_core for that state, then the cumulant spectral function from its
// Im Sigma.  The server owns n_slots worker threads, each with its own HIP
// stream.  A free worker takes the oldest queued request as soon as the
// request's predicted device footprint fits in the HBM budget next to the
// requests already running (gwc::Admission, gwc_admission.h), so requests
// arriving while others are on the GPU start as slots and memory free up, and
// the kernels of concurrent requests (molecules of different sizes) overlap on
// the device.  Every request's work
// is decomposed the same way whatever runs beside it (the batch sizes depend
// only on the request and the server's per-request batch budget), so its
// results do not depend on the mix.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gwc.h"
#include "gwc_admission.h"
#include "gwc_host.h"

gwc::ResidentSystem *gwc_handle_system(gwc_system_handle h);

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  gwc::ResidentSystem *sys = nullptr;
  int core = 0;
  std::vector<double> omega_imag, w_imag, omega_real;
  double eta = 0.0, vxc = 0.0;
  int mode = GWC_MODE_DECOUPLED, precision = GWC_PREC_FP64;
  int n_t = 0, n_out = 0;
  double d_omega = 0.0, out_min_rel = 0.0;
  size_t footprint = 0;
  size_t kept = 0;  // bytes this request built for its system (the split operands)
  // results
  bool done = false;
  bool claimed = false;  // a gwc_server_wait holds this ticket (set under the server lock)
  int status = GWC_OK;
  std::string error;
  double e_qp = 0.0, sigma_x = 0.0, sigma_c_eps[2] = {0.0, 0.0}, z[2] = {0.0, 0.0};
  std::vector<double> im_dec, A, sigma_c;
  double t_submit = 0.0, t_start = 0.0, t_end = 0.0;
};

}  // namespace

struct gwc_server_s {
  int n_slots = 1;
  size_t budget = 0, batch_bytes = 0;
  int device = 0;
  Clock::time_point t0;
  std::unique_ptr<gwc::Admission<Request>> adm;
  std::mutex mu;  // request table and completion flags
  std::condition_variable cv;
  std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_id = 1;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

void execute(gwc_server_s *srv, Request *r, hipStream_t s) {
  try {
    const int nr = (int)r->omega_real.size();
    gwc_sigma_args a{};
    int32_t core = r->core;
    a.n_core = 1;
    a.core_idx = &core;
    a.n_imag = (int)r->omega_imag.size();
    a.omega_imag = r->omega_imag.data();
    a.w_imag = r->w_imag.data();
    a.n_real = nr;
    a.omega_real = r->omega_real.data();
    a.eta = r->eta;
    a.vxc = &r->vxc;
    a.mode = r->mode;
    a.precision = r->precision;
    r->im_dec.assign(nr, 0.0);
    if (r->mode == GWC_MODE_FULL) r->sigma_c.assign(2 * (size_t)nr, 0.0);
    // the split operands first, so that the bytes this request leaves behind
    // are known to the admission
    r->kept = gwc::prepare_mixed_operands(*r->sys, r->precision, s);
    gwc_sigma_out o{};
    o.sigma_c = r->mode == GWC_MODE_FULL ? r->sigma_c.data() : nullptr;
    o.im_sigma_dec = r->im_dec.data();
    o.sigma_c_eps = r->sigma_c_eps;
    o.sigma_x = &r->sigma_x;
    o.e_qp = &r->e_qp;
    gwc::run_sigma(*r->sys, &a, &o, s, srv->batch_bytes);
    if (r->n_t > 0) {
      r->A.assign(r->n_out, 0.0);
      gwc_cumulant_args c{};
      c.n_real = nr;
      c.omega_real = r->omega_real.data();
      c.im_sigma = r->im_dec.data();
      c.eps_n = gwc::resident_eps(*r->sys, r->core);
      c.e_qp = r->e_qp;
      c.eta = r->eta;
      c.n_t = r->n_t;
      c.d_omega = r->d_omega;
      c.n_out = r->n_out;
      c.omega_out_min = r->e_qp + r->out_min_rel;
      gwc::run_cumulant(&c, r->A.data(), r->z, s);
    }
    r->status = GWC_OK;
  } catch (const gwc::GwcError &e) {
    r->status = e.code;
    r->error = e.msg;
  } catch (const std::exception &e) {
    r->status = GWC_ERR_DEVICE;
    r->error = e.what();
  }
}

void worker_loop(gwc_server_s *srv, int slot) {
  (void)hipSetDevice(srv->device);
  hipStream_t s = srv->streams[slot];
  for (;;) {
    size_t footprint = 0;
    bool refused = false;
    Request *r = srv->adm->acquire(footprint, nullptr, &refused);
    if (!r) return;
    if (refused) {
      std::lock_guard<std::mutex> lock(srv->mu);
      r->status = GWC_ERR_OUT_OF_MEMORY;
      r->error = "request footprint no longer fits beside the split operands kept for resident systems";
      r->t_start = r->t_end = srv->now();
      r->done = true;
      srv->cv.notify_all();
      continue;
    }
    {
      std::lock_guard<std::mutex> lock(srv->mu);
      r->t_start = srv->now();
    }
    execute(srv, r, s);
    {
      std::lock_guard<std::mutex> lock(srv->mu);
      r->t_end = srv->now();
      r->done = true;
    }
    srv->adm->release(footprint, r->kept);
    srv->cv.notify_all();
  }
}

template <class F>
int guarded_server(F &&fn) {
  std::string &err = gwc::last_error();
  err.clear();
  try {
    return fn();
  } catch (const gwc::GwcError &e) {
    err = e.msg;
    return e.code;
  } catch (const std::exception &e) {
    err = e.what();
    return GWC_ERR_DEVICE;
  }
}

}  // namespace

extern "C" {

int gwc_server_create(const gwc_server_config *cfg, gwc_server_handle *out) {
  return guarded_server([&] {
    if (!cfg || !out) gwc::fail(GWC_ERR_INVALID_ARG, "NULL config or handle");
    if (cfg->n_slots < 1 || cfg->n_slots > 64) gwc::fail(GWC_ERR_INVALID_ARG, "n_slots must be in [1, 64]");
    if (!(cfg->hbm_budget_bytes > 0)) gwc::fail(GWC_ERR_INVALID_ARG, "hbm_budget_bytes must be > 0");
    std::unique_ptr<gwc_server_s> srv(new gwc_server_s());
    srv->n_slots = cfg->n_slots;
    srv->budget = (size_t)cfg->hbm_budget_bytes;
    srv->batch_bytes = cfg->batch_bytes > 0 ? (size_t)cfg->batch_bytes : srv->budget / 4;
    srv->adm.reset(new gwc::Admission<Request>(srv->budget));
    srv->t0 = Clock::now();
    if (hipGetDevice(&srv->device) != hipSuccess) {
      (void)hipGetLastError();
      gwc::fail(GWC_ERR_DEVICE, "no HIP device");
    }
    for (int i = 0; i < srv->n_slots; ++i) {
      hipStream_t st;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        for (hipStream_t x : srv->streams) (void)hipStreamDestroy(x);
        gwc::fail(GWC_ERR_DEVICE, "hipStreamCreate failed");
      }
      srv->streams.push_back(st);
    }
    gwc_server_s *p = srv.release();
    for (int i = 0; i < p->n_slots; ++i) p->workers.emplace_back(worker_loop, p, i);
    *out = p;
    return GWC_OK;
  });
}

int gwc_server_submit(gwc_server_handle srv, const gwc_request *rq, int64_t *ticket) {
  return guarded_server([&] {
    if (!srv || !rq || !ticket) gwc::fail(GWC_ERR_INVALID_ARG, "NULL server, request or ticket");
    gwc::ResidentSystem *sys = gwc_handle_system(rq->system);
    if (!sys) gwc::fail(GWC_ERR_INVALID_ARG, "NULL system handle");
    if (rq->core_idx < 0 || rq->core_idx >= gwc::resident_n_occ(*sys))
      gwc::fail(GWC_ERR_SHAPE, "core_idx %d not in [0, n_occ)", rq->core_idx);
    if (rq->n_imag < 1 || rq->n_real < 1 || !rq->omega_imag || !rq->w_imag || !rq->omega_real)
      gwc::fail(GWC_ERR_INVALID_ARG, "grids missing");
    if (rq->n_t > 0 && (rq->n_out < 1 || rq->n_out > rq->n_t))
      gwc::fail(GWC_ERR_SHAPE, "n_out must be in [1, n_t]");
    std::unique_ptr<Request> r(new Request());
    r->sys = sys;
    r->core = rq->core_idx;
    r->omega_imag.assign(rq->omega_imag, rq->omega_imag + rq->n_imag);
    r->w_imag.assign(rq->w_imag, rq->w_imag + rq->n_imag);
    r->omega_real.assign(rq->omega_real, rq->omega_real + rq->n_real);
    r->eta = rq->eta;
    r->vxc = rq->vxc;
    r->mode = rq->mode;
    r->precision = rq->precision;
    r->n_t = rq->n_t;
    r->d_omega = rq->d_omega;
    r->n_out = rq->n_out;
    r->out_min_rel = rq->omega_out_min_rel;
    gwc_sigma_args a{};
    a.n_core = 1;
    a.n_imag = rq->n_imag;
    a.n_real = rq->n_real;
    a.mode = rq->mode;
    a.precision = rq->precision;
    // transient device memory, plus the split operands when this request may
    // be the one that builds them (they then stay with the system)
    r->footprint = gwc::predict_sigma_bytes(*sys, &a, srv->batch_bytes) +
                   (rq->n_t > 0 ? gwc::predict_cumulant_bytes(rq->n_real, rq->n_t, rq->n_out) : 0) +
                   gwc::mixed_operand_bytes(*sys, rq->precision);
    const size_t room = srv->budget - srv->adm->stats().kept;
    if (r->footprint > room)
      gwc::fail(GWC_ERR_OUT_OF_MEMORY, "request footprint %zu bytes exceeds the budget left, %zu of %zu",
                r->footprint, room, srv->budget);
    {
      // table entry and queue position under one lock: tickets follow queue order
      std::lock_guard<std::mutex> lock(srv->mu);
      r->id = srv->next_id++;
      r->t_submit = srv->now();
      *ticket = r->id;
      Request *rp = r.get();
      srv->reqs.emplace(rp->id, std::move(r));
      if (!srv->adm->submit(rp, rp->footprint)) {  // kept bytes grew since the check above
        const size_t fp = rp->footprint;
        srv->reqs.erase(rp->id);
        gwc::fail(GWC_ERR_OUT_OF_MEMORY, "request footprint %zu bytes exceeds the budget left", fp);
      }
    }
    return GWC_OK;
  });
}

int gwc_server_wait(gwc_server_handle srv, int64_t ticket, gwc_request_result *res) {
  return guarded_server([&] {
    if (!srv || !res) gwc::fail(GWC_ERR_INVALID_ARG, "NULL server or result");
    std::unique_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lock(srv->mu);
      auto it = srv->reqs.find(ticket);
      if (it == srv->reqs.end()) gwc::fail(GWC_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
      Request *rp = it->second.get();
      // one waiter per ticket: a second wait would find the entry erased and
      // its Request freed once the first returns
      if (rp->claimed) gwc::fail(GWC_ERR_INVALID_ARG, "ticket %lld is already being waited on", (long long)ticket);
      rp->claimed = true;
      srv->cv.wait(lock, [&] { return rp->done; });
      // the map's iterator may be stale after the wait (other tickets were
      // inserted or erased meanwhile): look the ticket up again
      auto again = srv->reqs.find(ticket);
      r = std::move(again->second);
      srv->reqs.erase(again);
    }
    res->status = r->status;
    res->e_qp = r->e_qp;
    res->sigma_x = r->sigma_x;
    res->sigma_c_eps[0] = r->sigma_c_eps[0];
    res->sigma_c_eps[1] = r->sigma_c_eps[1];
    res->z[0] = r->z[0];
    res->z[1] = r->z[1];
    res->t_submit = r->t_submit;
    res->t_start = r->t_start;
    res->t_end = r->t_end;
    res->footprint_bytes = (double)r->footprint;
    if (res->im_sigma_dec) std::copy(r->im_dec.begin(), r->im_dec.end(), res->im_sigma_dec);
    if (res->A && !r->A.empty()) std::copy(r->A.begin(), r->A.end(), res->A);
    if (res->sigma_c && !r->sigma_c.empty()) std::copy(r->sigma_c.begin(), r->sigma_c.end(), res->sigma_c);
    if (r->status != GWC_OK) gwc::last_error() = r->error;
    return r->status;
  });
}

int gwc_server_stats(gwc_server_handle srv, gwc_server_stats_t *st) {
  return guarded_server([&] {
    if (!srv || !st) gwc::fail(GWC_ERR_INVALID_ARG, "NULL server or stats");
    const auto a = srv->adm->stats();
    st->queued = (int32_t)a.queued;
    st->active = a.active;
    st->peak_active = a.peak_active;
    st->completed = a.completed;
    st->in_use_bytes = (double)a.in_use;
    st->peak_in_use_bytes = (double)a.peak_in_use;
    st->budget_bytes = (double)srv->budget;
    st->kept_bytes = (double)a.kept;
    st->refused = a.refused;
    return GWC_OK;
  });
}

int gwc_server_destroy(gwc_server_handle srv) {
  return guarded_server([&] {
    if (!srv) gwc::fail(GWC_ERR_INVALID_ARG, "NULL server");
    srv->adm->stop();
    for (auto &t : srv->workers) t.join();
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    delete srv;
    return GWC_OK;
  });
}

}  // extern "C"
