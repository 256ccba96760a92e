// Continuous batching of MGCG solves: admission by device-memory budget and
// free slots, one stream per resident problem so that solves of different
// sizes overlap on the device, and a step that advances every running solve
// by one chunk of PCG iterations without waiting on any of them.
#include "server.h"

#include <algorithm>
#include <memory>

namespace mgcg {

int admission_plan(size_t budget, size_t in_use, int free_slots, const size_t* queue_bytes,
                   int nqueue, uint8_t* admit) {
  int n = 0;
  bool blocked = false;  // a request needing memory did not fit
  for (int i = 0; i < nqueue; ++i) admit[i] = 0;
  for (int i = 0; i < nqueue && free_slots > 0; ++i) {
    const size_t b = queue_bytes[i];
    if (b == kCannotStart) continue;
    if (b > 0) {
      if (blocked) continue;
      if (b > budget || in_use + b > budget) {
        blocked = true;
        continue;
      }
    }
    admit[i] = 1;
    in_use += b;
    --free_slots;
    ++n;
  }
  return n;
}

Server::Server(int device, size_t budget, int max_slots)
    : device_(device), budget_(budget), max_slots_(max_slots) {
  if (max_slots < 1) throw Error(MGCG_EINVAL, "max_slots must be >= 1");
}

Server::~Server() {
  // A running request may be mid-solve: wait only for the work already
  // queued on its stream (no new chunk is launched), then drop it.
  for (Req* r : running_) {
    try {
      r->p->solve_abort();
    } catch (...) {
    }
    free_staging(r);
    delete r;
  }
  for (Req* r : queue_) {
    free_staging(r);
    delete r;
  }
  for (auto& kv : done_) delete kv.second;
}

// The device copy of a request's densities is released in stream order on
// its problem's stream, after every kernel that reads it.
void Server::free_staging(Req* r) {
  if (r->drho) {
    (void)hipFreeAsync(r->drho, r->p->stream());
    r->drho = nullptr;
  }
}

void Server::finish(Req* r, int status) {
  r->status = status;
  r->info.status = status;
  r->t_done = std::chrono::steady_clock::now();
  free_staging(r);
  done_[r->ticket] = r;
}

bool Server::busy(Problem* p) const {
  for (Req* r : running_)
    if (r->p == p) return true;
  return false;
}

uint64_t Server::submit(Problem* p, const double* rho, int mem, double rtol, int maxit, int warm) {
  if (p->device() != device_) throw Error(MGCG_EINVAL, "problem lives on another device");
  if (mem != MGCG_MEM_HOST && mem != MGCG_MEM_DEVICE) throw Error(MGCG_EINVAL, "bad memory kind");
  if (warm < MGCG_COLD || warm > MGCG_WARM_PLAIN) throw Error(MGCG_EINVAL, "bad warm-start mode");
  const size_t need = Problem::device_bytes(p->desc());
  if (need > budget_) throw Error(MGCG_EBUDGET, "problem exceeds the server's memory budget");
  std::unique_ptr<Req> r(new Req);
  r->p = p;
  if (mem == MGCG_MEM_HOST) {
    r->rho.assign(rho, rho + p->nrho());
  } else {
    // copied now, in order on the problem's stream: the caller's buffer may
    // be reused once this returns
    const size_t bytes = (size_t)p->nrho() * sizeof(double);
    hipStream_t st = p->ensure_stream();
    MGCG_HIP(hipMallocAsync((void**)&r->drho, bytes, st));
    MGCG_HIP(hipMemcpyAsync(r->drho, rho, bytes, hipMemcpyDeviceToDevice, st));
  }
  r->ticket = next_++;
  r->rtol = rtol;
  r->maxit = maxit;
  r->warm = warm;
  r->t_submit = std::chrono::steady_clock::now();
  queue_.push_back(r.get());
  return r.release()->ticket;
}

void Server::admit() {
  std::vector<size_t> bytes;
  for (Req* r : queue_) {
    if (busy(r->p))
      bytes.push_back(kCannotStart);  // its previous solve is still running
    else
      bytes.push_back(resident_.count(r->p) ? 0 : Problem::device_bytes(r->p->desc()));
  }
  std::vector<uint8_t> adm(queue_.size(), 0);
  const int free_slots = max_slots_ - (int)running_.size();
  if (admission_plan(budget_, in_use_, free_slots, bytes.data(), (int)bytes.size(), adm.data()) == 0)
    return;
  std::deque<Req*> rest;
  size_t i = 0;
  for (Req* r : queue_) {
    const bool take = adm[i++] && !busy(r->p);  // a problem queued twice starts once per step
    if (!take) {
      rest.push_back(r);
      continue;
    }
    // every failure (the allocation included) ends this request only; the
    // loop always completes, so no request is both admitted and queued
    try {
      if (!resident_.count(r->p)) {
        r->p->allocate();
        resident_[r->p] = r->p->bytes();
        in_use_ += r->p->bytes();
      }
      if (r->drho)
        r->p->set_densities_async(r->drho, MGCG_MEM_DEVICE);
      else
        r->p->set_densities_async(r->rho.data(), MGCG_MEM_HOST);
      r->p->solve_begin(r->rtol, r->maxit, r->warm);
      running_.push_back(r);
    } catch (const Error& e) {
      finish(r, e.code);
    } catch (const std::exception&) {
      finish(r, MGCG_ENOMEM);
    }
  }
  queue_.swap(rest);
}

void Server::step(int* active, int* queued) {
  admit();
  for (size_t i = 0; i < running_.size();) {
    Req* r = running_[i];
    bool finished = false;
    try {
      if (r->p->solve_poll(false)) {
        r->status = r->p->solve_finish(&r->info);
        finished = true;
      } else if (!r->p->solve_pending()) {
        r->p->solve_chunk(r->p->suggest_chunk());
      }
    } catch (const Error& e) {
      r->status = e.code;
      finished = true;
    }
    if (finished) {
      finish(r, r->status);
      running_.erase(running_.begin() + i);
    } else {
      ++i;
    }
  }
  admit();
  if (active) *active = (int)running_.size();
  if (queued) *queued = (int)queue_.size();
}

int Server::poll(uint64_t ticket, mgcg_info* info, double* latency_ms) {
  auto it = done_.find(ticket);
  if (it == done_.end()) return MGCG_EAGAIN;
  Req* r = it->second;
  if (info) *info = r->info;
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  const int st = r->status;
  done_.erase(it);
  delete r;
  return st;
}

void Server::release(Problem* p) {
  for (Req* r : queue_)
    if (r->p == p) throw Error(MGCG_ESTATE, "problem is queued");
  if (busy(p)) throw Error(MGCG_ESTATE, "problem is running");
  auto it = resident_.find(p);
  if (it == resident_.end()) return;
  in_use_ -= it->second;
  resident_.erase(it);
  p->release();
}

}  // namespace mgcg

struct mgcg_server {
  mgcg::Server* impl;
};

using mgcg::Error;

#define SGUARD(body)                    \
  try {                                 \
    mgcg::set_error("");                \
    body                                \
  } catch (const Error& e) {            \
    mgcg::set_error(e.what());          \
    return e.code;                      \
  } catch (const std::exception& e) {   \
    mgcg::set_error(e.what());          \
    return MGCG_EINVAL;                 \
  }

extern "C" {

int mgcg_server_create(int device, size_t hbm_budget, int max_slots, mgcg_server** out) {
  if (!out) return MGCG_EINVAL;
  SGUARD({
    *out = new mgcg_server{new mgcg::Server(device, hbm_budget, max_slots)};
    return MGCG_OK;
  })
}

int mgcg_server_destroy(mgcg_server* s) {
  if (!s) return MGCG_OK;
  SGUARD({
    delete s->impl;
    delete s;
    return MGCG_OK;
  })
}

int mgcg_server_submit(mgcg_server* s, mgcg_problem* p, const double* rho, int mem, double rtol,
                       int maxit, int warm_start, uint64_t* ticket) {
  if (!s || !p || !rho || !ticket) {
    mgcg::set_error("null argument");
    return MGCG_EINVAL;
  }
  SGUARD({
    *ticket = s->impl->submit(mgcg::problem_impl(p), rho, mem, rtol, maxit, warm_start);
    return MGCG_OK;
  })
}

int mgcg_server_step(mgcg_server* s, int* active, int* queued) {
  if (!s) return MGCG_EINVAL;
  SGUARD({
    s->impl->step(active, queued);
    return MGCG_OK;
  })
}

int mgcg_server_poll(mgcg_server* s, uint64_t ticket, mgcg_info* info, double* latency_ms) {
  if (!s) return MGCG_EINVAL;
  SGUARD({ return s->impl->poll(ticket, info, latency_ms); })
}

int mgcg_server_release(mgcg_server* s, mgcg_problem* p) {
  if (!s || !p) return MGCG_EINVAL;
  SGUARD({
    s->impl->release(mgcg::problem_impl(p));
    return MGCG_OK;
  })
}

size_t mgcg_server_resident_bytes(mgcg_server* s) { return s ? s->impl->resident_bytes() : 0; }

}  // extern "C"
