// Continuous-batching server over one GPU.
#pragma once

#include <chrono>
#include <deque>
#include <map>
#include <set>
#include <vector>

#include "problem.h"

struct mgcg_problem;

namespace mgcg {

Problem* problem_impl(mgcg_problem* p);

// Queue entry meaning "cannot start now" (its problem's previous solve still
// runs): skipped without blocking anything.
constexpr size_t kCannotStart = ~(size_t)0;

// Admission in queue order while slots are free: a request whose problem is
// already resident (0 bytes) starts at once; requests that need memory are
// first-come-first-served among themselves (one that does not fit blocks the
// memory-needing requests behind it, so large requests are not starved).
// Returns the number admitted.
int admission_plan(size_t budget, size_t in_use, int free_slots, const size_t* queue_bytes,
                   int nqueue, uint8_t* admit);

class Server {
 public:
  Server(int device, size_t budget, int max_slots);
  ~Server();
  uint64_t submit(Problem* p, const double* rho, int mem, double rtol, int maxit, int warm);
  void step(int* active, int* queued);
  int poll(uint64_t ticket, mgcg_info* info, double* latency_ms);
  void release(Problem* p);
  size_t resident_bytes() const { return in_use_; }

 private:
  struct Req {
    uint64_t ticket;
    Problem* p;
    std::vector<double> rho;   // host densities (submitted from host memory)
    double* drho = nullptr;    // device copy (submitted from device memory), stream-ordered
    double rtol;
    int maxit;
    int warm;
    int status = 0;
    mgcg_info info{};
    std::chrono::steady_clock::time_point t_submit, t_done;
  };
  bool busy(Problem* p) const;
  void admit();
  void finish(Req* r, int status);
  static void free_staging(Req* r);

  int device_;
  size_t budget_;
  int max_slots_;
  size_t in_use_ = 0;
  uint64_t next_ = 1;
  std::deque<Req*> queue_;
  std::vector<Req*> running_;
  std::map<uint64_t, Req*> done_;
  std::map<Problem*, size_t> resident_;
};

}  // namespace mgcg
