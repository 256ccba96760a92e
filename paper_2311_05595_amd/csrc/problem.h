// Host runtime: a problem's hierarchy plan, device arena and solver.
#pragma once

#include <chrono>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/mgcg.h"
#include "kernels.h"

namespace mgcg {

struct LevelPlan {
  Lat L;
  int kind;          // OP_MF_Q1 / OP_ST27 / OP_EQ2 / OP_EQ3
  int ncx, ncy, ncz; // element grid of the level
};

// Device buffers of one level (V-cycle precision T for vectors and operator copies).
struct LevelBufs {
  uint8_t* mask = nullptr;
  double* KE = nullptr;      // Q1-type element matrices [nel][576] (levels >= 1; level 0 ST27: Keff)
  void* coefV = nullptr;     // stencil in V precision (levels >= 1, level 0 ST27)
  double* coef64 = nullptr;  // FP64 stencil (level 0 ST27 when V precision is FP32)
  void* invD = nullptr;      // [ndof] V precision
  double* diag64 = nullptr;  // [ndof]
  void* b = nullptr;         // [nrhs][ndof] V precision
  void* xa = nullptr;
  void* xb = nullptr;
  void* r = nullptr;
};

// HIP events around every launch of one kernel (id): 0 = the CG operator
// apply q = A p on the finest level, 1 = the finest-level pre-smoothing +
// residual apply, 2 = the finest-level post-smoothing Jacobi apply.
struct KernelTimer {
  bool enabled = false;
  int kernel = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::vector<int> recs;  // iteration index of each recorded launch
  size_t used = 0;
  double total_ms = 0.0;
  long long launches = 0;
};

// The HBM budget of a context (mgcg_ctx): the device bytes its problems hold
// may not exceed it (0: no limit).  Thread-safe.
struct Budget {
  std::mutex m;
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  int problems = 0;
  bool charge(size_t b) {
    std::lock_guard<std::mutex> g(m);
    if (budget && in_use + b > budget) return false;
    in_use += b;
    return true;
  }
  void refund(size_t b) {
    std::lock_guard<std::mutex> g(m);
    in_use -= b;
  }
  void attach(int d) {
    std::lock_guard<std::mutex> g(m);
    problems += d;
  }
};

class Problem {
 public:
  Problem(const mgcg_desc& d, const uint8_t* mask, const double* f, int device);
  ~Problem();

  static void plan_levels(const mgcg_desc& d, std::vector<LevelPlan>& lv);
  static size_t device_bytes(const mgcg_desc& d);

  void allocate();
  void release();
  bool allocated() const { return arena_ != nullptr; }
  size_t bytes() const { return bytes_; }

  void set_stream(hipStream_t s);
  hipStream_t stream() const { return stream_; }
  // The stream the problem runs on (its own, created now, unless one was set);
  // no device memory is allocated.
  hipStream_t ensure_stream();
  int device() const { return device_; }

  // charge this problem's device memory to a context's budget (before the
  // first allocation; the problem counts as attached until destroyed)
  void attach_budget(Budget* b);
  void set_densities(const double* rho, int mem);
  // the same from FP32 densities (converted to FP64 on the way in)
  void set_densities_f32(const float* rho, int mem);
  // Enqueue the refresh without waiting; the density check happens when the
  // next solve finishes.
  void set_densities_async(const double* rho, int mem);
  // Blocking solve.
  int solve(double rtol, int maxit, int warm, mgcg_info* info);
  // Non-blocking pieces used by the server.
  void solve_begin(double rtol, int maxit, int warm);  // warm: MGCG_COLD / _WARM_SCALED / _WARM_PLAIN
  void solve_chunk(int iters);             // enqueue iterations + state readback
  bool solve_poll(bool block);             // true when every load case finished
  // fills info; returns status.  bad: the set-up flags already on the host
  // (else read back here when a set-up is pending its check).
  int solve_finish(mgcg_info* info, const int* bad = nullptr);
  // Gives up a solve: waits for the work already enqueued on the stream and
  // leaves the problem idle (its u is whatever the last iteration wrote).
  void solve_abort();
  int suggest_chunk() const;
  bool solve_pending() const { return chunk_pending_; }

  void get_u(double* u, int mem);
  void set_u(const double* u, int mem);
  void compliance_sensitivity(double* c, double* dc, int mem);

  // inspection
  void level_dims(int level, int32_t* dims, int64_t* ndof) const;
  void apply(int level, int prec, const double* x, double* y, int mem);
  void diag(int level, double* d, int mem);
  void restrict_(int level, const double* f, double* c, int mem);
  void prolong(int level, const double* c, double* f, int mem);
  void precondition(const double* r, double* z, int mem);
  void coarse_solve(const double* b, double* x, int mem);

  // MGCG_LAUNCH_GRAPH: the PCG iterations of a chunk replay one captured
  // iteration (a HIP graph of its kernels); MGCG_LAUNCH_EAGER: launched one
  // by one (always while kernel timing is on); MGCG_LAUNCH_FUSED: the whole
  // solve in one launch, a workgroup per load case (fused_ok problems only).
  void set_launch_mode(int mode);
  int launch_mode() const { return launch_mode_; }
  // The problem fits the fused solve (trilinear nsub = 1, FP64, Jacobi, its
  // finest and coarsest levels within the workgroup's LDS).
  static bool fused_ok(const mgcg_desc& d, const std::vector<LevelPlan>& lv);
  bool fused_ok() const { return fused_ok(d_, lv_); }
  // Host descriptors of the fused solve of every load case (after
  // fused_prepare, which also zeroes x for a cold start).
  void fused_prepare(double rtol, int maxit, int warm, std::vector<FzDesc>& out);
  // Bookkeeping after a fused solve ran on the device (scalars copied back).
  int fused_finish(mgcg_info* info);
  // Batched solves: where this problem's end-of-solve record lives on the
  // device, and the bookkeeping from a record already copied to the host
  // (after the launch's stream has been synchronised).
  FzGatherSrc gather_src() const { return FzGatherSrc{cs_, bad_, d_.nrhs, 0}; }
  int fused_finish(const FzRecord& rec, mgcg_info* info);
  void set_timing(bool on, int kernel = 0);
  void get_timing(int kernel, double* ms, long long* launches);
  void copy(const void* src, void* dst, size_t bytes);

  const mgcg_desc& desc() const { return d_; }
  static size_t layout(const mgcg_desc& d, const std::vector<LevelPlan>& lv, char* base, Problem* s);
  long ndof0() const { return lv_[0].L.ndof(); }
  long nrho() const;
  double last_setup_ms() const { return setup_ms_; }

 private:
  template <typename T> void vcycle(const double* r_in, int gate, bool fuse_dot,
                                    bool x0_ready = false);
  void precondition_and_direction(bool x0_ready = false);
  VPrep vprep() const;
  // the finest level smooths by multicolour Gauss-Seidel
  bool gs_smoother() const {
    return d_.smoother == MGCG_SMOOTH_GAUSS_SEIDEL && lv_.size() > 1 && Kn_ != nullptr;
  }
  template <typename T> VOps<T> vops(int level) const;
  template <typename T> void do_set_densities();
  template <typename T> void do_apply_v(int level, const double* x, double* y);
  void iteration();
  int solve_fused(double rtol, int maxit, int warm, mgcg_info* info);
  void build_iter_graph();
  void drop_iter_graph();
  void build_linear_galerkin();
  FineOp fine_op() const;
  int nblocks_fine(bool fp64) const;
  void sync();
  void check_bad(int which);
  void timed_begin(int id);
  void timed_end(int id);
  void harvest_timing(int itmax);

  mgcg_desc d_;
  int device_;
  int vbytes_;  // 8 or 4
  std::vector<LevelPlan> lv_;
  std::vector<uint8_t> hmask_;  // per level node masks, concatenated
  std::vector<size_t> hmask_off_;
  std::vector<double> hf_;
  std::vector<double> hKsub_;
  std::vector<double> hKp_;
  std::vector<int> hfree_;      // coarsest free DOF list
  std::vector<double> hG_;      // linear Galerkin matrices of the first coarse level [M][576]
  std::vector<int> hmasked_;    // first-coarse-level elements with supported child DOFs
  int gB_ = 0;                  // density cells per axis of a first-level coarse element
  std::vector<int> hdofpos_;

  hipStream_t stream_ = nullptr;
  hipStream_t own_stream_ = nullptr;
  char* arena_ = nullptr;
  size_t bytes_ = 0;

  // device pointers
  std::vector<LevelBufs> B_;
  double* f_ = nullptr;
  double* rho_ = nullptr;
  double* E_ = nullptr;
  float* E32_ = nullptr;
  Q1HaarVals<double> hv64_{};  // the same in the element's Haar basis
  Q1HaarVals<float> hv32_{};
  double* Ksub_ = nullptr;   // [n^3][nd*nd]
  double* Kp_ = nullptr;     // n = 4: the packed sub-element matrices (sens_pack)
  double* K0_ = nullptr;     // [576] (MF)
  float* K032_ = nullptr;
  double* Keff_ = nullptr;   // level-0 effective element matrices (ST27: 576, EQ2: 6561)
  double* Kq2_ = nullptr;    // EQ2: the same by wrapped diagonals (Q2_PACKED per element)
  float* Keff32_ = nullptr;  // EQ2 mixed copy
  double* Yeq_ = nullptr;    // EQ2 element products (FP64 or FP32 view), [nrhs][nel][81]
  Budget* budget_ = nullptr;  // context budget this problem is charged to, or null
  void* Kn_ = nullptr;       // Gauss-Seidel smoother: element rows by node, V-cycle precision
  void* Dn_ = nullptr;       // and each node's 3x3 diagonal block
  double *x_ = nullptr, *r_ = nullptr, *p_ = nullptr, *q_ = nullptr;
  CgScalars* cs_ = nullptr;
  RedBuf red_{nullptr};
  double* compout_ = nullptr;
  int* bad_ = nullptr;
  int* dfree_ = nullptr;
  int* ddofpos_ = nullptr;
  double *Ad_ = nullptr, *Ad2_ = nullptr, *Dgj_ = nullptr, *diag0_ = nullptr;
  double* Ainv_ = nullptr;  // Ad_ or Ad2_, whichever holds the inverse
  double* G_ = nullptr;
  int* dmasked_ = nullptr;
  double* tmp64_ = nullptr;  // [nrhs][ndof0] scratch for inspection
  double* dcbuf_ = nullptr;  // [n_rho] sensitivity staging for host output
  void* zbuf_ = nullptr;     // level-0 V-cycle output of the last cycle
  CgScalars* hcs_ = nullptr; // pinned host copy
  FzDesc* fz_ = nullptr;     // fused solve: one descriptor per load case (fused_ok problems)

  int nc_ = 0;
  bool have_ops_ = false;
  bool have_u_ = false;
  double setup_ms_ = 0.0;
  // solve state
  double rtol_ = 0.0;
  int maxit_ = 0;
  int chunk_iters_done_ = 0;
  std::chrono::steady_clock::time_point t0_;
  hipEvent_t ev_chunk_ = nullptr;
  hipEvent_t ev_s0_ = nullptr, ev_s1_ = nullptr;
  bool chunk_pending_ = false;
  int iter_launched_ = 0;
  size_t timer_used_base_ = 0;
  bool first_chunk_ = true;
  bool prev_rr_valid_ = false;
  double prev_worst_ = 0.0;
  int prev_iters_ = 0;
  double rate_log_ = 0.0;
  bool active_ = false;
  int replace_every_ = 0;  // periodic residual replacement off: only at convergence
  bool pending_check_ = false;
  int launch_mode_ = MGCG_LAUNCH_EAGER;
  hipGraphExec_t iter_exec_ = nullptr;  // one PCG iteration, captured
  KernelTimer timer_;
};

const char* set_error(const std::string& m);
const char* get_error();

}  // namespace mgcg
