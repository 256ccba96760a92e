// extern "C" boundary: argument checks, exception-to-status translation and
// the thread-local error message.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "problem.h"
#include "server.h"

namespace mgcg {
namespace {
thread_local std::string g_err;
}
const char* set_error(const std::string& m) {
  g_err = m;
  return g_err.c_str();
}
const char* get_error() { return g_err.c_str(); }
}  // namespace mgcg

using mgcg::Error;
using mgcg::Problem;
using mgcg::FzDesc;
using mgcg::FzGatherSrc;
using mgcg::FzRecord;

#define GUARD(body)                                 \
  try {                                             \
    mgcg::set_error("");                            \
    body                                            \
  } catch (const Error& e) {                        \
    mgcg::set_error(e.what());                      \
    return e.code;                                  \
  } catch (const std::exception& e) {               \
    mgcg::set_error(e.what());                      \
    return MGCG_EINVAL;                             \
  } catch (...) {                                   \
    mgcg::set_error("unknown error");               \
    return MGCG_EINVAL;                             \
  }

#define NEED(ptr)                                                         \
  if (!(ptr)) {                                                           \
    mgcg::set_error(std::string("null argument: ") + #ptr);              \
    return MGCG_EINVAL;                                                   \
  }

struct mgcg_problem {
  Problem* impl;
};
struct mgcg_ctx {
  mgcg::Budget b;
};

extern "C" {

const char* mgcg_last_error(void) { return mgcg::get_error(); }

int mgcg_version(void) { return 10000; }

size_t mgcg_problem_device_bytes(const mgcg_desc* d) {
  if (!d) return 0;
  try {
    return Problem::device_bytes(*d);
  } catch (...) {
    return 0;
  }
}

int mgcg_problem_create(const mgcg_desc* d, const uint8_t* mask, const double* f, int device,
                        mgcg_problem** out) {
  NEED(d);
  NEED(mask);
  NEED(f);
  NEED(out);
  GUARD({
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (device < 0 || (ndev > 0 && device >= ndev)) throw Error(MGCG_EINVAL, "bad device index");
    auto* p = new mgcg_problem{nullptr};
    try {
      p->impl = new Problem(*d, mask, f, device);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
    return MGCG_OK;
  })
}

int mgcg_ctx_create(mgcg_ctx** out, int device, size_t hbm_budget_bytes) {
  NEED(out);
  GUARD({
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (device < 0 || (ndev > 0 && device >= ndev)) throw Error(MGCG_EINVAL, "bad device index");
    auto* c = new mgcg_ctx;
    c->b.device = device;
    c->b.budget = hbm_budget_bytes;
    *out = c;
    return MGCG_OK;
  })
}

int mgcg_ctx_destroy(mgcg_ctx* c) {
  if (!c) return MGCG_OK;
  GUARD({
    int n;
    {
      std::lock_guard<std::mutex> g(c->b.m);
      n = c->b.problems;
    }
    if (n > 0) throw Error(MGCG_EINVAL, "problems of this context are still alive");
    delete c;
    return MGCG_OK;
  })
}

int mgcg_ctx_usage(mgcg_ctx* c, size_t* in_use, size_t* budget, int32_t* problems) {
  NEED(c);
  GUARD({
    std::lock_guard<std::mutex> g(c->b.m);
    if (in_use) *in_use = c->b.in_use;
    if (budget) *budget = c->b.budget;
    if (problems) *problems = c->b.problems;
    return MGCG_OK;
  })
}

int mgcg_problem_create_in(mgcg_ctx* c, const mgcg_desc* d, const uint8_t* mask, const double* f,
                           mgcg_problem** out) {
  NEED(c);
  NEED(d);
  NEED(mask);
  NEED(f);
  NEED(out);
  GUARD({
    auto* p = new mgcg_problem{nullptr};
    try {
      p->impl = new Problem(*d, mask, f, c->b.device);
      p->impl->attach_budget(&c->b);
    } catch (...) {
      delete p->impl;
      delete p;
      throw;
    }
    *out = p;
    return MGCG_OK;
  })
}

int mgcg_set_densities_f32(mgcg_problem* p, const float* rho, int mem) {
  NEED(p);
  NEED(rho);
  GUARD({
    p->impl->set_densities_f32(rho, mem);
    return MGCG_OK;
  })
}

int mgcg_problem_destroy(mgcg_problem* p) {
  if (!p) return MGCG_OK;
  GUARD({
    delete p->impl;
    delete p;
    return MGCG_OK;
  })
}

int mgcg_set_stream(mgcg_problem* p, void* stream) {
  NEED(p);
  GUARD({
    p->impl->allocate();
    p->impl->set_stream((hipStream_t)stream);
    return MGCG_OK;
  })
}

int mgcg_get_stream(mgcg_problem* p, void** stream) {
  NEED(p);
  if (!stream) {
    mgcg::set_error("null argument");
    return MGCG_EINVAL;
  }
  GUARD({
    *stream = (void*)p->impl->ensure_stream();
    return MGCG_OK;
  })
}

int mgcg_set_launch_mode(mgcg_problem* p, int mode) {
  NEED(p);
  GUARD({
    p->impl->set_launch_mode(mode);
    return MGCG_OK;
  })
}

int mgcg_problem_allocate(mgcg_problem* p) {
  NEED(p);
  GUARD({
    p->impl->allocate();
    return MGCG_OK;
  })
}

int mgcg_set_densities(mgcg_problem* p, const double* rho, int mem) {
  NEED(p);
  NEED(rho);
  GUARD({
    p->impl->set_densities(rho, mem);
    return MGCG_OK;
  })
}

int mgcg_solve(mgcg_problem* p, double rtol, int maxit, int warm_start, mgcg_info* info) {
  NEED(p);
  if (warm_start < MGCG_COLD || warm_start > MGCG_WARM_PLAIN) {
    mgcg::set_error("warm_start must be MGCG_COLD, MGCG_WARM_SCALED or MGCG_WARM_PLAIN");
    return MGCG_EINVAL;
  }
  GUARD({ return p->impl->solve(rtol, maxit, warm_start, info); })
}

namespace {
// One batch table per device, grown as needed and kept; batches share it, so
// they run one at a time.  Device: the load cases' descriptors, the
// problems' record sources and their packed records; pinned host: the same
// layout (staging for the upload, then the records read back).
struct BatchTable {
  void* dev = nullptr;
  void* host = nullptr;
  size_t bytes = 0;
};
std::mutex g_batch_mu;
std::vector<BatchTable> g_batch_tables;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Events of one batch call, destroyed on every way out of it.
struct EventList {
  std::vector<hipEvent_t> ev;
  ~EventList() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  hipEvent_t add() {
    hipEvent_t e;
    MGCG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ev.push_back(e);
    return e;
  }
};

int solve_batch(mgcg_problem* const* ps, int n, double rtol, int maxit, int warm_start,
                mgcg_info* infos) {
  std::lock_guard<std::mutex> g(g_batch_mu);
  Problem* p0 = ps[0]->impl;
  const int dev = p0->device();
  for (int i = 0; i < n; ++i) {
    if (ps[i]->impl->device() != dev) throw Error(MGCG_EINVAL, "batched problems must share a device");
    if (!ps[i]->impl->fused_ok())
      throw Error(MGCG_EINVAL, "a batched problem does not fit the fused solve");
    for (int j = 0; j < i; ++j)
      if (ps[j]->impl == ps[i]->impl) throw Error(MGCG_EINVAL, "a problem appears twice in the batch");
  }
  MGCG_HIP(hipSetDevice(dev));
  std::vector<FzDesc> all, one;
  for (int i = 0; i < n; ++i) {
    ps[i]->impl->fused_prepare(rtol, maxit, warm_start, one);
    all.insert(all.end(), one.begin(), one.end());
  }
  const size_t o_src = align256(all.size() * sizeof(FzDesc));
  const size_t o_rec = o_src + align256(n * sizeof(FzGatherSrc));
  const size_t bytes = o_rec + n * sizeof(FzRecord);
  if ((int)g_batch_tables.size() <= dev) g_batch_tables.resize(dev + 1);
  BatchTable& tb = g_batch_tables[dev];
  hipStream_t st = p0->ensure_stream();
  if (tb.bytes < bytes) {
    if (tb.dev) {
      MGCG_HIP(hipDeviceSynchronize());
      MGCG_HIP(hipFree(tb.dev));
      MGCG_HIP(hipHostFree(tb.host));
      tb = BatchTable{};
    }
    if (hipMalloc(&tb.dev, bytes) != hipSuccess) {
      (void)hipGetLastError();
      tb = BatchTable{};
      throw Error(MGCG_ENOMEM, "batch table device allocation failed");
    }
    if (hipHostMalloc(&tb.host, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(tb.dev);
      tb = BatchTable{};
      throw Error(MGCG_ENOMEM, "batch table host buffer allocation failed");
    }
    tb.bytes = bytes;
  }
  char* hb = static_cast<char*>(tb.host);
  char* db = static_cast<char*>(tb.dev);
  std::memcpy(hb, all.data(), all.size() * sizeof(FzDesc));
  FzGatherSrc* hsrc = reinterpret_cast<FzGatherSrc*>(hb + o_src);
  for (int i = 0; i < n; ++i) hsrc[i] = ps[i]->impl->gather_src();
  // the launch follows the work still pending on every problem's stream
  EventList evs;
  for (int i = 1; i < n; ++i) {
    hipStream_t si = ps[i]->impl->ensure_stream();
    const hipError_t q = hipStreamQuery(si);
    if (q == hipSuccess) continue;
    if (q != hipErrorNotReady) MGCG_HIP(q);
    (void)hipGetLastError();
    const hipEvent_t e = evs.add();
    MGCG_HIP(hipEventRecord(e, si));
    MGCG_HIP(hipStreamWaitEvent(st, e, 0));
  }
  MGCG_HIP(hipMemcpyAsync(db, hb, o_rec, hipMemcpyHostToDevice, st));
  mgcg::fused_solve(reinterpret_cast<const FzDesc*>(db), (int)all.size(), st);
  FzRecord* drec = reinterpret_cast<FzRecord*>(db + o_rec);
  mgcg::fused_gather(reinterpret_cast<const FzGatherSrc*>(db + o_src), n, drec, st);
  MGCG_HIP(hipMemcpyAsync(hb + o_rec, drec, n * sizeof(FzRecord), hipMemcpyDeviceToHost, st));
  // all done on return: later work on any problem's stream follows it
  MGCG_HIP(hipStreamSynchronize(st));
  const FzRecord* hrec = reinterpret_cast<const FzRecord*>(hb + o_rec);
  int status = MGCG_OK;
  for (int i = 0; i < n; ++i) {
    const int si = ps[i]->impl->fused_finish(hrec[i], infos ? &infos[i] : nullptr);
    if (status == MGCG_OK && si != MGCG_OK) status = si;
  }
  return status;
}
}  // namespace

int mgcg_solve_batch(mgcg_problem* const* ps, int n, double rtol, int maxit, int warm_start,
                     mgcg_info* infos) {
  NEED(ps);
  if (n < 1) {
    mgcg::set_error("need n >= 1 problems");
    return MGCG_EINVAL;
  }
  if (warm_start < MGCG_COLD || warm_start > MGCG_WARM_PLAIN) {
    mgcg::set_error("warm_start must be MGCG_COLD, MGCG_WARM_SCALED or MGCG_WARM_PLAIN");
    return MGCG_EINVAL;
  }
  for (int i = 0; i < n; ++i) NEED(ps[i]);
  GUARD({ return solve_batch(ps, n, rtol, maxit, warm_start, infos); })
}

int mgcg_get_displacement(mgcg_problem* p, double* u, int mem) {
  NEED(p);
  NEED(u);
  GUARD({
    p->impl->get_u(u, mem);
    return MGCG_OK;
  })
}

int mgcg_set_initial_guess(mgcg_problem* p, const double* u, int mem) {
  NEED(p);
  NEED(u);
  GUARD({
    p->impl->set_u(u, mem);
    return MGCG_OK;
  })
}

int mgcg_compliance_sensitivity(mgcg_problem* p, double* c, double* dc, int mem) {
  NEED(p);
  NEED(c);
  GUARD({
    p->impl->compliance_sensitivity(c, dc, mem);
    return MGCG_OK;
  })
}

int mgcg_level_dims(mgcg_problem* p, int level, int32_t* dims3, int64_t* ndof) {
  NEED(p);
  GUARD({
    p->impl->level_dims(level, dims3, ndof);
    return MGCG_OK;
  })
}

int mgcg_apply(mgcg_problem* p, int level, int prec, const double* x, double* y, int mem) {
  NEED(p);
  NEED(x);
  NEED(y);
  GUARD({
    p->impl->apply(level, prec, x, y, mem);
    return MGCG_OK;
  })
}

int mgcg_level_diag(mgcg_problem* p, int level, double* d, int mem) {
  NEED(p);
  NEED(d);
  GUARD({
    p->impl->diag(level, d, mem);
    return MGCG_OK;
  })
}

int mgcg_restrict(mgcg_problem* p, int level, const double* fine, double* coarse, int mem) {
  NEED(p);
  NEED(fine);
  NEED(coarse);
  GUARD({
    p->impl->restrict_(level, fine, coarse, mem);
    return MGCG_OK;
  })
}

int mgcg_prolong(mgcg_problem* p, int level, const double* coarse, double* fine, int mem) {
  NEED(p);
  NEED(fine);
  NEED(coarse);
  GUARD({
    p->impl->prolong(level, coarse, fine, mem);
    return MGCG_OK;
  })
}

int mgcg_precondition(mgcg_problem* p, const double* r, double* z, int mem) {
  NEED(p);
  NEED(r);
  NEED(z);
  GUARD({
    p->impl->precondition(r, z, mem);
    return MGCG_OK;
  })
}

int mgcg_coarse_solve(mgcg_problem* p, const double* b, double* x, int mem) {
  NEED(p);
  NEED(b);
  NEED(x);
  GUARD({
    p->impl->coarse_solve(b, x, mem);
    return MGCG_OK;
  })
}

int mgcg_set_kernel_timing(mgcg_problem* p, int enable) {
  NEED(p);
  GUARD({
    p->impl->set_timing(enable > 0, enable > 0 ? enable - 1 : 0);
    return MGCG_OK;
  })
}

int mgcg_get_kernel_timing(mgcg_problem* p, int kernel, double* total_ms, int64_t* launches) {
  NEED(p);
  GUARD({
    long long n = 0;
    p->impl->get_timing(kernel, total_ms, &n);
    if (launches) *launches = n;
    return MGCG_OK;
  })
}

int mgcg_copy_bytes(mgcg_problem* p, const void* src, void* dst, size_t bytes) {
  NEED(p);
  NEED(src);
  NEED(dst);
  GUARD({
    p->impl->copy(src, dst, bytes);
    return MGCG_OK;
  })
}

int mgcg_admission_plan(size_t budget, size_t in_use, int free_slots, const size_t* queue_bytes,
                        int nqueue, uint8_t* admit) {
  if (nqueue < 0 || (nqueue > 0 && (!queue_bytes || !admit))) {
    mgcg::set_error("bad admission arguments");
    return MGCG_EINVAL;
  }
  return mgcg::admission_plan(budget, in_use, free_slots, queue_bytes, nqueue, admit);
}

}  // extern "C"

// accessor for the server
namespace mgcg {
Problem* problem_impl(mgcg_problem* p) { return p ? p->impl : nullptr; }
}  // namespace mgcg

// ---- projection / density filter
#include "proj.h"

struct mgcg_proj {
  mgcg::Proj* impl;
};

extern "C" {

size_t mgcg_proj_device_bytes(const mgcg_proj_desc* d) {
  if (!d) return 0;
  try {
    return mgcg::Proj::device_bytes(*d);
  } catch (...) {
    return 0;
  }
}

int mgcg_proj_create(const mgcg_proj_desc* d, int device, mgcg_proj** out) {
  NEED(d);
  NEED(out);
  GUARD({
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (device < 0 || (ndev > 0 && device >= ndev)) throw Error(MGCG_EINVAL, "bad device index");
    (void)mgcg::Proj::geometry(*d);
    auto* p = new mgcg_proj{nullptr};
    try {
      p->impl = new mgcg::Proj(*d, device);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
    return MGCG_OK;
  })
}

int mgcg_proj_destroy(mgcg_proj* pr) {
  NEED(pr);
  GUARD({
    delete pr->impl;
    delete pr;
    return MGCG_OK;
  })
}

int mgcg_proj_set_stream(mgcg_proj* pr, void* stream) {
  NEED(pr);
  GUARD({
    pr->impl->set_stream((hipStream_t)stream);
    return MGCG_OK;
  })
}

int mgcg_proj_apply(mgcg_proj* pr, const double* x, double* rho, int mem) {
  NEED(pr);
  NEED(x);
  NEED(rho);
  GUARD({
    pr->impl->run(false, x, rho, mem);
    return MGCG_OK;
  })
}

int mgcg_proj_apply_transpose(mgcg_proj* pr, const double* g, double* gx, int mem) {
  NEED(pr);
  NEED(g);
  NEED(gx);
  GUARD({
    pr->impl->run(true, g, gx, mem);
    return MGCG_OK;
  })
}

}  // extern "C"

// ---- SLP step
#include "lp.h"

struct mgcg_lp {
  mgcg::Lp* impl;
};

extern "C" {

size_t mgcg_lp_device_bytes(int64_t n) {
  if (n < 1 || n > (1LL << 31)) return 0;
  return mgcg::Lp::device_bytes((long)n);
}

int mgcg_lp_create(int64_t n, int device, mgcg_lp** out) {
  NEED(out);
  GUARD({
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (device < 0 || (ndev > 0 && device >= ndev)) throw Error(MGCG_EINVAL, "bad device index");
    auto* p = new mgcg_lp{nullptr};
    try {
      p->impl = new mgcg::Lp((long)n, device);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
    return MGCG_OK;
  })
}

int mgcg_lp_destroy(mgcg_lp* lp) {
  NEED(lp);
  GUARD({
    delete lp->impl;
    delete lp;
    return MGCG_OK;
  })
}

int mgcg_lp_set_stream(mgcg_lp* lp, void* stream) {
  NEED(lp);
  GUARD({
    lp->impl->set_stream((hipStream_t)stream);
    return MGCG_OK;
  })
}

int mgcg_lp_solve(mgcg_lp* lp, const double* g, const double* a, const double* x, double b,
                  double delta, double x_l, double x_u, double* s, mgcg_lp_info* info, int mem) {
  NEED(lp);
  GUARD({
    lp->impl->solve(g, a, x, nullptr, b, delta, x_l, x_u, s, info, mem);
    return MGCG_OK;
  })
}

int mgcg_lp_solve_fixed(mgcg_lp* lp, const double* g, const double* a, const double* x,
                        const uint8_t* fixed, double b, double delta, double x_l, double x_u,
                        double* s, mgcg_lp_info* info, int mem) {
  NEED(lp);
  NEED(fixed);
  GUARD({
    lp->impl->solve(g, a, x, fixed, b, delta, x_l, x_u, s, info, mem);
    return MGCG_OK;
  })
}

int mgcg_threshold_lagrangian(mgcg_lp* lp, const double* rho, const double* gL, double v_u,
                              double v_l, double theta_max_deg, double* out, double* alpha,
                              int mem) {
  NEED(lp);
  GUARD({
    const double cmax = std::cos(theta_max_deg * (M_PI / 180.0));
    const double a = lp->impl->lagrangian(rho, gL, v_u, v_l, cmax, out, mem);
    if (alpha) *alpha = a;
    return MGCG_OK;
  })
}

int mgcg_lp_select_top(mgcg_lp* lp, const double* v, int64_t k, double* out, int mem) {
  NEED(lp);
  GUARD({
    lp->impl->select_top(v, (long)k, out, mem);
    return MGCG_OK;
  })
}

int mgcg_threshold_round(mgcg_lp* lp, const double* rho, double lo, double hi, double* out,
                         int mem) {
  NEED(lp);
  GUARD({
    lp->impl->round_bounds(rho, lo, hi, out, mem);
    return MGCG_OK;
  })
}

int mgcg_angle_cos(mgcg_lp* lp, const double* gL, const double* d, double* cosine, int mem) {
  NEED(lp);
  NEED(cosine);
  GUARD({
    *cosine = lp->impl->angle_cos(gL, d, mem);
    return MGCG_OK;
  })
}

int mgcg_heaviside(mgcg_lp* lp, const double* rho, double beta, double* out, double* eta,
                   int32_t* iters, int mem) {
  NEED(lp);
  GUARD({
    int it = 0;
    const double e = lp->impl->heaviside(rho, beta, out, mem, &it);
    if (eta) *eta = e;
    if (iters) *iters = it;
    return MGCG_OK;
  })
}

int mgcg_slp_decide(mgcg_slp_ctrl* ctrl, double f0, double f1, double c0, double c1, double gts,
                    double ats, double s_inf, double* theta, double* a_red, double* p_red) {
  NEED(ctrl);
  return mgcg::slp_decide(ctrl, f0, f1, c0, c1, gts, ats, s_inf, theta, a_red, p_red);
}

}  // extern "C"

// ---- variables fixed before raising the degree
#include "fix.h"

extern "C" {

int mgcg_fix_variables(const mgcg_fix_desc* desc, const double* rho, const double* grad_x,
                       uint8_t* elem_kind, uint8_t* design_fixed, uint8_t* dof_mask,
                       mgcg_fix_counts* counts, int mem) {
  NEED(desc);
  GUARD({
    mgcg::fix_variables(*desc, rho, grad_x, elem_kind, design_fixed, dof_mask, counts, mem);
    return MGCG_OK;
  })
}

int mgcg_fix_variables_noalloc(const mgcg_fix_desc* desc, const double* rho, const double* grad_x,
                               uint8_t* elem_kind, uint8_t* design_fixed, uint8_t* dof_mask,
                               int64_t* counts_dev, void* stream) {
  NEED(desc);
  GUARD({
    mgcg::fix_variables_noalloc(*desc, rho, grad_x, elem_kind, design_fixed, dof_mask, counts_dev,
                                (hipStream_t)stream);
    return MGCG_OK;
  })
}

}  // extern "C"
