// Host runtime of the SLP step: the LP subproblem on the device and the step
// control of Algorithm 2 on the host.
#pragma once

#include "../../include/mgcg.h"
#include "common.h"

namespace mgcg {

class Lp {
 public:
  Lp(long n, int device);
  ~Lp();
  static size_t device_bytes(long n);
  void set_stream(hipStream_t s);
  // fixed (may be NULL): variables held at s = 0 (l = u = 0)
  void solve(const double* g, const double* a, const double* x, const unsigned char* fixed,
             double b, double delta, double xl, double xu, double* s, mgcg_lp_info* info,
             int mem);
  long size() const { return n_; }
  // thresholding of Sec. 5 on n values
  void select_top(const double* v, long k, double* out, int mem);
  void round_bounds(const double* r, double lo, double hi, double* out, int mem);
  double angle_cos(const double* gl, const double* d, int mem);
  double heaviside(const double* r, double beta, double* out, int mem, int* iters);
  double lagrangian(const double* rho, const double* gl, double vu, double vl, double cmax,
                    double* out, int mem);

 private:
  void stage_io(int mem, int nin, const double* const* in, const double** din, double* out,
                double** dout, void** stage);
  static double key_ratio_host(unsigned long long k);
  static void hist_shape(int nb, int* ch, int* nh);
  long n_;
  int device_;
  int nb_ = 0, nr_ = 0;  // blocks of LP_BS items; rows of the first bin reduction
  int ch_ = 1, nh_ = 0;  // chunks per block and blocks of the digit passes
  int ns_ = 0;           // blocks of the grid-stride sums
  size_t bytes_ = 0;
  hipStream_t stream_ = nullptr;  // the null stream unless set
  void* arena_ = nullptr;
  unsigned long long* key_ = nullptr;
  double *cap_ = nullptr, *part_ = nullptr, *bins_ = nullptr, *red_ = nullptr, *tsum_ = nullptr,
         *info_ = nullptr;
  void* st_ = nullptr;
  void* hst_ = nullptr;  // pinned host copy of the state and the info
};

int slp_decide(mgcg_slp_ctrl* c, double f0, double f1, double c0, double c1, double gts, double ats,
               double s_inf, double* theta, double* a_red, double* p_red);

}  // namespace mgcg
