// Host runtime of the design-variable projection / density filter.
#pragma once

#include "../../include/mgcg.h"
#include "common.h"

namespace mgcg {

// Lattices and search extents of one projection.
struct ProjGeom {
  int nr[3], nx[3];  // density and design lattices (x, y, z)
  int n, d;
  int kd, kr;        // candidate half-widths (design cells / density cells)
  int ntab;          // entries of the weight-factor table e(|m|)
  double R2;         // (2 n d rmin)^2
  long nrho, nxv;    // cells of each lattice
};

class Proj {
 public:
  Proj(const mgcg_proj_desc& d, int device);
  ~Proj();
  // Validates the description (throws Error(MGCG_EINVAL) with the reason).
  static ProjGeom geometry(const mgcg_proj_desc& d);
  static size_t device_bytes(const mgcg_proj_desc& d);
  void set_stream(hipStream_t s);
  // rho = W x (transpose false) or gx = W^T g (transpose true).
  void run(bool transpose, const double* in, double* out, int mem);

 private:
  void launch_norm();
  void release();
  ProjGeom g_;
  int device_;
  hipStream_t stream_ = nullptr;  // the null stream unless set
  double* invw_ = nullptr;  // 1 / omega_i per density cell
  double* tab_ = nullptr;   // e(|m|)
};

}  // namespace mgcg
