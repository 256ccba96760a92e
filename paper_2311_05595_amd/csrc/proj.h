// Host runtime of the design-variable projection / density filter.
#pragma once

#include "../../include/mgcg.h"
#include "common.h"

namespace mgcg {

#include <vector>

// One stencil entry of a phase: the weight and the LDS offset of the design
// cell j + o relative to j in the staged tile.
struct ProjEntry {
  double w;
  int rel;
  int pad;
};

// Lattices, search extents and weight tables of one projection.
struct ProjGeom {
  int nr[3], nx[3];  // density and design lattices (x, y, z)
  int n, d;
  int kd, kr;        // candidate half-widths (design cells / density cells)
  int ntab;          // entries of the weight-factor table e(|m|)
  double R2;         // (2 n d rmin)^2
  long nrho, nxv;    // cells of each lattice
  std::vector<double> tab;  // e(|m|) = exp(-9 m^2 / (8 n^2 d^2 rmin^2))
  // tiled kernels (q > 0 when d divides n and the stencils reach at most 4
  // design cells): q^3 phase stencils, phase-major, and the halo h
  int q = 0, np = 0, h = 0;
  std::vector<ProjEntry> ent;
  std::vector<int> start;
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
  static void phase_tables(ProjGeom& g);
  void launch_norm();
  void release();
  ProjGeom g_;
  int device_;
  hipStream_t stream_ = nullptr;  // the null stream unless set
  double* invw_ = nullptr;  // 1 / omega_i per density cell
  double* tab_ = nullptr;   // e(|m|)
  ProjEntry* ent_ = nullptr;
  int* start_ = nullptr;
};

}  // namespace mgcg
