// Host runtime of the design-variable projection / density filter.
#pragma once

#include "../../include/mgcg.h"
#include "common.h"

namespace mgcg {

#include <vector>

// One entry of a gather table of the tiled kernels: the LDS offset of a
// stencil offset in the staged tile and the weights of the G outputs a
// thread accumulates from it (zero where an output's stencil misses it).
// 16-byte aligned, so that the kernels load an entry as whole 16-byte words
// and a batch of entries as one run of wide scalar loads.
template <int G>
struct alignas(16) ProjEntryG {
  double w[G];
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
  // design cells): halo h, forward tables per group of gf phases (gf = 4 when
  // the q^3 phases split into fours, else 1), transpose tables per phase
  // (the mirrored stencils)
  int q = 0, np = 0, h = 0, gf = 0;
  std::vector<ProjEntryG<1>> fwd1;
  std::vector<ProjEntryG<4>> fwd4;
  std::vector<ProjEntryG<1>> trg;
  std::vector<int> start_f, start_t;
  size_t table_bytes() const {
    return fwd1.size() * sizeof(ProjEntryG<1>) + fwd4.size() * sizeof(ProjEntryG<4>) +
           trg.size() * sizeof(ProjEntryG<1>) +
           (start_f.size() + start_t.size()) * sizeof(int);
  }
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
  void* fwd_ent_ = nullptr;  // forward table (ProjEntryG<gf>)
  void* tr_ent_ = nullptr;   // transpose table (ProjEntryG<4>)
  int* start_f_ = nullptr;
  int* start_t_ = nullptr;
};

}  // namespace mgcg
