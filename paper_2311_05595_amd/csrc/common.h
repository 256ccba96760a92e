// Internal definitions shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace mgcg {

// Thrown inside the library, caught at the C-ABI boundary.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MGCG_HIP(call)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::mgcg::Error(-5, std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

// Device buffers are read through 32-bit buffer offsets; an offset at or
// past this value marks "outside" (the load returns 0), so no buffer that a
// kernel addresses this way may reach it.
constexpr long kMaxBufferBytes = 0x7FFF0000;

// Operator kinds of a multigrid level.
enum OpKind : int {
  OP_MF_Q1 = 0,  // matrix-free trilinear elements: y = sum_e E_e K0 u_e (one density per element)
  OP_ST27 = 1,   // assembled 27-point stencil of 3x3 blocks (Q1-type lattice), symmetric half
  OP_EQ2 = 2,    // stored 81x81 element matrices of triquadratic elements
  OP_EQ3 = 3,    // stored 192x192 (serendipity: 96x96) element matrices of tricubic elements
};

// Number of stored stencil blocks per node: the diagonal block and the 13
// "forward" neighbour blocks (the other 13 are transposes of a neighbour's).
constexpr int ST_BLOCKS = 14;
constexpr int ST_COEF = ST_BLOCKS * 9;

// Forward neighbour offsets d (block A_{i,i+d}); entry 0 is the diagonal.
// Lexicographically positive offsets in (dz, dy, dx) order.
struct Off3 { int dx, dy, dz; };
__host__ __device__ constexpr Off3 st_offset(int b) {
  // b = 0: (0,0,0); b = 1..13 enumerate the positive half of {-1,0,1}^3
  // (dz > 0) or (dz == 0 && dy > 0) or (dz == 0 && dy == 0 && dx > 0).
  constexpr Off3 tab[ST_BLOCKS] = {
      {0, 0, 0},  {1, 0, 0},   {-1, 1, 0}, {0, 1, 0},  {1, 1, 0},  {-1, -1, 1}, {0, -1, 1},
      {1, -1, 1}, {-1, 0, 1},  {0, 0, 1},  {1, 0, 1},  {-1, 1, 1}, {0, 1, 1},   {1, 1, 1}};
  return tab[b];
}

// The same table for a run-time (wave-uniform) block index, decoded from two
// immediates instead of a table in memory: 6-bit codes (dx+1, dy+1, dz+1 as
// 2-bit fields), built from st_offset.
__host__ __device__ constexpr unsigned long long st_pack(int first, int count) {
  unsigned long long v = 0;
  for (int b = 0; b < count; ++b) {
    const Off3 d = st_offset(first + b);
    const unsigned long long code =
        (unsigned long long)((d.dx + 1) | ((d.dy + 1) << 2) | ((d.dz + 1) << 4));
    v |= code << (6 * b);
  }
  return v;
}

__host__ __device__ constexpr Off3 st_offset_rt(int b) {
  constexpr unsigned long long lo = st_pack(0, 10), hi = st_pack(10, ST_BLOCKS - 10);
  const unsigned code = b < 10 ? (unsigned)((lo >> (6 * b)) & 63ull)
                               : (unsigned)((hi >> (6 * (b - 10))) & 63ull);
  return Off3{(int)(code & 3) - 1, (int)((code >> 2) & 3) - 1, (int)((code >> 4) & 3) - 1};
}

constexpr bool st_tables_agree() {
  for (int b = 0; b < ST_BLOCKS; ++b) {
    const Off3 a = st_offset(b), r = st_offset_rt(b);
    if (a.dx != r.dx || a.dy != r.dy || a.dz != r.dz) return false;
  }
  return true;
}
static_assert(st_tables_agree(), "packed stencil offset table");

// Per load case CG scalars and state, resident on the device.
enum CgState : int { CG_ACTIVE = 0, CG_CHECK = 1, CG_DONE = 2, CG_BREAKDOWN = 3, CG_MAXIT = 4 };

struct CgScalars {
  double ff;      // ||f||^2
  double tol2;    // rtol^2 ||f||^2
  double rr;      // ||r||^2 (recurrence, or true after a check)
  double rzs[2];  // r^T z, double-buffered by iteration parity
  double alpha, beta;
  double pq;
  int iters;
  int state;
  int maxit;
  int replacements;
  int replace_every;
  int flexible;    // 1: Polak-Ribiere beta (non-symmetric FP32 preconditioner)
  double rr_best;  // smallest true ||r||^2 seen at a check
  int stall;       // consecutive checks without progress
  int bad;         // non-finite r^T z seen
  double rr_min;   // smallest recurrence ||r||^2 since the last true-residual check
  int since;       // iterations since rr_min last fell by 10 %
  int restart;     // 1: the next direction is z alone (beta = 0), after a replacement
};

}  // namespace mgcg
