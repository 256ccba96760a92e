// Device utilities: deterministic block/grid reductions.
#pragma once

#include "kernels.h"

namespace mgcg {

constexpr int BS = 256;  // threads per block of the node-parallel kernels

// ---- buffer loads: one VGPR byte offset shared by many loads, a scalar
// offset per load, and hardware bounds checks (an offset past the buffer
// returns 0).  Word 3 of the resource: raw (untyped) 32-bit dword access.
constexpr int kBufOOB = (int)kMaxBufferBytes;  // voffset marking "outside": loads return 0

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// Three consecutive values (a node's x, y, z) at byte offset voff.
template <typename T>
__device__ __forceinline__ void bload3(__amdgpu_buffer_rsrc_t r, int voff, T v[3]) {
  v[0] = bload<T>(r, voff, 0);
  v[1] = bload<T>(r, voff + (int)sizeof(T), 0);
  v[2] = bload<T>(r, voff + 2 * (int)sizeof(T), 0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Deterministic block-wide sum of p[0..n) (fixed order for a fixed n);
// every thread receives the result.  sh: BS/64 doubles of shared memory.
// Four independent buffer loads per thread and pass (reads past n return 0),
// so a few hundred partials cost one memory round trip.
__device__ __forceinline__ double block_sum(const double* __restrict__ p, int n, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const __amdgpu_buffer_rsrc_t rp = make_rsrc(p, (size_t)n * sizeof(double));
  double s = 0.0;
  for (int b = 0; b < n; b += 4 * BS) {
    const int o = (b + (int)threadIdx.x) * (int)sizeof(double);
    // (the whole offset in the vector operand: the range check covers it)
    const double v0 = bload<double>(rp, o, 0);
    const double v1 = bload<double>(rp, o + BS * 8, 0);
    const double v2 = bload<double>(rp, o + 2 * BS * 8, 0);
    const double v3 = bload<double>(rp, o + 3 * BS * 8, 0);
    s += (v0 + v1) + (v2 + v3);
  }
  s = wave_sum(s);
  if (lane == 0) sh[wid] = s;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < BS / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// Block sums of one / two per-thread values written to dst0 / dst1 by
// thread 0 (one partial per block; no atomics).
__device__ __forceinline__ void block_partial1(double a, double* dst) {
  __shared__ double sh1[BS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a = wave_sum(a);
  if (lane == 0) sh1[wid] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) t += sh1[w];
    *dst = t;
  }
  __syncthreads();
}

__device__ __forceinline__ void block_partial2(double a0, double a1, double* d0, double* d1) {
  __shared__ double sh2[2][BS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if (lane == 0) {
    sh2[0][wid] = a0;
    sh2[1][wid] = a1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) {
      t0 += sh2[0][w];
      t1 += sh2[1][w];
    }
    *d0 = t0;
    *d1 = t1;
  }
  __syncthreads();
}

__device__ __forceinline__ bool any_state(const CgScalars* cs, int nrhs, int state) {
  if (!cs) return true;
  for (int r = 0; r < nrhs; ++r)
    if (cs[r].state == state) return true;
  return false;
}

inline int nblocks(long n, int per = BS) { return (int)((n + per - 1) / per); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Remapping the linear workgroup id so that XCD x walks one contiguous
// range of tiles keeps the neighbour halos of consecutive tiles in the same
// L2 (a bijection of [0, gx*gy) for any grid size).  Returns the tile
// (bx, by) this workgroup handles.
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  constexpr int NX = 8;
  const int gx = gridDim.x, n = gx * gridDim.y;
  const int b = blockIdx.x + gx * blockIdx.y;
  const int x = b % NX, i = b / NX, per = n / NX, rem = n % NX;
  const int t = x * per + (x < rem ? x : rem) + i;
  bx = t % gx;
  by = t / gx;
}

// Vector kernels: each thread handles VU elements i0 + k BS (k < VU) per
// pass, loads first; the grid is at most 1024 blocks (four per CU), so the
// per-block partial sums stay few for the kernels that re-sum them, and a
// level-0 vector of up to 1M entries takes one pass.
constexpr int VU = 4;
inline int vec_grid(long n) {
  long b = (n + (long)BS * VU - 1) / ((long)BS * VU);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

}  // namespace mgcg
