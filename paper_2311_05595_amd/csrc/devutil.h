// Device utilities: deterministic block/grid reductions.
#pragma once

#include "kernels.h"

namespace mgcg {

constexpr int BS = 256;  // threads per block of the node-parallel kernels

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Coherent (L1-bypassing) load of a value written by another workgroup of
// the same kernel.
__device__ __forceinline__ double load_coherent(const double* p) {
  unsigned long long b =
      __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)b);
}

// Sum nv per-thread values over the whole grid in a fixed order; the last
// block to finish calls fin(totals) from thread 0.  Every block of the grid
// must call this exactly once (blockDim.x == BS).
template <class Fin>
__device__ void grid_reduce(const double* acc, int nv, RedBuf red, int slot, const Fin& fin) {
  __shared__ double sh[MAX_RED_VALUES][BS / 64];
  __shared__ double tot[MAX_RED_VALUES];
  __shared__ int last;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < MAX_RED_VALUES; ++v) {
    if (v < nv) {
      double s = wave_sum(acc[v]);
      if (lane == 0) sh[v][wid] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 0; v < nv; ++v) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < BS / 64; ++w) s += sh[v][w];
      red.partials[(size_t)v * MAX_BLOCKS + blockIdx.x] = s;
    }
    __threadfence();
    unsigned t = atomicAdd(&red.counter[slot], 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  for (int v = 0; v < nv; ++v) {
    double s = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += BS)
      s += load_coherent(&red.partials[(size_t)v * MAX_BLOCKS + b]);
    s = wave_sum(s);
    if (lane == 0) sh[v][wid] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 0; v < nv; ++v) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < BS / 64; ++w) s += sh[v][w];
      tot[v] = s;
    }
    fin(tot);
    atomicExch(&red.counter[slot], 0u);
  }
}

// Grid reduction of two per-thread values for grids whose y index is the load
// case: tot[r] = sum over the blocks of row r of value 0, tot[nrhs + r] of
// value 1.  The last block calls fin(tot).
template <class Fin>
__device__ void grid_reduce_rhs(double a0, double a1, int nrhs, RedBuf red, int slot,
                                const Fin& fin) {
  __shared__ double sh[2][BS / 64];
  __shared__ double tot[2 * 4];
  __shared__ int last;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nbx = gridDim.x;
  const int bid = blockIdx.x + nbx * blockIdx.y;
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if (lane == 0) {
    sh[0][wid] = a0;
    sh[1][wid] = a1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) {
      s0 += sh[0][w];
      s1 += sh[1][w];
    }
    red.partials[bid] = s0;
    red.partials[MAX_BLOCKS + bid] = s1;
    __threadfence();
    unsigned t = atomicAdd(&red.counter[slot], 1u);
    last = (t == gridDim.x * gridDim.y - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  for (int v = 0; v < 2 * nrhs; ++v) {
    const int r = v % nrhs, which = v / nrhs;
    double s = 0.0;
    for (int b = threadIdx.x; b < nbx; b += BS)
      s += load_coherent(&red.partials[(size_t)which * MAX_BLOCKS + b + (size_t)nbx * r]);
    s = wave_sum(s);
    if (lane == 0) sh[0][wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < BS / 64; ++w) t += sh[0][w];
      tot[v] = t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    fin(tot);
    atomicExch(&red.counter[slot], 0u);
  }
}

__device__ __forceinline__ bool any_state(const CgScalars* cs, int nrhs, int state) {
  if (!cs) return true;
  for (int r = 0; r < nrhs; ++r)
    if (cs[r].state == state) return true;
  return false;
}

inline int nblocks(long n, int per = BS) { return (int)((n + per - 1) / per); }

// Grid for grid-stride vector kernels: bounded so that reductions fit the
// partials buffer; fixed for a given length (deterministic summation order).
inline int vec_grid(long n) {
  long b = (n + BS - 1) / BS;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (int)b;
}

}  // namespace mgcg
