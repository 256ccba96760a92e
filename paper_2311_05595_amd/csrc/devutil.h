// Device utilities: deterministic block/grid reductions.
#pragma once

#include <cstddef>

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
// so a few hundred partials cost one memory round trip.  In two parts, so
// that a kernel can pin values loaded before the sum's loads (their wait
// then comes after those loads are issued, and before the barrier that the
// compiler might otherwise sink their loads past).
__device__ __forceinline__ double block_sum_loads(const double* __restrict__ p, int n) {
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
  return s;
}
__device__ __forceinline__ double block_sum_finish(double s, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  s = wave_sum(s);
  if (lane == 0) sh[wid] = s;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < BS / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}
__device__ __forceinline__ double block_sum(const double* __restrict__ p, int n, double* sh) {
  return block_sum_finish(block_sum_loads(p, n), sh);
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

// The same for blocks of NT threads (a multiple of 64).
template <int NT>
__device__ __forceinline__ void block_partial2_nt(double a0, double a1, double* d0, double* d1) {
  __shared__ double sh2n[2][NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if (lane == 0) {
    sh2n[0][wid] = a0;
    sh2n[1][wid] = a1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      t0 += sh2n[0][w];
      t1 += sh2n[1][w];
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

// Keeps a value's computation (and its loads) above this point: without it
// the compiler may sink loads whose only use follows a gate test below that
// test, where they would wait for it.
__device__ __forceinline__ void pin(double& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(float& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void pin(int& v) { asm volatile("" : "+v"(v)); }

// Stand-in read by ungated launches (never written).
static __device__ CgScalars g_no_gate[4];

// The state word of load case r, read through the vector memory path:
// scalar loads complete out of order, so the kernel's first wait on any
// scalar value (a kernel argument, say) would wait for it too.
__device__ __forceinline__ int state_of(const CgScalars* cs, int r) {
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(cs, 4 * sizeof(CgScalars));
  return (int)__builtin_amdgcn_raw_buffer_load_b32(
      rs, r * (int)sizeof(CgScalars) + (int)offsetof(CgScalars, state), 0, 0);
}

// One field of load case r's CgScalars (at byte offset off), through the
// vector memory path like state_of.
__device__ __forceinline__ int cs_int(const CgScalars* cs, int r, int off) {
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(cs, 4 * sizeof(CgScalars));
  return (int)__builtin_amdgcn_raw_buffer_load_b32(rs, r * (int)sizeof(CgScalars) + off, 0, 0);
}
__device__ __forceinline__ double cs_dbl(const CgScalars* cs, int r, int off) {
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(cs, 4 * sizeof(CgScalars));
  return bload<double>(rs, r * (int)sizeof(CgScalars) + off, 0);
}
#define CS_OFF(field) ((int)offsetof(CgScalars, field))

// Gate of a kernel of the device-driven iteration.  gate_load() issues the
// loads of the four load cases' states (a problem always holds four
// CgScalars) with the kernel's first data loads; gate_open() is called only
// before the kernel's first store.  Testing first and returning early would
// put the state's memory latency in front of every other load of the
// kernel.  gate_open() pins the states, which keeps the test (and the wait
// for those loads) at its place in the program, after the loads above it.
struct Gate {
  int s[4];
  int nrhs, state;
  bool none;  // ungated launch: always open
};
__device__ __forceinline__ Gate gate_load(const CgScalars* cs, int nrhs, int state) {
  Gate g;
  g.none = cs == nullptr;
  const CgScalars* p = g.none ? g_no_gate : cs;
#pragma unroll
  for (int q = 0; q < 4; ++q) g.s[q] = state_of(p, q);
  g.nrhs = nrhs;
  g.state = state;
  return g;
}
// Open when any load case is in the gate's state; with r >= 0, when load
// case r is (epilogues that store per load case).
__device__ __forceinline__ bool gate_open(Gate g, int r = -1) {
#pragma unroll
  for (int q = 0; q < 4; ++q) pin(g.s[q]);
  if (g.none) return true;
  if (r >= 0) {
    const int sr = r == 0 ? g.s[0] : r == 1 ? g.s[1] : r == 2 ? g.s[2] : g.s[3];
    return sr == g.state;
  }
  return (g.s[0] == g.state) | ((g.nrhs > 1) & (g.s[1] == g.state)) |
         ((g.nrhs > 2) & (g.s[2] == g.state)) | ((g.nrhs > 3) & (g.s[3] == g.state));
}

// Linear node index i + nx (j + ny k) with 24-bit multiplies (every lattice
// dimension and plane index is far below 2^24).
__device__ __forceinline__ int lat_index(const Lat& L, int i, int j, int k) {
  return i + __mul24(L.nx, j + __mul24(L.ny, k));
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
