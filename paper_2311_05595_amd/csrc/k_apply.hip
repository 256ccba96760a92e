// Operator applies (node-centred gathers, no atomics), the CG recurrences
// and the V-cycle level kernels.
//
// Every apply computes, for one output node per thread, the three rows of
// A = Z K Z + (I - Z) (K assembled from element matrices, Sec. 3.3; Z keeps
// free DOFs) by gathering its neighbours — the element-by-element product of
// eq. (7) reorganised so that each output is written exactly once.  Fused
// epilogues turn the product into a residual, a weighted-Jacobi update
// (Algorithm 1, smoothing steps) or a CG step with its dot product.
#include <algorithm>
#include <type_traits>

#include <hip/hip_ext.h>

#include "devutil.h"

namespace mgcg {

// ------------------------------------------------------------------ inputs
template <typename T>
struct InPlain {
  const T* x;
  long ndof;
  __device__ __forceinline__ void load(int r, long node, T v[3]) const {
    const T* p = x + (size_t)r * ndof + 3 * node;
    v[0] = p[0];
    v[1] = p[1];
    v[2] = p[2];
  }
  // buffer view of load case r: load(voff) reads the node at byte offset voff
  struct Buf {
    __amdgpu_buffer_rsrc_t rx;
    __device__ __forceinline__ void load(int voff, T v[3]) const { bload3<T>(rx, voff, v); }
    // node (i, j, k), dz above or below the centre's plane, at byte offset
    // voff (kBufOOB: off the lattice, reads 0)
    __device__ __forceinline__ void load_node(int, int, int, int, int voff, T v[3]) const {
      bload3<T>(rx, voff, v);
    }
  };
  __device__ __forceinline__ Buf buf(int r) const {
    return Buf{make_rsrc(x + (size_t)r * ndof, ndof * sizeof(T))};
  }
};

// Trilinear prolongation of a coarse field at fine node (i, j, k): the sum of
// the 1, 2, 4 or 8 coarse nodes around it (a second corner per odd
// coordinate) times 1/2 per odd coordinate.  Unused corners, and every corner
// when !ok, read through out-of-range offsets (0), so there are no branches.
// Coarse values vanish on fixed coarse DOFs; the caller masks fixed fine ones.
template <typename T>
__device__ __forceinline__ void prolong_at(const Lat& C, __amdgpu_buffer_rsrc_t re, int i, int j,
                                           int k, bool ok, T pe[3]) {
  const int i0 = i >> 1, j0 = j >> 1, k0 = k >> 1;
  const bool oi = i & 1, oj = j & 1, ok_ = k & 1;
  const T w = (oi ? T(0.5) : T(1)) * (oj ? T(0.5) : T(1)) * (ok_ ? T(0.5) : T(1));
  T acc[3] = {T(0), T(0), T(0)};
  // the corner index is kept opaque: left to itself the compiler folds the
  // eight corners into full 32-bit multiplies (see lat_index)
  int base = lat_index(C, i0, j0, k0);
  asm volatile("" : "+v"(base));
  const int sy = C.nx, sz = C.nx * C.ny;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int a = q & 1, b = (q >> 1) & 1, cc = q >> 2;
    const bool use = ok && (!a || oi) && (!b || oj) && (!cc || ok_);
    const int off = use ? 3 * (base + a + b * sy + cc * sz) * (int)sizeof(T) : kBufOOB;
    T v[3];
    bload3<T>(re, off, v);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += v[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) pe[c] = w * acc[c];
}

__device__ __forceinline__ int bload_u8(__amdgpu_buffer_rsrc_t r, int voff) {
  return (int)__builtin_amdgcn_raw_buffer_load_b8(r, voff, 0, 0);
}


// ------------------------------------------------------------ operators
__device__ __forceinline__ void node_ijk(long node, const Lat& L, int& i, int& j, int& k) {
  // 32-bit divisions: node counts are bounded far below 2^32 by the buffer
  // offsets (see Problem::Problem)
  const unsigned n = (unsigned)node, nx = (unsigned)L.nx, ny = (unsigned)L.ny;
  const unsigned t = n / nx;
  i = (int)(n - t * nx);
  const unsigned kk = t / ny;
  j = (int)(t - kk * ny);
  k = (int)kk;
}

// The blocks b = part, part + LPN, ... of the stencil apply (partial sum of
// one node's rows).  `part` is wave-uniform, so every coefficient row offset
// is a scalar.  The loop has no branches: a block index past the table (and
// the transpose of the diagonal block) reads through out-of-range offsets,
// which return 0, so all of a wave's loads can be in flight together.
template <int LPN, typename T, class In>
__device__ __forceinline__ void ax_st_part(const OpST<T>& op, const In& in, int r, int i, int j,
                                           int k, long node, int part, T y[3]) {
  const Lat L = op.L;
  const long nn = L.nn();
  const auto xb = in.buf(r);
  const int row = (int)(nn * sizeof(T));
  const int vself = (int)(node * sizeof(T));
  T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < (ST_BLOCKS + LPN - 1) / LPN; ++q) {
    const int b0 = part + q * LPN;
    const bool valid = b0 < ST_BLOCKS;
    const int b = valid ? b0 : 0;
    const Off3 d = st_offset_rt(b);
    // the block's 9 coefficient rows (a resource per block keeps every
    // offset below 9 rows)
    const __amdgpu_buffer_rsrc_t rc =
        make_rsrc(op.coef + (size_t)b * 9 * nn, (size_t)9 * nn * sizeof(T));
    {
      const int ii = i + d.dx, jj = j + d.dy, kk = k + d.dz;
      const bool ok = valid && (unsigned)ii < (unsigned)L.nx && (unsigned)jj < (unsigned)L.ny &&
                      (unsigned)kk < (unsigned)L.nz;
      // 32-bit offsets (the host bounds every level vector below 2 GiB),
      // with 24-bit multiplies: a full 32-bit multiply-add is emitted as a
      // 64-bit one whose unused upper input half can alias a register with a
      // load in flight, and the wait for that load then stalls the gathers
      const int xo = ok ? lat_index(L, ii, jj, kk) * 3 * (int)sizeof(T) : kBufOOB;
      const int co = ok ? vself : kBufOOB;
      T v[3];
      xb.load_node(ii, jj, kk, d.dz, xo, v);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int e = 0; e < 3; ++e)
          acc[c] = fma(bload<T>(rc, co, (3 * c + e) * row), v[e], acc[c]);
    }
    {
      const int ii = i - d.dx, jj = j - d.dy, kk = k - d.dz;
      const bool ok = valid && b > 0 && (unsigned)ii < (unsigned)L.nx &&
                      (unsigned)jj < (unsigned)L.ny && (unsigned)kk < (unsigned)L.nz;
      const int nb = lat_index(L, ii, jj, kk);
      const int xo = ok ? nb * 3 * (int)sizeof(T) : kBufOOB;
      const int co = ok ? nb * (int)sizeof(T) : kBufOOB;
      T v[3];
      xb.load_node(ii, jj, kk, -d.dz, xo, v);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int e = 0; e < 3; ++e)
          acc[c] = fma(bload<T>(rc, co, (3 * e + c) * row), v[e], acc[c]);
    }
  }
  y[0] = acc[0];
  y[1] = acc[1];
  y[2] = acc[2];
}

// Second pass of the stored-matrix triquadratic apply: a node sums the rows
// of the element products K_e u_e (first pass) of the 1..8 elements that
// contain it; fixed rows return the input (identity rows).
template <typename T>
struct OpEQ2Y {
  Lat L;
  const T* Y;
  const uint8_t* mask;
};
template <typename T, class In>
__device__ __forceinline__ void ax_any(const OpEQ2Y<T>& op, const In& in, int r, long node, T y[3]) {
  const Lat L = op.L;
  int i, j, k;
  node_ijk(node, L, i, j, k);
  const int nex = (L.nx - 1) / 2, ney = (L.ny - 1) / 2, nez = (L.nz - 1) / 2;
  const long nel = (long)nex * ney * nez;
  int es[3][2], as[3][2], ne[3];
  const int p[3] = {i, j, k}, nmax[3] = {nex, ney, nez};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ne[d] = 0;
    if (p[d] & 1) {
      es[d][0] = (p[d] - 1) / 2;
      as[d][0] = 1;
      ne[d] = 1;
    } else {
      if (p[d] / 2 - 1 >= 0) { es[d][ne[d]] = p[d] / 2 - 1; as[d][ne[d]] = 2; ++ne[d]; }
      if (p[d] / 2 < nmax[d]) { es[d][ne[d]] = p[d] / 2; as[d][ne[d]] = 0; ++ne[d]; }
    }
  }
  T acc[3] = {T(0), T(0), T(0)};
  const T* Yr = op.Y + (size_t)r * nel * 81;
  for (int cz = 0; cz < ne[2]; ++cz)
    for (int cy = 0; cy < ne[1]; ++cy)
      for (int cx = 0; cx < ne[0]; ++cx) {
        const long e = es[0][cx] + (long)nex * (es[1][cy] + (long)ney * es[2][cz]);
        const int a = as[0][cx] + 3 * (as[1][cy] + 3 * as[2][cz]);
        const T* ye = Yr + e * 81 + 3 * a;
        acc[0] += ye[0];
        acc[1] += ye[1];
        acc[2] += ye[2];
      }
  const uint8_t m = op.mask[node];
  if (m) {
    T v[3];
    in.load(r, node, v);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if ((m >> c) & 1) acc[c] = v[c];
  }
  y[0] = acc[0];
  y[1] = acc[1];
  y[2] = acc[2];
}

// First pass: y_e = K_e u_e for every element and load case, one thread per
// (element, row), three elements per block.  K_e is symmetric and stored by
// wrapped diagonals, D[s][i] = K_e[i][(i + s) mod 81] for s = 0..40 (3321
// values, every entry once: half the bytes of the full matrix).  Row i is
// D[0][i], D[s][i] (column i + s) and D[s][i - s] (column i - s, by
// symmetry), s = 1..40, mod 81: at step s the 81 threads of an element read
// the 81 consecutive values D[s][*] once from memory (the rotated second
// read hits the same lines).  Each coefficient read serves every load case;
// u_e of every load case is staged in LDS.
constexpr int EQ_EPB = 3;  // elements per block (243 of 256 threads busy)
template <typename T, int NR, class In>
__global__ __launch_bounds__(BS) void k_eq2_elem(OpEQ2<T> op, In in, int nrhs,
                                                  const CgScalars* gate, int gate_state) {
  const Gate g = gate_load(gate, nrhs, gate_state);
  // the true-residual check's gate is usually closed: test it first there
  if (gate_state == CG_CHECK && !gate_open(g)) return;
  __shared__ T ue[NR][EQ_EPB][81];
  int bx, by;
  xcd_tile(bx, by);
  const Lat L = op.L;
  const int nex = (L.nx - 1) / 2, ney = (L.ny - 1) / 2, nez = (L.nz - 1) / 2;
  const long nel = (long)nex * ney * nez;
  const int le = threadIdx.x / 81, row = threadIdx.x - 81 * le;
  const long e = (long)bx * EQ_EPB + le;
  const bool on = le < EQ_EPB && e < nel;
  if (on) {
    const int ex = (int)(e % nex), ey = (int)((e / nex) % ney), ez = (int)(e / ((long)nex * ney));
    const int b = row / 3, comp = row - 3 * b;
    const int bxl = b % 3, byl = (b / 3) % 3, bzl = b / 9;
    const long node = (2 * ex + bxl) + (long)L.nx * ((2 * ey + byl) + (long)L.ny * (2 * ez + bzl));
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T v[3];
      in.load(r, node, v);
      ue[r][le][row] = v[comp];
    }
  }
  __syncthreads();
  if (!gate_open(g) || !on) return;
  const T* D = op.Ke + (size_t)e * Q2_PACKED;
  T acc[NR][2];
  const T d0 = D[row];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    acc[r][0] = d0 * ue[r][le][row];
    acc[r][1] = T(0);
  }
  // 5 batches of 8 diagonals, double-buffered: the 16 coefficient loads of
  // batch b + 1 are issued before the arithmetic of batch b
  T kb[2][16];
  auto issue = [&](int b, T (&k)[16]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sd = 1 + 8 * b + q;
      int jm = row - sd;
      jm += jm < 0 ? 81 : 0;
      k[2 * q] = D[sd * 81 + row];
      k[2 * q + 1] = D[sd * 81 + jm];
    }
  };
  issue(0, kb[0]);
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    if (b + 1 < 5) issue(b + 1, kb[(b + 1) & 1]);
    // (pinned: the wait covers this batch only, and the compiler does not
    // interleave the loads with the arithmetic)
#pragma unroll
    for (int q = 0; q < 16; ++q) pin(kb[b & 1][q]);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sd = 1 + 8 * b + q;
      int jp = row + sd, jm = row - sd;
      jp -= jp >= 81 ? 81 : 0;
      jm += jm < 0 ? 81 : 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        acc[r][0] = fma(kb[b & 1][2 * q], ue[r][le][jp], acc[r][0]);
        acc[r][1] = fma(kb[b & 1][2 * q + 1], ue[r][le][jm], acc[r][1]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) op.Y[((size_t)r * nel + e) * 81 + row] = acc[r][0] + acc[r][1];
  (void)by;
}

// First pass for serendipity elements: the same scheme over their 60 DOFs,
// four elements per block (240 of 256 threads busy).  Row i is D[0][i],
// D[s][i] and D[s][i - s] for s = 1..29, and D[30][i] once (columns i + 30
// and i - 30 coincide mod 60).  y_e is written at the DOFs of the 27-node
// layout; the 7 other nodes of each element are fixed, and the gather
// replaces their rows by the input.
constexpr int ES_EPB = 4;
template <typename T, int NR, class In>
__global__ __launch_bounds__(BS) void k_es2_elem(OpEQ2<T> op, In in, int nrhs,
                                                  const CgScalars* gate, int gate_state) {
  const Gate g = gate_load(gate, nrhs, gate_state);
  if (gate_state == CG_CHECK && !gate_open(g)) return;
  __shared__ T ue[NR][ES_EPB][60];
  int bx, by;
  xcd_tile(bx, by);
  const Lat L = op.L;
  const int nex = (L.nx - 1) / 2, ney = (L.ny - 1) / 2, nez = (L.nz - 1) / 2;
  const long nel = (long)nex * ney * nez;
  const int le = threadIdx.x / 60, row = threadIdx.x - 60 * le;
  const long e = (long)bx * ES_EPB + le;
  const bool on = le < ES_EPB && e < nel;
  const int b = on ? s2_node(row / 3) : 0, comp = row - 3 * (row / 3);
  if (on) {
    const int ex = (int)(e % nex), ey = (int)((e / nex) % ney), ez = (int)(e / ((long)nex * ney));
    const int bxl = b % 3, byl = (b / 3) % 3, bzl = b / 9;
    const long node = (2 * ex + bxl) + (long)L.nx * ((2 * ey + byl) + (long)L.ny * (2 * ez + bzl));
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T v[3];
      in.load(r, node, v);
      ue[r][le][row] = v[comp];
    }
  }
  __syncthreads();
  if (!gate_open(g) || !on) return;
  const T* D = op.Ke + (size_t)e * S2_PACKED;
  T acc[NR][2];
  const T d0 = D[row];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    acc[r][0] = d0 * ue[r][le][row];
    acc[r][1] = T(0);
  }
  // 4 batches of 8 diagonals (s = 1..32; 31 and 32 do not exist),
  // double-buffered like the 27-node pass
  T kb[2][16];
  auto issue = [&](int bt, T (&k)[16]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sd = 1 + 8 * bt + q;
      if (sd > 30) continue;
      int jm = row - sd;
      jm += jm < 0 ? 60 : 0;
      k[2 * q] = D[sd * 60 + row];
      if (sd < 30) k[2 * q + 1] = D[sd * 60 + jm];
    }
  };
  issue(0, kb[0]);
#pragma unroll
  for (int bt = 0; bt < 4; ++bt) {
    if (bt + 1 < 4) issue(bt + 1, kb[(bt + 1) & 1]);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sd = 1 + 8 * bt + q;
      if (sd > 30) continue;
      pin(kb[bt & 1][2 * q]);
      if (sd < 30) pin(kb[bt & 1][2 * q + 1]);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sd = 1 + 8 * bt + q;
      if (sd > 30) continue;
      int jp = row + sd, jm = row - sd;
      jp -= jp >= 60 ? 60 : 0;
      jm += jm < 0 ? 60 : 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        acc[r][0] = fma(kb[bt & 1][2 * q], ue[r][le][jp], acc[r][0]);
        if (sd < 30) acc[r][1] = fma(kb[bt & 1][2 * q + 1], ue[r][le][jm], acc[r][1]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    op.Y[((size_t)r * nel + e) * 81 + 3 * b + comp] = acc[r][0] + acc[r][1];
  (void)by;
}

// ------------------------------------------------------------ tricubic
// Second pass on the cubic lattice: a node sums the rows of the element
// products of the 1..8 elements that contain it (per axis: one element when
// the index is inside an edge, else the two that meet there); fixed rows
// return the input.  The serendipity element leaves the face- and
// body-interior nodes' products unwritten: those nodes are fixed.
template <typename T>
struct OpEQ3Y {
  Lat L;
  const T* Y;
  const uint8_t* mask;
};
template <typename T, class In>
__device__ __forceinline__ void ax_any(const OpEQ3Y<T>& op, const In& in, int r, long node, T y[3]) {
  const Lat L = op.L;
  int i, j, k;
  node_ijk(node, L, i, j, k);
  const int nex = (L.nx - 1) / 3, ney = (L.ny - 1) / 3, nez = (L.nz - 1) / 3;
  const long nel = (long)nex * ney * nez;
  int es[3][2], as[3][2], ne[3];
  const int p[3] = {i, j, k}, nmax[3] = {nex, ney, nez};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ne[d] = 0;
    const int q = p[d] / 3, m = p[d] - 3 * q;
    if (m) {
      es[d][0] = q;
      as[d][0] = m;
      ne[d] = 1;
    } else {
      if (q - 1 >= 0) { es[d][ne[d]] = q - 1; as[d][ne[d]] = 3; ++ne[d]; }
      if (q < nmax[d]) { es[d][ne[d]] = q; as[d][ne[d]] = 0; ++ne[d]; }
    }
  }
  T acc[3] = {T(0), T(0), T(0)};
  const T* Yr = op.Y + (size_t)r * nel * L3_ND;
  for (int cz = 0; cz < ne[2]; ++cz)
    for (int cy = 0; cy < ne[1]; ++cy)
      for (int cx = 0; cx < ne[0]; ++cx) {
        const long e = es[0][cx] + (long)nex * (es[1][cy] + (long)ney * es[2][cz]);
        const int a = as[0][cx] + 4 * (as[1][cy] + 4 * as[2][cz]);
        const T* ye = Yr + e * L3_ND + 3 * a;
        acc[0] += ye[0];
        acc[1] += ye[1];
        acc[2] += ye[2];
      }
  const uint8_t m = op.mask[node];
  if (m) {
    T v[3];
    in.load(r, node, v);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if ((m >> c) & 1) acc[c] = v[c];
  }
  y[0] = acc[0];
  y[1] = acc[1];
  y[2] = acc[2];
}

// First pass: y_e = K_e u_e, one thread per (element, row) over the N DOFs
// of the element (192 for the 64-node element, 96 for the 32-node
// serendipity one), E3_BS / N elements per block.  K_e by wrapped
// diagonals, D[s][i] = K_e[i][(i + s) mod N] for s = 0..N/2: row i is
// D[0][i] u_i + sum_{s=1}^{N/2-1} (D[s][i] u_{i+s} + D[s][i-s] u_{i-s})
// + D[N/2][i] u_{i+N/2} (columns i + N/2 and i - N/2 coincide).  At step s
// an element's N threads read the N consecutive values D[s][*] once (the
// rotated second read hits the same lines); each value serves every load
// case, whose u_e are staged in LDS.  Batches of 8 diagonals, the loads of
// batch b + 1 issued before the arithmetic of batch b.
constexpr int E3_BS = 192;
template <typename T, int NR, class In, int N>
__global__ __launch_bounds__(E3_BS) void k_e3_elem(OpEQ2<T> op, In in, int nrhs,
                                                    const CgScalars* gate, int gate_state) {
  constexpr int EPB = E3_BS / N, H = N / 2, PK = (H + 1) * N, NBT = H / 8;
  static_assert(EPB * N == E3_BS && NBT * 8 == H, "tile shape");
  const Gate g = gate_load(gate, nrhs, gate_state);
  if (gate_state == CG_CHECK && !gate_open(g)) return;
  __shared__ T ue[NR][EPB][N];
  int bx, by;
  xcd_tile(bx, by);
  const Lat L = op.L;
  const int nex = (L.nx - 1) / 3, ney = (L.ny - 1) / 3, nez = (L.nz - 1) / 3;
  const long nel = (long)nex * ney * nez;
  const int le = threadIdx.x / N, row = threadIdx.x - N * le;
  const long e = (long)bx * EPB + le;
  const bool on = e < nel;
  const int a = N == L3_ND ? row / 3 : s3_node(row / 3), comp = row - 3 * (row / 3);
  if (on) {
    const int ex = (int)(e % nex), ey = (int)((e / nex) % ney), ez = (int)(e / ((long)nex * ney));
    const int ax = a % 4, ay = (a / 4) % 4, az = a / 16;
    const long node = (3 * ex + ax) + (long)L.nx * ((3 * ey + ay) + (long)L.ny * (3 * ez + az));
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T v[3];
      in.load(r, node, v);
      ue[r][le][row] = v[comp];
    }
  }
  __syncthreads();
  if (!gate_open(g) || !on) return;
  const T* D = op.Ke + (size_t)e * PK;
  T acc[NR][2];
  const T d0 = D[row];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    acc[r][0] = d0 * ue[r][le][row];
    acc[r][1] = T(0);
  }
  T kb[2][16];
  auto issue = [&](int b, T (&k)[16]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sd = 1 + 8 * b + q;
      int jm = row - sd;
      jm += jm < 0 ? N : 0;
      k[2 * q] = D[sd * N + row];
      k[2 * q + 1] = sd < H ? D[sd * N + jm] : T(0);
    }
  };
  issue(0, kb[0]);
#pragma unroll
  for (int b = 0; b < NBT; ++b) {
    if (b + 1 < NBT) issue(b + 1, kb[(b + 1) & 1]);
#pragma unroll
    for (int q = 0; q < 16; ++q) pin(kb[b & 1][q]);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sd = 1 + 8 * b + q;
      int jp = row + sd, jm = row - sd;
      jp -= jp >= N ? N : 0;
      jm += jm < 0 ? N : 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        acc[r][0] = fma(kb[b & 1][2 * q], ue[r][le][jp], acc[r][0]);
        if (sd < H) acc[r][1] = fma(kb[b & 1][2 * q + 1], ue[r][le][jm], acc[r][1]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
    op.Y[((size_t)r * nel + e) * L3_ND + 3 * a + comp] = acc[r][0] + acc[r][1];
  (void)by;
}

// ------------------------------------------------------------ epilogues
// pre(r, node) loads the epilogue's operands and is called before the
// operator's gathers, so that those loads travel with them; put() then only
// computes and stores.  (Loading them after the output store would also force
// one round trip per value: the output may alias them.)
template <typename T>
struct Pre3 {
  T v[3];
};
template <typename T>
__device__ __forceinline__ Pre3<T> ld3(const T* p) {
  return Pre3<T>{{p[0], p[1], p[2]}};
}

// Writes the V-cycle input for residual value rn of DOF i (offset oi of its
// load case); wd is W D^-1 at DOF i in the V-cycle precision.
__device__ __forceinline__ void vprep_put(const VPrep& vp, size_t oi, double rn, double wd) {
  if (vp.f32) {
    const float b = (float)rn;
    ((float*)vp.b0)[oi] = b;
    ((float*)vp.x0)[oi] = (float)wd * b;
  } else {
    ((double*)vp.x0)[oi] = wd * rn;
  }
}
__device__ __forceinline__ double vprep_wd(const VPrep& vp, size_t i) {
  return vp.f32 ? (double)((const float*)vp.wD)[i] : ((const double*)vp.wD)[i];
}

template <typename T>
struct EpStore {
  T* y;
  long ndof;
  static constexpr bool RED = false;
  struct Pre {};
  __device__ Pre pre(int, long) const { return Pre{}; }
  __device__ void put(int r, long node, const T ax[3], const Pre&, double&, double&) const {
    T* p = y + (size_t)r * ndof + 3 * node;
    p[0] = ax[0];
    p[1] = ax[1];
    p[2] = ax[2];
  }
};

template <typename T>
struct EpResid {  // r = b - A x
  const T* b;
  T* rout;
  long ndof;
  static constexpr bool RED = false;
  struct Pre {
    Pre3<T> b;
  };
  __device__ Pre pre(int r, long node) const { return Pre{ld3(b + (size_t)r * ndof + 3 * node)}; }
  __device__ void put(int r, long node, const T ax[3], const Pre& pv, double&, double&) const {
    const size_t o = (size_t)r * ndof + 3 * node;
#pragma unroll
    for (int c = 0; c < 3; ++c) rout[o + c] = pv.b.v[c] - ax[c];
  }
};

template <typename T>
struct EpJacobi {  // xo = x + wD (b - A x)  (weights folded into wD)
  const T* b;
  const T* x;
  const T* invD;
  T omega;
  T* xo;
  long ndof;
  static constexpr bool RED = false;
  struct Pre {
    Pre3<T> b, x, d;
  };
  __device__ Pre pre(int r, long node) const {
    const size_t o = (size_t)r * ndof + 3 * node;
    return Pre{ld3(b + o), ld3(x + o), ld3(invD + 3 * node)};
  }
  __device__ void put(int r, long node, const T ax[3], const Pre& pv, double&, double&) const {
    const size_t o = (size_t)r * ndof + 3 * node;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      xo[o + c] = pv.x.v[c] + omega * pv.d.v[c] * (pv.b.v[c] - ax[c]);
  }
};

// The last finest-level sweep of the V-cycle: its output is z, so the CG dot
// products r.z and, for the flexible beta of the FP32 V-cycle, q.z (with
// r - r_old = -alpha q) are accumulated here (partials per block).
template <typename T>
struct EpJacobiDot {
  const T* b;
  const T* x;
  const T* invD;
  T omega;
  T* xo;
  long ndof;
  const double* r;
  const double* q;  // the CG's A p (FP32 V-cycle only: the flexible beta)
  static constexpr bool RED = true;
  struct Pre {
    Pre3<T> b, x, d;
    Pre3<double> r, q;
  };
  __device__ Pre pre(int rr, long node) const {
    const size_t o = (size_t)rr * ndof + 3 * node;
    Pre pv{ld3(b + o), ld3(x + o), ld3(invD + 3 * node), ld3(r + o), {}};
    if constexpr (sizeof(T) == 4) pv.q = ld3(q + o);
    return pv;
  }
  __device__ void put(int rr, long node, const T ax[3], const Pre& pv, double& a0,
                      double& a1) const {
    const size_t o = (size_t)rr * ndof + 3 * node;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T z = pv.x.v[c] + omega * pv.d.v[c] * (pv.b.v[c] - ax[c]);
      xo[o + c] = z;
      a0 += pv.r.v[c] * (double)z;
      if constexpr (sizeof(T) == 4) a1 += pv.q.v[c] * (double)z;
    }
  }
};

struct EpDotPQ {  // q = A p; acc[r] += p.q  (active load cases)
  const double* p;
  double* q;
  long ndof;
  static constexpr bool RED = true;
  struct Pre {
    Pre3<double> p;
  };
  __device__ Pre pre(int r, long node) const { return Pre{ld3(p + (size_t)r * ndof + 3 * node)}; }
  __device__ void put(int r, long node, const double ax[3], const Pre& pv, double& a0,
                      double&) const {
    const size_t o = (size_t)r * ndof + 3 * node;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q[o + c] = ax[c];
      a0 += pv.p.v[c] * ax[c];
    }
  }
};

struct EpInitResid {  // r = f - A x; acc[r] += r.r; acc[nrhs + r] += f.f
  const double* f;
  double* rout;
  long ndof;
  int nrhs;
  static constexpr bool RED = true;
  struct Pre {
    Pre3<double> f;
  };
  __device__ Pre pre(int r, long node) const { return Pre{ld3(f + (size_t)r * ndof + 3 * node)}; }
  __device__ void put(int r, long node, const double ax[3], const Pre& pv, double& a0,
                      double& a1) const {
    const size_t o = (size_t)r * ndof + 3 * node;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double rr = pv.f.v[c] - ax[c];
      rout[o + c] = rr;
      a0 += rr * rr;
      a1 += pv.f.v[c] * pv.f.v[c];
    }
  }
};

struct EpTrueResid {  // for load cases under check: r = f - A x; acc[r] += r.r
  const double* f;
  double* rout;
  long ndof;
  VPrep vp;  // the replaced residual is the next V-cycle's input
  static constexpr bool RED = true;
  struct Pre {
    Pre3<double> f;
    double wd[3];
  };
  __device__ Pre pre(int r, long node) const {
    Pre pv{ld3(f + (size_t)r * ndof + 3 * node), {0.0, 0.0, 0.0}};
    if (vp.x0)
      for (int c = 0; c < 3; ++c) pv.wd[c] = vprep_wd(vp, 3 * node + c);
    return pv;
  }
  __device__ void put(int r, long node, const double ax[3], const Pre& pv, double& a0,
                      double&) const {
    const size_t o = (size_t)r * ndof + 3 * node;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double rr = pv.f.v[c] - ax[c];
      rout[o + c] = rr;
      a0 += rr * rr;
      if (vp.x0) vprep_put(vp, o + c, rr, pv.wd[c]);
    }
  }
};

// Epilogues of kernels that usually find their gate closed (a true-residual
// check runs on few iterations) test it first and return at once; every
// other kernel tests it just before its first store.
template <class Ep> struct GateEarly { static constexpr bool v = false; };
template <> struct GateEarly<EpTrueResid> { static constexpr bool v = true; };
// Epilogues that store only for the load cases in the gate's state (the
// others store for every load case while any is).
template <class Ep> struct PerRhs { static constexpr bool v = false; };
template <> struct PerRhs<EpDotPQ> { static constexpr bool v = true; };
template <> struct PerRhs<EpTrueResid> { static constexpr bool v = true; };

// ------------------------------------------------------------ apply kernel
// One output node per thread, one load case per grid row (blockIdx.y).
// Register budgets: the matrix-free kernel keeps the 27-node neighbourhood in
// registers (2 waves per SIMD); the stored-operator kernels stream their
// coefficients (4 waves per SIMD).  Reducing epilogues write one partial sum
// per block (value a0 at row r, a1 at row 4 + r of the region); the
// consumers sum them in a fixed order (no atomics).
template <class Op> struct Waves { static constexpr int w = 4; };

template <typename T, class Op, class In, class Ep>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(Waves<Op>::w)))
void k_apply(Op op, In in, Ep ep, int nrhs, const CgScalars* gate, int gate_state, double* part) {
  int bx, r;
  xcd_tile(bx, r);
  const Gate g = gate_load(gate, nrhs, gate_state);
  const int gr = PerRhs<Ep>::v ? r : -1;
  if constexpr (GateEarly<Ep>::v) {
    if (!gate_open(g, gr)) return;
  }
  const long node = (long)bx * BS + threadIdx.x;
  const long nn = op.L.nn();
  const long nodec = node < nn ? node : nn - 1;  // tail threads compute a copy, store nothing
  double a0 = 0.0, a1 = 0.0;
  const typename Ep::Pre pv = ep.pre(r, nodec);
  T ax[3];
  ax_any(op, in, r, nodec, ax);
  // the gathers complete before the gate test (kept from sinking into it)
  asm volatile("" : "+v"(ax[0]), "+v"(ax[1]), "+v"(ax[2]));
  if (!gate_open(g, gr)) return;
  if (node < nn) ep.put(r, node, ax, pv, a0, a1);
  if constexpr (Ep::RED) {
    block_partial2(a0, a1, part + (size_t)r * MAX_BLOCKS + bx,
                   part + (size_t)(4 + r) * MAX_BLOCKS + bx);
  }
}

// Matrix-free trilinear apply by independent wave tiles (no LDS, no block
// barrier until the final partial sums).  A wave takes an 8 x 8 tile of
// element columns, lane (li, lj) = (lane & 7, lane >> 3) the column with
// lower corner node (WT_OWN tx - 1 + li, WT_OWN ty - 1 + lj), and marches
// through the element layers of a chunk of node planes:
//  * each lane loads the top face of its element (4 nodes x 3 components,
//    one layer ahead) and takes its 2-D Haar transform; the bottom face's
//    transform is kept from the previous layer;
//  * the element product in the Haar basis gives its corner values
//    (haar_element);
//  * node (i, j) of a face sums the corners of elements (i, j), (i - 1, j),
//    (i, j - 1), (i - 1, j - 1): a shift by one lane in x (DPP within rows of
//    16 lanes) and one by eight lanes in y (a lane permute) bring them to the
//    lane of element (i, j), which owns that node when li, lj >= 1 (7 x 7
//    nodes per tile);
//  * a layer's bottom corners finish node plane L (the epilogue stores it),
//    its top corners start plane L + 1.
// Elements off the mesh read modulus 0 (their products vanish; node values
// off the lattice only meet such elements).  Inputs vanish on fixed DOFs;
// fixed rows return 0.  Any lattice size; the chunk height kz sets the
// number of waves.
// One element in its tensor Haar basis (q1table.h: K0 u = T K_h T^T u, 45
// nonzeros in K_h instead of 576 in K0): bottom face fb and top face ft as
// 2-D Haar modes f[comp][q], q = mx + 2 my, modulus E ->
// corner values of the bottom face gb[comp][corner] and top face gt, corner
// = ax + 2 ay.
template <typename T>
__device__ __forceinline__ void haar_element(const Q1HaarVals<T>& hv, const T (&fb)[3][4],
                                           const T (&ft)[3][4], T E, T gb[3][4], T gt[3][4]) {
  // mode coefficients c[3 m + comp], m = q + 4 mz (the constant mode m = 0
  // is never used)
  T cm[24];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cm[3 * q + k] = fb[k][q] + ft[k][q];
      cm[3 * (q + 4) + k] = ft[k][q] - fb[k][q];
    }
  T y[24];
#pragma unroll
  for (int i = 0; i < 24; ++i) {
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int j = 0; j < 24; ++j) {
      const int cl = kQ1H.cls[i * 24 + j];
      if (cl < 0) continue;
      const T h = kQ1H.sgn[i * 24 + j] > 0 ? hv.v[cl] : -hv.v[cl];
      acc = first ? h * cm[j] : fma(h, cm[j], acc);
      first = false;
    }
    y[i] = first ? T(0) : E * acc;
  }
  // inverse z (node 0: s - d, node 1: s + d), then the inverse 2-D transform
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T b[4], t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      b[q] = y[3 * q + k] - y[3 * (q + 4) + k];
      t[q] = y[3 * q + k] + y[3 * (q + 4) + k];
    }
    {
      const T p = b[0] - b[2], r = b[1] - b[3], u = b[0] + b[2], v = b[1] + b[3];
      gb[k][0] = p - r;
      gb[k][1] = p + r;
      gb[k][2] = u - v;
      gb[k][3] = u + v;
    }
    {
      const T p = t[0] - t[2], r = t[1] - t[3], u = t[0] + t[2], v = t[1] + t[3];
      gt[k][0] = p - r;
      gt[k][1] = p + r;
      gt[k][2] = u - v;
      gt[k][3] = u + v;
    }
  }
}

constexpr int WT_OWN = 7;  // owned nodes per tile and direction
constexpr int WT_WAVES = 4;  // independent waves per block

__device__ __forceinline__ int wt_shx32(int v) {  // lane - 1 within rows of 16 (row start: 0)
  return __builtin_amdgcn_mov_dpp(v, 0x111, 0xf, 0xf, true);
}
__device__ __forceinline__ double wt_shx(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = wt_shx32((int)b), hi = wt_shx32((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float wt_shx(float v) {
  return __builtin_bit_cast(float, wt_shx32(__builtin_bit_cast(int, v)));
}
// value of lane - 8 (lanes 0 .. 7: their own); addr = 4 max(lane - 8, 0)
__device__ __forceinline__ double wt_shy(double v, int addr) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)b);
  const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ float wt_shy(float v, int addr) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}

// Resident waves per SIMD the kernel is built for (FP64 / FP32 register
// budgets: 168 / 128 VGPRs).
#ifndef WT_WPE64
#define WT_WPE64 2
#endif
template <typename T>
struct WtShape {
  static constexpr int wpe = sizeof(T) == 8 ? WT_WPE64 : 4;
};
struct WtGrid {
  int ntx, nty, kz, nzc;
  long waves() const { return (long)ntx * nty * nzc; }
  int blocks() const { return (int)((waves() + WT_WAVES - 1) / WT_WAVES); }
};
// Chunk height: a wave of a chunk of kz planes computes kz + 1 element
// layers, and the chip holds 1024 wpe waves at once; the height that
// minimises (rounds of resident waves) x (layers per wave) plus a prologue
// of about half a layer, within the reduction buffer's block count.
inline WtGrid wt_grid(const Lat& L, bool fp64) {
  WtGrid g;
  g.ntx = (L.nx + WT_OWN - 1) / WT_OWN;
  g.nty = (L.ny + WT_OWN - 1) / WT_OWN;
  const long tiles = (long)g.ntx * g.nty;
  const long slots = 1024L * (fp64 ? WtShape<double>::wpe : WtShape<float>::wpe);
  double best = 0.0;
  g.kz = 0;
  for (int kz = 1; kz <= 32; ++kz) {
    const long nzc = (L.nz + kz - 1) / kz, waves = tiles * nzc;
    if ((waves + WT_WAVES - 1) / WT_WAVES > MAX_BLOCKS) continue;
    const double cost = (double)((waves + slots - 1) / slots) * (kz + 1.5);
    if (g.kz == 0 || cost < best) {
      best = cost;
      g.kz = kz;
    }
  }
  if (g.kz == 0) g.kz = 32;  // (the launch rejects a grid past the buffer)
  g.nzc = (L.nz + g.kz - 1) / g.kz;
  return g;
}

template <typename T, class Ep>
__global__ __launch_bounds__(64 * WT_WAVES)
__attribute__((amdgpu_waves_per_eu(WtShape<T>::wpe, WtShape<T>::wpe)))
void k_apply_mf_wt(OpMF<T> op, InPlain<T> in, Ep ep, int nrhs, const CgScalars* gate,
                   int gate_state, double* part, int ntx, int nty, int kz, int nwaves) {
  int bx, r;
  xcd_tile(bx, r);
  const Gate g = gate_load(gate, nrhs, gate_state);
  const int gr = PerRhs<Ep>::v ? r : -1;
  if constexpr (GateEarly<Ep>::v) {
    if (!gate_open(g, gr)) return;
  }
  const int lane = threadIdx.x & 63;
  // wave-uniform tile coordinates (scalar arithmetic)
  const int wv = bx * WT_WAVES + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  double a0 = 0.0, a1 = 0.0;
  if (wv < nwaves) {
    const Lat L = op.L;
    const int nx = L.nx, ny = L.ny, nz = L.nz, P = nx * ny;
    const int ex1 = nx - 1, ey1 = ny - 1, ez1 = nz - 1;
    const int tx = wv % ntx, ty = (wv / ntx) % nty, zc = wv / (ntx * nty);
    const int li = lane & 7, lj = lane >> 3;
    const int i = WT_OWN * tx - 1 + li, j = WT_OWN * ty - 1 + lj;
    const int yaddr = 4 * max(lane - 8, 0);
    const int k0 = zc * kz, k1 = min(nz, k0 + kz);
    const int nsteps = k1 - k0 + 1;  // element layers k0 - 1 .. k1 - 1
    const bool owner = li >= 1 && lj >= 1 && i < nx && j < ny;
    const int nodec = owner ? i + nx * j : 0;  // plane index of the owned node
    const __amdgpu_buffer_rsrc_t rx =
        make_rsrc(in.x + (size_t)r * in.ndof, (size_t)in.ndof * sizeof(T));
    const __amdgpu_buffer_rsrc_t re = make_rsrc(op.E, (size_t)ex1 * ey1 * ez1 * sizeof(T));
    const bool eon = i >= 0 && i < ex1 && j >= 0 && j < ey1;
    // byte offsets of node (i, j) and (i, j + 1) in plane 0 (negative, or
    // past the end of the vector: the loads read 0)
    constexpr int SZ = (int)sizeof(T);
    const int xo0 = 3 * (i + nx * j) * SZ, xo1 = xo0 + 3 * nx * SZ;
    const int planeb = 3 * P * SZ;
    const unsigned eo = eon ? (unsigned)((i + ex1 * j) * SZ) : (unsigned)kBufOOB;
    const int lstrideb = ex1 * ey1 * SZ;
    // top face of layer L (node plane L + 1).  Planes off the lattice (the
    // layers below plane 0 and above the last) are replaced by a plane on
    // it: those layers' elements have modulus 0.
    auto load_face = [&](int k, T (&v)[12]) {
      const int ko = min(max(k, 0), nz - 1) * planeb;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        v[c] = bload<T>(rx, xo0 + ko + c * SZ, 0);
        v[6 + c] = bload<T>(rx, xo1 + ko + c * SZ, 0);
      }
    };
    auto load_E = [&](int layer) {
      const bool on = layer >= 0 && layer < ez1;  // uniform
      // (an element off the mesh: an offset at or past kBufOOB, read as 0)
      const T e = bload<T>(re, (int)(eo + (unsigned)(min(max(layer, 0), ez1 - 1) * lstrideb)), 0);
      return on ? e : T(0);
    };
    // 2-D Haar transform of a face from its 4 nodes (q = mx + 2 my)
    auto face = [&](const T (&v)[12], T (&f)[3][4]) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T u00 = v[c], u10 = v[3 + c], u01 = v[6 + c], u11 = v[9 + c];
        const T a = u00 + u10, b = u10 - u00, cc = u01 + u11, d = u11 - u01;
        f[c][0] = a + cc;
        f[c][1] = b + d;
        f[c][2] = cc - a;
        f[c][3] = d - b;
      }
    };
    // node value of this lane's node from the four elements' corners
    auto gather = [&](const T (&gc)[3][4], T (&out)[3]) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T A = gc[c][0] + wt_shx(gc[c][1]);
        const T B = gc[c][2] + wt_shx(gc[c][3]);
        out[c] = A + wt_shy(B, yaddr);
      }
    };
    // one face in flight: a layer transforms its top face, then loads the
    // next layer's (used one layer later); two face transforms (bottom and
    // top swap roles every layer) and two moduli
    T v[12];
    T Ev[2];
    T f[2][3][4];
    load_face(k0 - 1, v);
    face(v, f[1]);
    load_face(k0, v);
    Ev[0] = load_E(k0 - 1);
    typename Ep::Pre pv = ep.pre(r, (long)min(k0, nz - 1) * P + nodec);
    uint8_t mk = op.mask[(size_t)min(k0, nz - 1) * P + nodec];
    T acc[3] = {T(0), T(0), T(0)};
    // layer k0 - 1 + s (q = s & 1): bottom transform in f[q ^ 1], its top
    // face's transform to f[q], modulus in Ev[q]
    auto step = [&](int s, int q) {
      face(v, f[q]);
      // (unconditional: past the last layer the clamped plane is read and
      // never used, so every step issues the same loads)
      load_face(k0 + s + 1, v);
      Ev[q ^ 1] = load_E(k0 + s);
      T gb[3][4], gt[3][4];
      haar_element<T>(op.hv, f[q ^ 1], f[q], Ev[q], gb, gt);
      T bot[3], top[3];
      gather(gb, bot);
      gather(gt, top);
      if (s >= 1) {  // node plane k0 - 1 + s is complete
        const int kp = k0 - 1 + s;
        T ax[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) ax[c] = ((mk >> c) & 1) ? T(0) : acc[c] + bot[c];
        if (owner) ep.put(r, (long)kp * P + nodec, ax, pv, a0, a1);
        const int kn = min(kp + 1, nz - 1);  // (past the chunk: read, unused)
        pv = ep.pre(r, (long)kn * P + nodec);
        mk = op.mask[(size_t)kn * P + nodec];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] = top[c];
    };
    if (!gate_open(g, gr)) return;  // uniform over the block
    for (int s = 0; s < nsteps; s += 2) {
      step(s, 0);
      if (s + 1 < nsteps) step(s + 1, 1);
    }
  } else {
    if (!gate_open(g, gr)) return;  // uniform over the block
  }
  if constexpr (Ep::RED) {
    block_partial2_nt<64 * WT_WAVES>(a0, a1, part + (size_t)r * MAX_BLOCKS + bx,
                                     part + (size_t)(4 + r) * MAX_BLOCKS + bx);
  }
}

// Stencil operators: the LPN waves of a block share 64 consecutive nodes,
// wave w summing the stencil blocks w, w + LPN, ... (coalesced loads, part of
// the load chain per lane, LPN x the waves of one-thread-per-node); the
// partial rows meet in LDS and wave 0 runs the epilogue.  Two shapes:
// 7 waves (two blocks each, 4 waves per SIMD) and 4 waves (3-4 blocks each,
// 2 waves per SIMD with up to 256 registers).  Measured: 7 waves win on
// FP32 levels and on small FP64 levels (+2 % on the 96x48x48 cantilever,
// latency-bound), 4 waves on large FP64 levels (+5 % on the 64x32x32 n = 4
// cantilever in FP64, +8 % on the FP64 served mix).
constexpr int ST_NODES = 64;  // nodes per block
constexpr long ST_BIG_FP64_NODES = 65536;
template <int LPN>
struct StShape {
  static constexpr int threads = LPN * ST_NODES;
  static constexpr int waves_per_eu = LPN == 7 ? 4 : 2;
};
template <typename T>
inline int st_lpn(long nn) { return (sizeof(T) == 8 && nn > ST_BIG_FP64_NODES) ? 4 : 7; }

template <typename T, class In, class Ep, int LPN>
__global__ __launch_bounds__(StShape<LPN>::threads)
__attribute__((amdgpu_waves_per_eu(StShape<LPN>::waves_per_eu, StShape<LPN>::waves_per_eu)))
void k_apply_st(OpST<T> op, In in, Ep ep, int nrhs,
                                                 const CgScalars* gate, int gate_state,
                                                 double* part) {
  constexpr int ST_LPN = LPN;
  __shared__ T red[ST_LPN - 1][3][ST_NODES];
  // the wave index must be provably uniform: it selects the coefficient
  // rows through the scalar offset of every buffer load (a divergent value
  // there turns each load into a serialised readfirstlane loop)
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / ST_NODES);
  const int lane = threadIdx.x % ST_NODES;
  int bx, r;
  xcd_tile(bx, r);
  const Gate g = gate_load(gate, nrhs, gate_state);
  const int gr = PerRhs<Ep>::v ? r : -1;
  if constexpr (GateEarly<Ep>::v) {
    if (!gate_open(g, gr)) return;
  }
  const long node = (long)bx * ST_NODES + lane;
  double a0 = 0.0, a1 = 0.0;
  const bool on = node < op.L.nn();
  T ax[3] = {T(0), T(0), T(0)};
  // epilogue operands, loaded by wave 0 only (which runs the epilogue) under
  // a wave-uniform branch, before its gathers; for the other six waves they
  // would be redundant loads
  const long nn = op.L.nn();
  typename Ep::Pre pv{};
  if (wave == 0) pv = ep.pre(r, node < nn ? node : nn - 1);
  if (on) {
    int i, j, k;
    node_ijk(node, op.L, i, j, k);
    ax_st_part<ST_LPN>(op, in, r, i, j, k, node, wave, ax);
  }
  if (wave > 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) red[wave - 1][c][lane] = ax[c];
  }
  __syncthreads();
  if (!gate_open(g, gr)) return;  // uniform
  if (wave == 0 && on) {
#pragma unroll
    for (int w = 0; w < ST_LPN - 1; ++w)
#pragma unroll
      for (int c = 0; c < 3; ++c) ax[c] += red[w][c][lane];
    ep.put(r, node, ax, pv, a0, a1);
  }
  if constexpr (Ep::RED) {
    // only wave 0 holds epilogue sums
    if (wave == 0) {
      a0 = wave_sum(a0);
      a1 = wave_sum(a1);
      if (lane == 0) {
        part[(size_t)r * MAX_BLOCKS + bx] = a0;
        part[(size_t)(4 + r) * MAX_BLOCKS + bx] = a1;
      }
    }
  }
}

int apply_blocks(int kind, const Lat& L, bool fp64) {
  const long nn = L.nn();
  if (kind == OP_ST27) return (int)((nn + ST_NODES - 1) / ST_NODES);
  if (kind == OP_MF_Q1) return wt_grid(L, fp64).blocks();
  return nblocks(nn);
}

// Instrumentation: events attached to the next operator launch receive the
// kernel's own start and end timestamps (the dispatch packet's, as a
// profiler's kernel trace records them), not those of separate markers.
static thread_local hipEvent_t g_time_start = nullptr, g_time_stop = nullptr;
void time_next_apply(hipEvent_t start, hipEvent_t stop) {
  g_time_start = start;
  g_time_stop = stop;
}

template <typename K, typename... Args>
static void launch_op_lds(K kernel, dim3 grid, size_t lds, hipStream_t st, Args... args) {
  if (g_time_start || g_time_stop) {
    hipExtLaunchKernelGGL(kernel, grid, dim3(BS), (uint32_t)lds, st, g_time_start, g_time_stop, 0,
                          args...);
    g_time_start = g_time_stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, dim3(BS), lds, st, args...);
  }
  MGCG_HIP(hipGetLastError());
}

template <typename K, typename... Args>
static void launch_op_b(K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args) {
  if (g_time_start || g_time_stop) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, st, g_time_start, g_time_stop, 0, args...);
    g_time_start = g_time_stop = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
  }
  MGCG_HIP(hipGetLastError());
}
template <typename K, typename... Args>
static void launch_op(K kernel, dim3 grid, hipStream_t st, Args... args) {
  launch_op_b(kernel, grid, dim3(BS), st, args...);
}

template <typename T, class Op, class In, class Ep>
static void run_apply(const Op& op, const In& in, const Ep& ep, int nrhs, const CgScalars* gate,
                      int gate_state, hipStream_t st, double* part = nullptr) {
  const long nn = op.L.nn();
  if constexpr (std::is_same<Op, OpST<T>>::value) {
    const int nb = (int)((nn + ST_NODES - 1) / ST_NODES);
    if (Ep::RED && nb > MAX_BLOCKS) throw Error(-1, "mesh too large for the reduction buffer");
    if (st_lpn<T>(nn) == 7)
      launch_op_b(k_apply_st<T, In, Ep, 7>, dim3(nb, nrhs), dim3(StShape<7>::threads), st, op, in,
                  ep, nrhs, gate, gate_state, part);
    else
      launch_op_b(k_apply_st<T, In, Ep, 4>, dim3(nb, nrhs), dim3(StShape<4>::threads), st, op, in,
                  ep, nrhs, gate, gate_state, part);
  } else if constexpr (std::is_same<Op, OpEQ2<T>>::value) {
    // two passes: element products, then the node gather with the epilogue
    // (timing events, when set, span both)
    const int ne = (int)(((long)(op.L.nx - 1) / 2 * ((op.L.ny - 1) / 2) * ((op.L.nz - 1) / 2) +
                          EQ_EPB - 1) / EQ_EPB);
    hipEvent_t t_stop = g_time_stop;
    g_time_stop = nullptr;
    if (op.p == 3) {
      const long nel3 = (long)((op.L.nx - 1) / 3) * ((op.L.ny - 1) / 3) * ((op.L.nz - 1) / 3);
      if (op.s2) {
        const dim3 g3((unsigned)((nel3 + E3_BS / S3_ND - 1) / (E3_BS / S3_ND)), 1);
        switch (nrhs) {
          case 1: launch_op_b(k_e3_elem<T, 1, In, S3_ND>, g3, dim3(E3_BS), st, op, in, nrhs, gate, gate_state); break;
          case 2: launch_op_b(k_e3_elem<T, 2, In, S3_ND>, g3, dim3(E3_BS), st, op, in, nrhs, gate, gate_state); break;
          case 3: launch_op_b(k_e3_elem<T, 3, In, S3_ND>, g3, dim3(E3_BS), st, op, in, nrhs, gate, gate_state); break;
          default: launch_op_b(k_e3_elem<T, 4, In, S3_ND>, g3, dim3(E3_BS), st, op, in, nrhs, gate, gate_state); break;
        }
      } else {
        const dim3 g3((unsigned)nel3, 1);
        switch (nrhs) {
          case 1: launch_op_b(k_e3_elem<T, 1, In, L3_ND>, g3, dim3(E3_BS), st, op, in, nrhs, gate, gate_state); break;
          case 2: launch_op_b(k_e3_elem<T, 2, In, L3_ND>, g3, dim3(E3_BS), st, op, in, nrhs, gate, gate_state); break;
          case 3: launch_op_b(k_e3_elem<T, 3, In, L3_ND>, g3, dim3(E3_BS), st, op, in, nrhs, gate, gate_state); break;
          default: launch_op_b(k_e3_elem<T, 4, In, L3_ND>, g3, dim3(E3_BS), st, op, in, nrhs, gate, gate_state); break;
        }
      }
      g_time_stop = t_stop;
      const OpEQ3Y<T> gy{op.L, op.Y, op.mask};
      const int nb = nblocks(nn);
      if (Ep::RED && nb > MAX_BLOCKS) throw Error(-1, "mesh too large for the reduction buffer");
      launch_op(k_apply<T, OpEQ3Y<T>, In, Ep>, dim3(nb, nrhs), st, gy, in, ep, nrhs, gate,
                gate_state, part);
      return;
    }
    if (op.s2) {
      const int ns = (int)(((long)(op.L.nx - 1) / 2 * ((op.L.ny - 1) / 2) * ((op.L.nz - 1) / 2) +
                            ES_EPB - 1) / ES_EPB);
      switch (nrhs) {
        case 1: launch_op(k_es2_elem<T, 1, In>, dim3(ns, 1), st, op, in, nrhs, gate, gate_state); break;
        case 2: launch_op(k_es2_elem<T, 2, In>, dim3(ns, 1), st, op, in, nrhs, gate, gate_state); break;
        case 3: launch_op(k_es2_elem<T, 3, In>, dim3(ns, 1), st, op, in, nrhs, gate, gate_state); break;
        default: launch_op(k_es2_elem<T, 4, In>, dim3(ns, 1), st, op, in, nrhs, gate, gate_state); break;
      }
    } else {
      switch (nrhs) {
        case 1: launch_op(k_eq2_elem<T, 1, In>, dim3(ne, 1), st, op, in, nrhs, gate, gate_state); break;
        case 2: launch_op(k_eq2_elem<T, 2, In>, dim3(ne, 1), st, op, in, nrhs, gate, gate_state); break;
        case 3: launch_op(k_eq2_elem<T, 3, In>, dim3(ne, 1), st, op, in, nrhs, gate, gate_state); break;
        default: launch_op(k_eq2_elem<T, 4, In>, dim3(ne, 1), st, op, in, nrhs, gate, gate_state); break;
      }
    }
    g_time_stop = t_stop;
    const OpEQ2Y<T> gy{op.L, op.Y, op.mask};
    const int nb = nblocks(nn);
    if (Ep::RED && nb > MAX_BLOCKS) throw Error(-1, "mesh too large for the reduction buffer");
    launch_op(k_apply<T, OpEQ2Y<T>, In, Ep>, dim3(nb, nrhs), st, gy, in, ep, nrhs, gate,
              gate_state, part);
  } else {
    static_assert(std::is_same<Op, OpMF<T>>::value, "operator kind");
    const WtGrid wg = wt_grid(op.L, sizeof(T) == 8);
    const int nb = wg.blocks();
    if (Ep::RED && nb > MAX_BLOCKS) throw Error(-1, "mesh too large for the reduction buffer");
    launch_op_b(k_apply_mf_wt<T, Ep>, dim3(nb, nrhs), dim3(64 * WT_WAVES), st, op, in, ep, nrhs,
                gate, gate_state, part, wg.ntx, wg.nty, wg.kz, (int)wg.waves());
  }
}

template <typename T>
void launch_apply_mf(const OpMF<T>& op, const T* x, T* y, int nrhs, hipStream_t st) {
  const long nd = op.L.ndof();
  run_apply<T>(op, InPlain<T>{x, nd}, EpStore<T>{y, nd}, nrhs, nullptr, 0, st);
}
template <typename T>
void launch_apply_st(const OpST<T>& op, const T* x, T* y, int nrhs, hipStream_t st) {
  const long nd = op.L.ndof();
  run_apply<T>(op, InPlain<T>{x, nd}, EpStore<T>{y, nd}, nrhs, nullptr, 0, st);
}
template <typename T>
void launch_apply_eq2(const OpEQ2<T>& op, const T* x, T* y, int nrhs, hipStream_t st) {
  const long nd = op.L.ndof();
  run_apply<T>(op, InPlain<T>{x, nd}, EpStore<T>{y, nd}, nrhs, nullptr, 0, st);
}
template void launch_apply_mf<double>(const OpMF<double>&, const double*, double*, int, hipStream_t);
template void launch_apply_mf<float>(const OpMF<float>&, const float*, float*, int, hipStream_t);
template void launch_apply_st<double>(const OpST<double>&, const double*, double*, int, hipStream_t);
template void launch_apply_st<float>(const OpST<float>&, const float*, float*, int, hipStream_t);
template void launch_apply_eq2<double>(const OpEQ2<double>&, const double*, double*, int, hipStream_t);
template void launch_apply_eq2<float>(const OpEQ2<float>&, const float*, float*, int, hipStream_t);

// ------------------------------------------------------------ CG (FP64)
// Per iteration (load cases in parallel, each with its own scalars):
//   q = A p              [apply, partials p.q]
//   x += a p, r -= a q   [every block re-sums p.q -> a; partials r.r]
//   state                [1 block: r.r -> converged? -> CHECK]
//   r = f - A x          [only for load cases under CHECK; partials]
//   state                [1 block: true residual -> DONE / continue]
//   z = M r              [V-cycle]
//   r.z, r_old.z         [partials]
//   p = z + b p          [every block re-sums -> b]
// The scalar r.z is double-buffered by iteration parity so that no kernel
// reads a value another block of the same kernel writes.
template <class In, class Ep>
static void fine_dispatch(const FineOp& A, const In& in, const Ep& ep, int nrhs,
                          const CgScalars* gate, int gate_state, hipStream_t st, double* part) {
  switch (A.kind) {
    case OP_MF_Q1: run_apply<double>(A.mf, in, ep, nrhs, gate, gate_state, st, part); break;
    case OP_ST27: run_apply<double>(A.st, in, ep, nrhs, gate, gate_state, st, part); break;
    default: run_apply<double>(A.eq2, in, ep, nrhs, gate, gate_state, st, part); break;
  }
}

static int fine_blocks(const FineOp& A) { return apply_blocks(A.kind, A.lat(), true); }

__global__ void k_fin_init(CgScalars* cs, int nrhs, const double* part, int nb) {
  __shared__ double sh[BS / 64];
  for (int r = 0; r < nrhs; ++r) {
    const double rr = block_sum(part + (size_t)r * MAX_BLOCKS, nb, sh);
    const double ff = block_sum(part + (size_t)(4 + r) * MAX_BLOCKS, nb, sh);
    if (threadIdx.x == 0) {
      CgScalars& c = cs[r];
      c.rr = rr;
      c.ff = ff;
      c.tol2 = c.tol2 * ff;  // cg_reset stored rtol^2
      c.iters = 0;
      c.replacements = 0;
      c.rzs[0] = c.rzs[1] = 0.0;
      c.beta = 0.0;
      c.rr_best = rr;
      c.stall = 0;
      c.bad = 0;
      c.rr_min = rr;
      c.since = 0;
      c.restart = 0;
      if (!isfinite(rr) || !isfinite(ff))
        c.state = CG_BREAKDOWN;
      else if (ff == 0.0 || rr <= c.tol2)
        c.state = CG_DONE;
      else
        c.state = CG_ACTIVE;
    }
  }
}

void cg_init_residual(const FineOp& A, const double* f, const double* x, double* r, int nrhs,
                      CgScalars* cs, RedBuf red, hipStream_t st) {
  const long nd = A.lat().ndof();
  double* part = red.partials + RED_INIT * RED_REGION;
  fine_dispatch(A, InPlain<double>{x, nd}, EpInitResid{f, r, nd, nrhs}, nrhs, nullptr, 0, st, part);
  hipLaunchKernelGGL(k_fin_init, dim3(1), dim3(BS), 0, st, cs, nrhs, part, fine_blocks(A));
  MGCG_HIP(hipGetLastError());
}

// Warm start scaled along the previous solution: the minimiser of the energy
// J(a x) = a^2/2 x^T A x - a f^T x is a = f^T x / x^T A x, and x^T A x =
// x^T (f - r) with the residual r = f - A x already computed; J(a x) is then
// at most min(J(0), J(x)).  Fixed-order block partials, no atomics.
__global__ __launch_bounds__(BS) void k_warm_dots(const double* __restrict__ f,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ r, long ndof,
                                                  int nrhs, double* part) {
  for (int rr = 0; rr < nrhs; ++rr) {
    const size_t o = (size_t)rr * ndof;
    double fx = 0.0, xr = 0.0;
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < ndof; i += (long)gridDim.x * BS) {
      const double xv = x[o + i];
      fx = fma(f[o + i], xv, fx);
      xr = fma(xv, r[o + i], xr);
    }
    block_partial2(fx, xr, part + (size_t)rr * MAX_BLOCKS + blockIdx.x,
                   part + (size_t)(4 + rr) * MAX_BLOCKS + blockIdx.x);
  }
}

__device__ __forceinline__ double warm_alpha(double fx, double xr) {
  const double xax = fx - xr;  // x^T A x
  const double a = fx / xax;
  return (xax > 0.0 && isfinite(a)) ? a : 0.0;
}

__global__ __launch_bounds__(BS) void k_warm_scale(const double* __restrict__ f, double* x,
                                                   double* r, long ndof, int nrhs,
                                                   const double* part, int nbp, double* part2) {
  __shared__ double sh[BS / 64];
  for (int rr = 0; rr < nrhs; ++rr) {
    const double fx = block_sum(part + (size_t)rr * MAX_BLOCKS, nbp, sh);
    const double xr = block_sum(part + (size_t)(4 + rr) * MAX_BLOCKS, nbp, sh);
    const double a = warm_alpha(fx, xr);
    const size_t o = (size_t)rr * ndof;
    double s = 0.0;
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < ndof; i += (long)gridDim.x * BS) {
      const double rn = (1.0 - a) * f[o + i] + a * r[o + i];
      x[o + i] = a * x[o + i];
      r[o + i] = rn;
      s = fma(rn, rn, s);
    }
    block_partial1(s, part2 + (size_t)rr * MAX_BLOCKS + blockIdx.x);
  }
}

__global__ void k_fin_warm(CgScalars* cs, int nrhs, const double* part2, int nb) {
  __shared__ double sh[BS / 64];
  for (int r = 0; r < nrhs; ++r) {
    const double rr = block_sum(part2 + (size_t)r * MAX_BLOCKS, nb, sh);
    if (threadIdx.x == 0) {
      CgScalars& c = cs[r];
      if (c.state != CG_ACTIVE && c.state != CG_DONE) continue;  // breakdown stays
      c.rr = rr;
      c.rr_best = rr;
      c.rr_min = rr;
      c.since = 0;
      if (!isfinite(rr))
        c.state = CG_BREAKDOWN;
      else if (c.ff == 0.0 || rr <= c.tol2)
        c.state = CG_DONE;
      else
        c.state = CG_ACTIVE;
    }
  }
}

void cg_scale_warm(const double* f, double* x, double* r, long ndof, int nrhs, CgScalars* cs,
                   RedBuf red, hipStream_t st) {
  const int nb = vec_grid(ndof);
  double* part = red.partials + RED_INIT * RED_REGION;  // read by k_fin_init before
  double* part2 = red.partials + RED_RR * RED_REGION;
  hipLaunchKernelGGL(k_warm_dots, dim3(nb), dim3(BS), 0, st, f, (const double*)x,
                     (const double*)r, ndof, nrhs, part);
  hipLaunchKernelGGL(k_warm_scale, dim3(nb), dim3(BS), 0, st, f, x, r, ndof, nrhs,
                     (const double*)part, nb, part2);
  hipLaunchKernelGGL(k_fin_warm, dim3(1), dim3(BS), 0, st, cs, nrhs, (const double*)part2, nb);
  MGCG_HIP(hipGetLastError());
}

void cg_apply_alpha(const FineOp& A, const double* p, double* q, int nrhs, CgScalars* cs,
                    RedBuf red, hipStream_t st) {
  const long nd = A.lat().ndof();
  fine_dispatch(A, InPlain<double>{p, nd}, EpDotPQ{p, q, nd}, nrhs, cs, CG_ACTIVE, st,
                red.partials + RED_PQ * RED_REGION);
}

// x += a p, r -= a q with a = r.z / p.q re-summed by every block.
// WB: bytes of a W D^-1 value of the V-cycle input written with r (0: none),
// a template parameter so that the operand loads carry no branch.
template <int WB>
__global__ __launch_bounds__(BS) void k_update_xr(const double* __restrict__ p,
                                                  const double* __restrict__ q, double* x, double* r,
                                                  long ndof, int nrhs, CgScalars* cs,
                                                  const double* __restrict__ ppq, int nbq,
                                                  double* prr, VPrep vp) {
  __shared__ double sh[BS / 64];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const long step = (long)gridDim.x * BS * VU;
  // the load case's scalars are loaded first and tested once its first
  // operands and partial sums are on their way
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    if (rr >= nrhs) continue;
    int state = state_of(cs, rr), it = cs_int(cs, rr, CS_OFF(iters));
    double rz0 = cs_dbl(cs, rr, CS_OFF(rzs)), rz1 = cs_dbl(cs, rr, CS_OFF(rzs) + 8);
    const size_t o = (size_t)rr * ndof;
    const size_t nb = (size_t)ndof * sizeof(double);
    const __amdgpu_buffer_rsrc_t bp = make_rsrc(p + o, nb), bq = make_rsrc(q + o, nb),
                                 bx = make_rsrc(x + o, nb), br = make_rsrc(r + o, nb);
    const __amdgpu_buffer_rsrc_t bw = make_rsrc(vp.wD, (size_t)ndof * (WB ? WB : 8));
    double pv[VU], qv[VU], xv[VU], rv[VU], wv[VU];
    auto fetch = [&](long i0) {
#pragma unroll
      for (int k = 0; k < VU; ++k) {
        const int off = (int)((i0 + k * BS) * sizeof(double));  // past ndof: reads 0
        pv[k] = bload<double>(bp, off, 0);
        qv[k] = bload<double>(bq, off, 0);
        xv[k] = bload<double>(bx, off, 0);
        rv[k] = bload<double>(br, off, 0);
        if constexpr (WB == 4)
          wv[k] = (double)bload<float>(bw, (int)((i0 + k * BS) * sizeof(float)), 0);
        else if constexpr (WB == 8)
          wv[k] = bload<double>(bw, off, 0);
        else
          wv[k] = 0.0;
      }
    };
    long i0 = (long)blockIdx.x * BS * VU + threadIdx.x;
    fetch(i0);  // the first pass's operands travel with the partial sums
    const double spq = block_sum_loads(ppq + (size_t)rr * MAX_BLOCKS, nbq);
    pin(state);
    pin(it);
    pin(rz0);
    pin(rz1);
    const double pq = block_sum_finish(spq, sh);
    if (state != CG_ACTIVE) continue;  // uniform
    const double rz = ((it + 1) & 1) ? rz1 : rz0;
    const double a = (pq > 0.0 && isfinite(pq)) ? rz / pq : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cs[rr].pq = pq;
      cs[rr].alpha = a;
    }
    double s = 0.0;
    for (; i0 < ndof; i0 += step) {
#pragma unroll
      for (int k = 0; k < VU; ++k) {
        const long i = i0 + k * BS;
        const double rn = rv[k] - a * qv[k];
        s += rn * rn;
        if (i < ndof) {
          x[o + i] = xv[k] + a * pv[k];
          r[o + i] = rn;
          if constexpr (WB == 4) {
            const float b = (float)rn;
            ((float*)vp.b0)[o + i] = b;
            ((float*)vp.x0)[o + i] = (float)wv[k] * b;
          } else if constexpr (WB == 8) {
            ((double*)vp.x0)[o + i] = wv[k] * rn;
          }
        }
      }
      if (i0 + step < ndof) fetch(i0 + step);
    }
    acc[rr] = s;
  }
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
    if (rr < nrhs) block_partial1(acc[rr], prr + (size_t)rr * MAX_BLOCKS + blockIdx.x);
}

// Convergence test of the recurrence residual (one block).
__global__ void k_fin_rr(CgScalars* cs, int nrhs, const double* part, int nb) {
  __shared__ double sh[BS / 64];
  for (int r = 0; r < nrhs; ++r) {
    // the scalars the test needs travel with the partial sums
    int state = state_of(cs, r), it = cs_int(cs, r, CS_OFF(iters)),
        bad = cs_int(cs, r, CS_OFF(bad)), maxit = cs_int(cs, r, CS_OFF(maxit)),
        every = cs_int(cs, r, CS_OFF(replace_every)), since = cs_int(cs, r, CS_OFF(since)),
        reps = cs_int(cs, r, CS_OFF(replacements));
    double pq = cs_dbl(cs, r, CS_OFF(pq)), tol2 = cs_dbl(cs, r, CS_OFF(tol2)),
           rmin = cs_dbl(cs, r, CS_OFF(rr_min));
    const double s = block_sum_loads(part + (size_t)r * MAX_BLOCKS, nb);
    pin(state);
    pin(it);
    pin(bad);
    pin(maxit);
    pin(every);
    pin(since);
    pin(reps);
    pin(pq);
    pin(tol2);
    pin(rmin);
    const double rr = block_sum_finish(s, sh);
    if (state != CG_ACTIVE) continue;  // uniform
    if (threadIdx.x == 0) {
      CgScalars& c = cs[r];
      c.rr = rr;
      it += 1;
      c.iters = it;
      c.restart = 0;  // consumed by this iteration's direction update
      const bool progress = rr < 0.81 * rmin;
      if (progress) c.rr_min = rr;
      c.since = progress ? 0 : since + 1;
      // Below the attainable accuracy the recurrence residual no longer
      // tracks the true one: after a replacement it can sit above the
      // tolerance, or grow.  Either sends the iteration to a true-residual
      // check, where the stall count ends it.
      const bool stuck = reps > 0 && since + 1 >= 32;
      const bool grows = !(rr <= 1e8 * rmin);
      if (!(pq > 0.0) || !isfinite(pq) || bad || !isfinite(rr))
        c.state = CG_BREAKDOWN;
      else if (rr <= tol2 || it >= maxit || (every > 0 && it % every == 0) || stuck || grows)
        c.state = CG_CHECK;
    }
    __syncthreads();
  }
}

void cg_update_xr(const double* p, const double* q, double* x, double* r, long ndof, int nrhs,
                  CgScalars* cs, RedBuf red, int nbq, VPrep vp, hipStream_t st) {
  double* prr = red.partials + RED_RR * RED_REGION;
  const int g = vec_grid(ndof);
  auto kern = !vp.x0 ? k_update_xr<0> : vp.f32 ? k_update_xr<4> : k_update_xr<8>;
  hipLaunchKernelGGL(kern, dim3(g), dim3(BS), 0, st, p, q, x, r, ndof, nrhs, cs,
                     red.partials + RED_PQ * RED_REGION, nbq, prr, vp);
  MGCG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_fin_rr, dim3(1), dim3(BS), 0, st, cs, nrhs, prr, g);
  MGCG_HIP(hipGetLastError());
}

// After a true-residual check: converged, out of iterations, stagnated
// (three checks in a row without a 10% decrease of the true residual, i.e.
// at the attainable accuracy), diverged, or continue with the residual
// replaced by the true one.
__global__ void k_fin_true(CgScalars* cs, int nrhs, const double* part, int nb) {
  if (!any_state(cs, nrhs, CG_CHECK)) return;
  __shared__ double sh[BS / 64];
  for (int r = 0; r < nrhs; ++r) {
    if (cs[r].state != CG_CHECK) continue;
    const double rr = block_sum(part + (size_t)r * MAX_BLOCKS, nb, sh);
    if (threadIdx.x == 0) {
      CgScalars& c = cs[r];
      c.rr = rr;
      c.replacements += 1;
      if (rr < 0.81 * c.rr_best) {
        c.rr_best = rr;
        c.stall = 0;
      } else {
        c.stall += 1;
      }
      if (!isfinite(rr) || rr > 1e30 * c.ff) {
        c.state = CG_BREAKDOWN;
      } else if (rr <= c.tol2) {
        c.state = CG_DONE;
      } else if (c.iters >= c.maxit || c.stall >= 3) {
        c.state = CG_MAXIT;
      } else {
        // continue from the true residual with a fresh direction: the old
        // one belongs to the recurrence it replaces
        c.state = CG_ACTIVE;
        c.rr_min = rr;
        c.since = 0;
        c.restart = 1;
      }
    }
    __syncthreads();
  }
}

void cg_true_residual(const FineOp& A, const double* f, const double* x, double* r, int nrhs,
                      CgScalars* cs, RedBuf red, VPrep vp, hipStream_t st) {
  const long nd = A.lat().ndof();
  double* part = red.partials + RED_TR * RED_REGION;
  fine_dispatch(A, InPlain<double>{x, nd}, EpTrueResid{f, r, nd, vp}, nrhs, cs, CG_CHECK, st,
                part);
  hipLaunchKernelGGL(k_fin_true, dim3(1), dim3(BS), 0, st, cs, nrhs, part, fine_blocks(A));
  MGCG_HIP(hipGetLastError());
}

// r.z and, for the FP32 V-cycle's flexible beta, q.z (partials per block).
template <typename TZ>
__global__ __launch_bounds__(BS) void k_beta(const double* __restrict__ r,
                                             const double* __restrict__ q,
                                             const TZ* __restrict__ z, long ndof, int nrhs,
                                             const CgScalars* cs, double* part) {
  constexpr bool flexible = sizeof(TZ) == 4;
  if (!any_state(cs, nrhs, CG_ACTIVE)) return;
  double a0[4] = {0, 0, 0, 0}, a1[4] = {0, 0, 0, 0};
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    if (rr >= nrhs || cs[rr].state != CG_ACTIVE) continue;
    const size_t o = (size_t)rr * ndof;
    const size_t nb = (size_t)ndof * sizeof(double);
    const __amdgpu_buffer_rsrc_t br = make_rsrc(r + o, nb), bo = make_rsrc(q + o, nb),
                                 bz = make_rsrc(z + o, (size_t)ndof * sizeof(TZ));
    double s0 = 0.0, s1 = 0.0;
    for (long i0 = (long)blockIdx.x * BS * VU + threadIdx.x; i0 < ndof;
         i0 += (long)gridDim.x * BS * VU) {
      double rv[VU], ov[VU], zv[VU];
#pragma unroll
      for (int k = 0; k < VU; ++k) {
        const long i = i0 + k * BS;
        rv[k] = bload<double>(br, (int)(i * sizeof(double)), 0);
        ov[k] = flexible ? bload<double>(bo, (int)(i * sizeof(double)), 0) : 0.0;
        zv[k] = (double)bload<TZ>(bz, (int)(i * sizeof(TZ)), 0);
      }
#pragma unroll
      for (int k = 0; k < VU; ++k) {
        s0 += rv[k] * zv[k];
        s1 += ov[k] * zv[k];
      }
    }
    a0[rr] = s0;
    a1[rr] = s1;
  }
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
    if (rr < nrhs)
      block_partial2(a0[rr], a1[rr], part + (size_t)rr * MAX_BLOCKS + blockIdx.x,
                     part + (size_t)(4 + rr) * MAX_BLOCKS + blockIdx.x);
}

int cg_beta_blocks(long ndof) { return vec_grid(ndof); }

template <typename TZ>
void cg_beta(const double* r, const double* q, const TZ* z, long ndof, int nrhs, CgScalars* cs,
             RedBuf red, hipStream_t st) {
  hipLaunchKernelGGL(k_beta<TZ>, dim3(vec_grid(ndof)), dim3(BS), 0, st, r, q, z, ndof, nrhs, cs,
                     red.partials + RED_RZ * RED_REGION);
  MGCG_HIP(hipGetLastError());
}
template void cg_beta<double>(const double*, const double*, const double*, long, int, CgScalars*,
                              RedBuf, hipStream_t);
template void cg_beta<float>(const double*, const double*, const float*, long, int, CgScalars*,
                             RedBuf, hipStream_t);

// p = z + b p; b re-summed by every block: standard beta for the symmetric
// FP64 V-cycle, flexible (Polak-Ribiere) beta for the FP32 one, whose
// numerator (r - r_old).z is -alpha q.z (r - r_old = -alpha q), b = 0 for
// the first direction and after a restart.
template <typename TZ>
__global__ __launch_bounds__(BS) void k_update_p(const TZ* __restrict__ z, double* p, long ndof,
                                                 int nrhs, CgScalars* cs,
                                                 const double* __restrict__ part, int nbz) {
  __shared__ double sh[BS / 64];
  const long step = (long)gridDim.x * BS * VU;
  // the FP32 V-cycle is the flexible one
  constexpr bool flexible = sizeof(TZ) == 4;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    if (rr >= nrhs) continue;
    // scalars loaded first, tested once the first operands are on their way
    int state = state_of(cs, rr), it = cs_int(cs, rr, CS_OFF(iters)),
        restart = cs_int(cs, rr, CS_OFF(restart));
    double rz0 = cs_dbl(cs, rr, CS_OFF(rzs)), rz1 = cs_dbl(cs, rr, CS_OFF(rzs) + 8),
           alpha = cs_dbl(cs, rr, CS_OFF(alpha));
    const size_t o = (size_t)rr * ndof;
    const size_t nb = (size_t)ndof * sizeof(double);
    const __amdgpu_buffer_rsrc_t bp = make_rsrc(p + o, nb),
                                 bz = make_rsrc(z + o, (size_t)ndof * sizeof(TZ));
    double pv[VU], zv[VU];
    auto fetch = [&](long i0) {
#pragma unroll
      for (int k = 0; k < VU; ++k) {
        const long i = i0 + k * BS;
        pv[k] = bload<double>(bp, (int)(i * sizeof(double)), 0);
        zv[k] = (double)bload<TZ>(bz, (int)(i * sizeof(TZ)), 0);
      }
    };
    long i0 = (long)blockIdx.x * BS * VU + threadIdx.x;
    fetch(i0);
    const double sn = block_sum_loads(part + (size_t)rr * MAX_BLOCKS, nbz);
    const double sm = flexible ? block_sum_loads(part + (size_t)(4 + rr) * MAX_BLOCKS, nbz) : 0.0;
    pin(state);
    pin(it);
    pin(restart);
    pin(rz0);
    pin(rz1);
    pin(alpha);
    const double rzn = block_sum_finish(sn, sh);
    const double qz = flexible ? block_sum_finish(sm, sh) : 0.0;
    if (state != CG_ACTIVE) continue;  // uniform
    const int par = it & 1;
    const double rzo = par ? rz1 : rz0;
    const bool ok = isfinite(rzn) && isfinite(qz);
    const double num = flexible ? -alpha * qz : rzn;
    const double b = (!ok || rzo == 0.0 || restart) ? 0.0 : num / rzo;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cs[rr].rzs[par ^ 1] = rzn;
      cs[rr].beta = b;
      if (!ok) cs[rr].bad = 1;
    }
    for (; i0 < ndof; i0 += step) {
#pragma unroll
      for (int k = 0; k < VU; ++k) {
        const long i = i0 + k * BS;
        if (i < ndof) p[o + i] = zv[k] + b * pv[k];
      }
      if (i0 + step < ndof) fetch(i0 + step);
    }
  }
}

template <typename TZ>
void cg_update_p(const TZ* z, double* p, long ndof, int nrhs, CgScalars* cs, RedBuf red, int nbz,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_update_p<TZ>, dim3(vec_grid(ndof)), dim3(BS), 0, st, z, p, ndof, nrhs, cs,
                     red.partials + RED_RZ * RED_REGION, nbz);
  MGCG_HIP(hipGetLastError());
}
template void cg_update_p<double>(const double*, double*, long, int, CgScalars*, RedBuf, int,
                                  hipStream_t);
template void cg_update_p<float>(const float*, double*, long, int, CgScalars*, RedBuf, int,
                                 hipStream_t);

// ------------------------------------------------------------ V-cycle
template <typename T, class In, class Ep>
static void v_dispatch(const VOps<T>& v, const In& in, const Ep& ep, int nrhs, const CgScalars* cs,
                       hipStream_t st) {
  switch (v.kind) {
    case OP_MF_Q1: run_apply<T>(v.mf, in, ep, nrhs, cs, CG_ACTIVE, st); break;
    case OP_ST27: run_apply<T>(v.st, in, ep, nrhs, cs, CG_ACTIVE, st); break;
    default: run_apply<T>(v.eq2, in, ep, nrhs, cs, CG_ACTIVE, st); break;
  }
}

template <typename T>
void v_jacobi(const VOps<T>& v, const T* b, const T* x, T* xo, T omega, int nrhs,
              const CgScalars* cs, hipStream_t st) {
  const long nd = v.L.ndof();
  v_dispatch(v, InPlain<T>{x, nd}, EpJacobi<T>{b, x, v.invD, omega, xo, nd}, nrhs, cs, st);
}

// First post-smoothing sweep of a small stencil level fused with the
// prolongation of the coarse correction.  The block's 64 nodes read their
// neighbours from LDS, where the block has staged y = x + P~ e over the three
// node ranges around it (plane dz holds nodes [n0 + dz P - nx - 1, + lr)),
// the prolongation done once per staged node.
template <typename T>
struct InLds {
  const T* sh;
  int n0, nx, ny, P, lr;
  struct Buf {
    const T* sh;
    int n0, nx, ny, P, lr;
    __device__ __forceinline__ void load_node(int ii, int jj, int kk, int dz, int voff,
                                              T v[3]) const {
      const int nb = ii + __mul24(nx, jj + __mul24(ny, kk));
      const int q = (dz + 1) * lr + (nb - (n0 + dz * P - nx - 1));
      const bool ok = voff != kBufOOB;
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] = ok ? sh[3 * q + c] : T(0);
    }
  };
  __device__ __forceinline__ Buf buf(int) const { return Buf{sh, n0, nx, ny, P, lr}; }
};

template <typename T>
__global__ __launch_bounds__(StShape<7>::threads) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_st_jacobi_prolong(OpST<T> op, const T* __restrict__ x, const T* __restrict__ e, Lat C,
                         const uint8_t* __restrict__ mf, const T* __restrict__ b,
                         const T* __restrict__ wD, T omega, T* xo, int nrhs,
                         const CgScalars* gate) {
  constexpr int ST_LPN = 7, ST_THREADS = StShape<7>::threads;  // small levels
  extern __shared__ __align__(16) unsigned char sh_raw[];
  T* sh = reinterpret_cast<T*>(sh_raw);
  __shared__ T red[ST_LPN - 1][3][ST_NODES];
  const Gate g = gate_load(gate, nrhs, CG_ACTIVE);
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / ST_NODES);
  const int lane = threadIdx.x % ST_NODES;
  int bx, r;
  xcd_tile(bx, r);
  const Lat L = op.L;
  const int nn = (int)L.nn(), nd = (int)L.ndof(), cnd = (int)C.ndof();
  const int nx = L.nx, P = L.nx * L.ny, lr = ST_NODES + 2 * L.nx + 2;
  const int n0 = bx * ST_NODES;
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(x + (size_t)r * nd, (size_t)nd * sizeof(T)),
                               re = make_rsrc(e + (size_t)r * cnd, (size_t)cnd * sizeof(T)),
                               rm = make_rsrc(mf, (size_t)nn);
  for (int q = threadIdx.x; q < 3 * lr; q += ST_THREADS) {
    const int plane = q / lr;
    const int node = n0 + (plane - 1) * P - nx - 1 + (q - plane * lr);
    const bool ok = node >= 0 && node < nn;
    int i, j, k;
    node_ijk(ok ? node : 0, L, i, j, k);
    T v[3], pe[3];
    bload3<T>(rx, ok ? 3 * node * (int)sizeof(T) : kBufOOB, v);
    prolong_at<T>(C, re, i, j, k, ok, pe);
    const int mfn = bload_u8(rm, ok ? node : kBufOOB);
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[3 * q + c] = v[c] + (((mfn >> c) & 1) ? T(0) : pe[c]);
  }
  const int node = n0 + lane;
  const bool on = node < nn;
  const int nodec = on ? node : nn - 1;
  // epilogue operands (wave 0 only: uniform branch)
  Pre3<T> bv{}, dv{};
  if (wave == 0) {
    bv = ld3(b + (size_t)r * nd + 3 * nodec);
    dv = ld3(wD + 3 * nodec);
  }
  __syncthreads();
  T ax[3] = {T(0), T(0), T(0)};
  if (on) {
    int i, j, k;
    node_ijk(node, L, i, j, k);
    ax_st_part<ST_LPN>(op, InLds<T>{sh, n0, nx, L.ny, P, lr}, r, i, j, k, node, wave, ax);
  }
  if (wave > 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) red[wave - 1][c][lane] = ax[c];
  }
  __syncthreads();
  if (!gate_open(g)) return;  // uniform
  if (wave == 0 && on) {
#pragma unroll
    for (int w = 0; w < ST_LPN - 1; ++w)
#pragma unroll
      for (int c = 0; c < 3; ++c) ax[c] += red[w][c][lane];
    const int qc = lr + nx + 1 + lane;  // the node itself: plane dz = 0
    T* out = xo + (size_t)r * nd + 3 * node;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T y = sh[3 * qc + c];
      out[c] = y + omega * dv.v[c] * (bv.v[c] - ax[c]);
    }
  }
}

template <typename T>
void v_jacobi_prolong(const VOps<T>& v, const VOps<T>& vc, const T* b, const T* x, T* xo,
                      T omega, const T* e, int nrhs, const CgScalars* cs, hipStream_t st) {
  if (v.kind != OP_ST27) throw Error(-1, "fused prolongation needs a stencil level");
  const long nn = v.L.nn();
  const int lr = ST_NODES + 2 * v.L.nx + 2;
  const size_t lds = (size_t)9 * lr * sizeof(T);
  if (lds > 64 * 1024) throw Error(-1, "level too wide for the fused prolongation");
  hipLaunchKernelGGL(k_st_jacobi_prolong<T>, dim3(apply_blocks(OP_ST27, v.L, sizeof(T) == 8), nrhs),
                     dim3(StShape<7>::threads), lds, st, v.st, x, e, vc.L, v.mask, b, v.invD, omega,
                     xo, nrhs, cs);
  MGCG_HIP(hipGetLastError());
}

template <typename T>
void v_jacobi_dot(const VOps<T>& v, const T* b, const T* x, T* xo, T omega, const double* r,
                  const double* q, int nrhs, const CgScalars* cs, RedBuf red, hipStream_t st) {
  const long nd = v.L.ndof();
  const EpJacobiDot<T> ep{b, x, v.invD, omega, xo, nd, r, q};
  double* part = red.partials + RED_RZ * RED_REGION;
  switch (v.kind) {
    case OP_MF_Q1: run_apply<T>(v.mf, InPlain<T>{x, nd}, ep, nrhs, cs, CG_ACTIVE, st, part); break;
    case OP_ST27: run_apply<T>(v.st, InPlain<T>{x, nd}, ep, nrhs, cs, CG_ACTIVE, st, part); break;
    default: run_apply<T>(v.eq2, InPlain<T>{x, nd}, ep, nrhs, cs, CG_ACTIVE, st, part); break;
  }
}

template <typename T>
void v_residual(const VOps<T>& v, const T* b, const T* x, T* r, int nrhs, const CgScalars* cs,
                hipStream_t st) {
  const long nd = v.L.ndof();
  v_dispatch(v, InPlain<T>{x, nd}, EpResid<T>{b, r, nd}, nrhs, cs, st);
}

// Level-0 input of the V-cycle: b0 = r in the V-cycle precision (only stored
// when it differs from FP64) and the first smoothing sweep x0 = W D^-1 b0.
template <typename T>
__global__ __launch_bounds__(BS) void k_prepare0(const double* __restrict__ r, T* b0,
                                                 const T* __restrict__ wD, T* x0, long ndof,
                                                 int nrhs, const CgScalars* cs) {
  if (!any_state(cs, nrhs, CG_ACTIVE)) return;
  for (int rr = 0; rr < nrhs; ++rr) {
    const size_t o = (size_t)rr * ndof;
    const __amdgpu_buffer_rsrc_t br = make_rsrc(r + o, (size_t)ndof * sizeof(double)),
                                 bw = make_rsrc(wD, (size_t)ndof * sizeof(T));
    for (long i0 = (long)blockIdx.x * BS * VU + threadIdx.x; i0 < ndof;
         i0 += (long)gridDim.x * BS * VU) {
      T bv[VU], wv[VU];
#pragma unroll
      for (int k = 0; k < VU; ++k) {
        const long i = i0 + k * BS;
        bv[k] = (T)bload<double>(br, (int)(i * sizeof(double)), 0);
        wv[k] = bload<T>(bw, (int)(i * sizeof(T)), 0);
      }
#pragma unroll
      for (int k = 0; k < VU; ++k) {
        const long i = i0 + k * BS;
        if (i < ndof) {
          if (b0) b0[o + i] = bv[k];
          x0[o + i] = wv[k] * bv[k];
        }
      }
    }
  }
}

template <typename T>
void v_prepare0(const double* r, T* b0, const T* wD, T* x0, long ndof, int nrhs,
                const CgScalars* cs, hipStream_t st) {
  hipLaunchKernelGGL(k_prepare0<T>, dim3(vec_grid(ndof)), dim3(BS), 0, st, r, b0, wD, x0, ndof,
                     nrhs, cs);
  MGCG_HIP(hipGetLastError());
}


// Restriction: coarse DOF (I, c) gathers component c of the 3x3x3 fine nodes
// around 2I with weights prod_d (1 - |offset_d| / 2).  Fine inputs vanish on
// fixed DOFs; the caller zeroes fixed coarse DOFs.  Out-of-range neighbours
// read through out-of-range offsets (0): no branches, so all 27 loads are
// issued back to back.
template <typename T>
__device__ __forceinline__ T restrict_at(const Lat& F, __amdgpu_buffer_rsrc_t rb, int I, int J,
                                         int K, int c) {
  int off[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const int i = 2 * I + q % 3 - 1, j = 2 * J + (q / 3) % 3 - 1, k = 2 * K + q / 9 - 1;
    const bool ok = (unsigned)i < (unsigned)F.nx && (unsigned)j < (unsigned)F.ny &&
                    (unsigned)k < (unsigned)F.nz;
    off[q] = ok ? (3 * lat_index(F, i, j, k) + c) * (int)sizeof(T) : kBufOOB;
  }
  T v[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) v[q] = bload<T>(rb, off[q], 0);
  T acc = T(0);
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
    const T w = T((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
    acc = fma(w, v[q], acc);
  }
  return acc;
}

// One thread per coarse DOF; also the coarse level's first smoothing sweep
// from zero, x = W D^-1 b, when xc is given.
template <typename T>
__global__ __launch_bounds__(BS) void k_restrict(Lat F, Lat C, const uint8_t* __restrict__ mf,
                                                 const uint8_t* __restrict__ mc,
                                                 const T* __restrict__ rf, T* bc,
                                                 const T* __restrict__ wDc, T* xc, int nrhs,
                                                 const CgScalars* cs) {
  const Gate g = gate_load(cs, nrhs, CG_ACTIVE);
  int bx, r;
  xcd_tile(bx, r);  // r: load case
  const long t = (long)bx * BS + threadIdx.x;
  const long cnd = C.ndof();
  if (t >= cnd) return;
  const long node = t / 3;
  const int c = (int)(t - 3 * node);
  int I, J, K;
  node_ijk(node, C, I, J, K);
  const long fnd = F.ndof();
  T acc = restrict_at<T>(F, make_rsrc(rf + (size_t)r * fnd, (size_t)fnd * sizeof(T)), I, J, K, c);
  // (mask read after the gathers so that all loads are in flight together)
  int mcn = mc[node];
  T wd = xc ? wDc[t] : T(0);
  pin(acc);
  pin(mcn);
  pin(wd);
  if (!gate_open(g)) return;
  const bool fixed = (mcn >> c) & 1;
  const T bv = fixed ? T(0) : acc;
  bc[(size_t)r * cnd + t] = bv;
  if (xc) xc[(size_t)r * cnd + t] = wd * bv;
  (void)mf;
}

// The cubic lattice's step onto its vertex lattice (coarse node I on fine
// node 3I), R = P^T of the linear interpolation with 1-D weights 1 at
// coincident nodes and (3 - |d|) / 3 at the fine nodes d = +-1, +-2 steps
// away: one thread per coarse DOF over the 5x5x5 fine nodes around 3I.
template <typename T>
__global__ __launch_bounds__(BS) void k_restrict3(Lat F, Lat C, const uint8_t* __restrict__ mc,
                                                  const T* __restrict__ rf, T* bc,
                                                  const T* __restrict__ wDc, T* xc, int nrhs,
                                                  const CgScalars* cs) {
  const Gate g = gate_load(cs, nrhs, CG_ACTIVE);
  int bx, r;
  xcd_tile(bx, r);  // r: load case
  const long t = (long)bx * BS + threadIdx.x;
  const long cnd = C.ndof();
  if (t >= cnd) return;
  const long node = t / 3;
  const int c = (int)(t - 3 * node);
  int I, J, K;
  node_ijk(node, C, I, J, K);
  const T* rr = rf + (size_t)r * F.ndof();
  T acc = T(0);
  for (int dz = -2; dz <= 2; ++dz) {
    const int k = 3 * K + dz;
    if ((unsigned)k >= (unsigned)F.nz) continue;
    for (int dy = -2; dy <= 2; ++dy) {
      const int j = 3 * J + dy;
      if ((unsigned)j >= (unsigned)F.ny) continue;
      const T wyz = T((3 - abs(dy)) * (3 - abs(dz))) / T(9);
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        const int i = 3 * I + dx;
        if ((unsigned)i >= (unsigned)F.nx) continue;
        acc = fma(wyz * T(3 - abs(dx)) / T(3), rr[3 * ((long)i + (long)F.nx * (j + (long)F.ny * k)) + c],
                  acc);
      }
    }
  }
  if (!gate_open(g)) return;
  const bool fixed = (mc[node] >> c) & 1;
  const T bv = fixed ? T(0) : acc;
  bc[(size_t)r * cnd + t] = bv;
  if (xc) xc[(size_t)r * cnd + t] = wDc[t] * bv;
}

template <typename T>
void v_restrict(Lat fine, Lat coarse, const uint8_t* mask_f, const uint8_t* mask_c, const T* rf,
                T* bc, const T* wDc, T* xc, int nrhs, const CgScalars* cs, hipStream_t st) {
  if (fine.nx - 1 == 3 * (coarse.nx - 1))
    hipLaunchKernelGGL(k_restrict3<T>, dim3(nblocks(coarse.ndof()), nrhs), dim3(BS), 0, st, fine,
                       coarse, mask_c, rf, bc, wDc, xc, nrhs, cs);
  else
    hipLaunchKernelGGL(k_restrict<T>, dim3(nblocks(coarse.ndof()), nrhs), dim3(BS), 0, st, fine,
                       coarse, mask_f, mask_c, rf, bc, wDc, xc, nrhs, cs);
  MGCG_HIP(hipGetLastError());
}

// Prolongation: fine node i interpolates the coarse nodes around i/2.
template <typename T>
__global__ __launch_bounds__(BS) void k_prolong(Lat F, Lat C, const uint8_t* __restrict__ mf,
                                                const uint8_t* __restrict__ mc,
                                                const T* __restrict__ ec, T* xf, int nrhs,
                                                int accumulate, const CgScalars* cs) {
  const Gate g = gate_load(cs, nrhs, CG_ACTIVE);
  int bx, r;
  xcd_tile(bx, r);  // r: load case
  const long node = (long)bx * BS + threadIdx.x;
  if (node >= F.nn()) return;
  int i, j, k;
  node_ijk(node, F, i, j, k);
  const int fnd = (int)F.ndof(), cnd = (int)C.ndof();
  // the old fine value (accumulate) is read branch-free together with the
  // corners: an out-of-range offset gives 0 when overwriting
  const __amdgpu_buffer_rsrc_t rq = make_rsrc(xf + (size_t)r * fnd, (size_t)fnd * sizeof(T));
  T pe[3], old[3];
  bload3<T>(rq, accumulate ? 3 * (int)node * (int)sizeof(T) : kBufOOB, old);
  prolong_at<T>(C, make_rsrc(ec + (size_t)r * cnd, (size_t)cnd * sizeof(T)), i, j, k, true, pe);
  int mfn = mf[node];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    pin(pe[c]);
    pin(old[c]);
  }
  pin(mfn);
  if (!gate_open(g)) return;
  T* qv = xf + (size_t)r * fnd + 3 * node;
#pragma unroll
  for (int c = 0; c < 3; ++c) qv[c] = old[c] + (((mfn >> c) & 1) ? T(0) : pe[c]);
}

// The cubic lattice's prolongation from its vertex lattice: fine node i
// lies q = i mod 3 steps past coarse node i / 3 and takes 1 - q/3 of it and
// q/3 of the next, per axis.
template <typename T>
__global__ __launch_bounds__(BS) void k_prolong3(Lat F, Lat C, const uint8_t* __restrict__ mf,
                                                 const T* __restrict__ ec, T* xf, int nrhs,
                                                 int accumulate, const CgScalars* cs) {
  const Gate g = gate_load(cs, nrhs, CG_ACTIVE);
  int bx, r;
  xcd_tile(bx, r);  // r: load case
  const long node = (long)bx * BS + threadIdx.x;
  if (node >= F.nn()) return;
  int i, j, k;
  node_ijk(node, F, i, j, k);
  const int p[3] = {i, j, k};
  int c0[3], nc[3];
  T w[3][2];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c0[d] = p[d] / 3;
    const int q = p[d] - 3 * c0[d];
    nc[d] = q ? 2 : 1;
    w[d][0] = T(3 - q) / T(3);
    w[d][1] = T(q) / T(3);
  }
  const T* er = ec + (size_t)r * C.ndof();
  T pe[3] = {T(0), T(0), T(0)};
  for (int cz = 0; cz < nc[2]; ++cz)
    for (int cy = 0; cy < nc[1]; ++cy)
      for (int cx = 0; cx < nc[0]; ++cx) {
        const T wt = w[0][cx] * w[1][cy] * w[2][cz];
        const long cn = (c0[0] + cx) + (long)C.nx * ((c0[1] + cy) + (long)C.ny * (c0[2] + cz));
#pragma unroll
        for (int c = 0; c < 3; ++c) pe[c] = fma(wt, er[3 * cn + c], pe[c]);
      }
  if (!gate_open(g)) return;
  const int mfn = mf[node];
  T* qv = xf + (size_t)r * F.ndof() + 3 * node;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T add = ((mfn >> c) & 1) ? T(0) : pe[c];
    qv[c] = accumulate ? qv[c] + add : add;
  }
}

template <typename T>
void v_prolong(Lat fine, Lat coarse, const uint8_t* mask_f, const uint8_t* mask_c, const T* ec,
               T* xf, int nrhs, bool accumulate, const CgScalars* cs, hipStream_t st) {
  if (fine.nx - 1 == 3 * (coarse.nx - 1))
    hipLaunchKernelGGL(k_prolong3<T>, dim3(nblocks(fine.nn()), nrhs), dim3(BS), 0, st, fine, coarse,
                       mask_f, ec, xf, nrhs, accumulate ? 1 : 0, cs);
  else
    hipLaunchKernelGGL(k_prolong<T>, dim3(nblocks(fine.nn()), nrhs), dim3(BS), 0, st, fine, coarse,
                       mask_f, mask_c, ec, xf, nrhs, accumulate ? 1 : 0, cs);
  MGCG_HIP(hipGetLastError());
}

// Coarsest solve x = A_c^{-1} b: one wavefront per row, the lanes split the
// columns (all loads of a row issued together; past ndof they read 0).
template <typename T>
__global__ __launch_bounds__(BS) void k_coarse_solve(const double* __restrict__ Ainv, int ld,
                                                     long ndof, const T* __restrict__ b, T* x,
                                                     int nrhs, const CgScalars* cs) {
  const Gate g = gate_load(cs, nrhs, CG_ACTIVE);
  const int row = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= ndof) return;
  const int r = blockIdx.y;  // load case
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(Ainv + (size_t)row * ld, (size_t)ndof * 8);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(b + (size_t)r * ndof, (size_t)ndof * sizeof(T));
  double s = 0.0;
  for (int c0 = 0; c0 < ndof; c0 += 8 * 64) {
    double a[8], v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = c0 + lane + 64 * q;
      a[q] = bload<double>(ra, c * 8, 0);
      v[q] = (double)bload<T>(rb, c * (int)sizeof(T), 0);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) s = fma(a[q], v[q], s);
  }
  pin(s);
  if (!gate_open(g)) return;
  s = wave_sum(s);
  if (lane == 0) x[(size_t)r * ndof + row] = (T)s;
}

template <typename T>
void v_coarse_solve(const double* Ainv, int ld, long ndof, const T* b, T* x, int nrhs,
                    const CgScalars* cs, hipStream_t st) {
  if (ndof == 0) return;
  hipLaunchKernelGGL(k_coarse_solve<T>, dim3((int)((ndof + 3) / 4), nrhs), dim3(BS), 0, st, Ainv,
                     ld, ndof, b, x, nrhs, cs);
  MGCG_HIP(hipGetLastError());
}

// Coarsest solve fused with the last restriction: b = P~^T r_f is computed by
// every block into LDS (at most CS_FUSE_MAX values, 27 L2 reads each), then
// the block's waves take one row of x = A_c^{-1} b each.  Saves a launch on
// a level where the launch costs more than the redundant restriction.
template <typename T>
__global__ __launch_bounds__(BS) void k_coarse_solve_r(const double* __restrict__ Ainv, int ld,
                                                       Lat F, Lat C, const uint8_t* __restrict__ mc,
                                                       const T* __restrict__ rf, T* x, int nrhs,
                                                       const CgScalars* cs) {
  __shared__ double bsh[CS_FUSE_MAX];
  const Gate g = gate_load(cs, nrhs, CG_ACTIVE);
  const int r = blockIdx.y;  // load case
  const int ndof = (int)C.ndof(), fnd = (int)F.ndof();
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(rf + (size_t)r * fnd, (size_t)fnd * sizeof(T));
  for (int t = threadIdx.x; t < ndof; t += BS) {
    const int node = t / 3, c = t - 3 * node;
    int I, J, K;
    node_ijk(node, C, I, J, K);
    const T acc = restrict_at<T>(F, rb, I, J, K, c);
    bsh[t] = ((mc[node] >> c) & 1) ? 0.0 : (double)acc;
  }
  __syncthreads();
  const int row = blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  if (row < ndof) {
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(Ainv + (size_t)row * ld, (size_t)ndof * 8);
    for (int c0 = 0; c0 < ndof; c0 += 4 * 64) {
      double a[4], v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = c0 + lane + 64 * q;
        a[q] = bload<double>(ra, c * 8, 0);
        v[q] = c < ndof ? bsh[c] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) s = fma(a[q], v[q], s);
    }
  }
  pin(s);
  if (!gate_open(g) || row >= ndof) return;
  s = wave_sum(s);
  if (lane == 0) x[(size_t)r * ndof + row] = (T)s;
}

template <typename T>
void v_coarse_solve_r(const double* Ainv, int ld, Lat fine, Lat coarse, const uint8_t* mask_c,
                      const T* rf, T* x, int nrhs, const CgScalars* cs, hipStream_t st) {
  const long ndof = coarse.ndof();
  if (ndof == 0) return;
  if (ndof > CS_FUSE_MAX) throw Error(-1, "coarsest level too large for the fused solve");
  hipLaunchKernelGGL(k_coarse_solve_r<T>, dim3((int)((ndof + 3) / 4), nrhs), dim3(BS), 0, st,
                     Ainv, ld, fine, coarse, mask_c, rf, x, nrhs, cs);
  MGCG_HIP(hipGetLastError());
}

#define VINST(T)                                                                                  \
  template void v_jacobi<T>(const VOps<T>&, const T*, const T*, T*, T, int, const CgScalars*,      \
                            hipStream_t);                                                         \
  template void v_jacobi_dot<T>(const VOps<T>&, const T*, const T*, T*, T, const double*,          \
                                const double*, int, const CgScalars*, RedBuf, hipStream_t);       \
  template void v_residual<T>(const VOps<T>&, const T*, const T*, T*, int, const CgScalars*,       \
                              hipStream_t);                                                       \
  template void v_restrict<T>(Lat, Lat, const uint8_t*, const uint8_t*, const T*, T*, const T*,   \
                              T*, int, const CgScalars*, hipStream_t);                            \
  template void v_prepare0<T>(const double*, T*, const T*, T*, long, int, const CgScalars*,        \
                              hipStream_t);                                                       \
  template void v_prolong<T>(Lat, Lat, const uint8_t*, const uint8_t*, const T*, T*, int, bool,    \
                             const CgScalars*, hipStream_t);                                      \
  template void v_coarse_solve<T>(const double*, int, long, const T*, T*, int, const CgScalars*,   \
                                  hipStream_t);                                                   \
  template void v_coarse_solve_r<T>(const double*, int, Lat, Lat, const uint8_t*, const T*, T*,    \
                                    int, const CgScalars*, hipStream_t);                          \
  template void v_jacobi_prolong<T>(const VOps<T>&, const VOps<T>&, const T*, const T*, T*, T,     \
                                    const T*, int, const CgScalars*, hipStream_t);
VINST(double)
VINST(float)

// ------------------------------------------------------------ inspection helpers
__global__ void k_mask_copy(const double* __restrict__ x, double* xm, const uint8_t* __restrict__ m,
                            long nn, int nrhs) {
  const long n3 = 3 * nn;
  for (long t = (long)blockIdx.x * BS + threadIdx.x; t < n3 * nrhs; t += (long)gridDim.x * BS) {
    const long i = t % n3;
    xm[t] = ((m[i / 3] >> (i % 3)) & 1) ? 0.0 : x[t];
  }
}
void mask_copy(const double* x, double* xm, const uint8_t* mask, long nn, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_mask_copy, dim3(vec_grid(3 * nn * nrhs)), dim3(BS), 0, st, x, xm, mask, nn,
                     nrhs);
  MGCG_HIP(hipGetLastError());
}
__global__ void k_identity_rows(const double* __restrict__ x, double* y,
                                const uint8_t* __restrict__ m, long nn, int nrhs) {
  const long n3 = 3 * nn;
  for (long t = (long)blockIdx.x * BS + threadIdx.x; t < n3 * nrhs; t += (long)gridDim.x * BS) {
    const long i = t % n3;
    if ((m[i / 3] >> (i % 3)) & 1) y[t] = x[t];
  }
}
void identity_rows(const double* x, double* y, const uint8_t* mask, long nn, int nrhs,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_identity_rows, dim3(vec_grid(3 * nn * nrhs)), dim3(BS), 0, st, x, y, mask,
                     nn, nrhs);
  MGCG_HIP(hipGetLastError());
}

// ------------------------------------------------------------ small utilities
template <typename TA, typename TB>
__global__ void k_convert(const TA* __restrict__ a, TB* b, long n) {
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) b[i] = (TB)a[i];
}
template <typename TA, typename TB>
void convert(const TA* a, TB* b, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_convert<TA, TB>), dim3(vec_grid(n)), dim3(BS), 0, st, a, b, n);
  MGCG_HIP(hipGetLastError());
}
template void convert<double, float>(const double*, float*, long, hipStream_t);
template void convert<float, double>(const float*, double*, long, hipStream_t);
template void convert<double, double>(const double*, double*, long, hipStream_t);

template <typename T>
__global__ void k_fill(T* a, T v, long n) {
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) a[i] = v;
}
template <typename T>
void fill(T* a, T v, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(vec_grid(n)), dim3(BS), 0, st, a, v, n);
  MGCG_HIP(hipGetLastError());
}
template void fill<double>(double*, double, long, hipStream_t);
template void fill<float>(float*, float, long, hipStream_t);
template void fill<int>(int*, int, long, hipStream_t);
template void fill<unsigned>(unsigned*, unsigned, long, hipStream_t);

__global__ void k_copy16(const uint4* __restrict__ a, uint4* b, long n) {
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) b[i] = a[i];
}
__global__ void k_copy1(const uint8_t* __restrict__ a, uint8_t* b, long n) {
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) b[i] = a[i];
}
void copy_bytes(const void* src, void* dst, size_t bytes, hipStream_t st) {
  const long n16 = (long)(bytes / 16);
  if (n16 > 0) {
    long g = (n16 + BS * 4 - 1) / (BS * 4);
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_copy16, dim3(g), dim3(BS), 0, st, (const uint4*)src, (uint4*)dst, n16);
  }
  const long rem = (long)(bytes - 16 * (size_t)n16);
  if (rem > 0)
    hipLaunchKernelGGL(k_copy1, dim3(1), dim3(BS), 0, st, (const uint8_t*)src + 16 * n16,
                       (uint8_t*)dst + 16 * n16, rem);
  MGCG_HIP(hipGetLastError());
}

}  // namespace mgcg

namespace mgcg {

__global__ void k_cg_reset(CgScalars* cs, int nrhs, double rtol2, int maxit, int replace_every,
                           int flexible) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  cs[r].flexible = flexible;
  cs[r].tol2 = rtol2;  // scaled by ||f||^2 in the initial residual kernel
  cs[r].maxit = maxit;
  cs[r].replace_every = replace_every;
  cs[r].state = CG_ACTIVE;
  cs[r].iters = 0;
  cs[r].replacements = 0;
  cs[r].restart = 0;
  cs[r].since = 0;
}

void cg_reset(CgScalars* cs, int nrhs, double rtol2, int maxit, int replace_every, int flexible,
              hipStream_t st) {
  hipLaunchKernelGGL(k_cg_reset, dim3(1), dim3(64), 0, st, cs, nrhs, rtol2, maxit, replace_every,
                     flexible);
  MGCG_HIP(hipGetLastError());
}

}  // namespace mgcg

namespace mgcg {

// ------------------------------------------------------------ fused small solves
// A whole PCG solve (Sec. 2.3: CG preconditioned by Algorithm 1) of one load
// case of a small trilinear problem in one workgroup: every operator, the
// V-cycle's levels, the coarsest inverse and the CG recurrences run between
// workgroup barriers instead of kernel boundaries, and one launch takes
// several problems and load cases, a workgroup each.  For meshes whose
// kernels are too small to fill the chip, where the cost of a kernel is its
// launch, ramp and drain (about 5 us), not its work.
//
// Finest level: matrix-free trilinear elements in their Haar basis
// (haar_element), the element products added into LDS accumulators of
// every node in 8 colour phases (elements of one colour, the parities of
// their indices, share no node), so no atomics are needed and the sums
// have a fixed order.  Coarse levels: the Galerkin stencils (ax_st_part).
// Coarsest: the explicit inverse, a wave per row.  Dot products: fixed-order
// workgroup sums.  The recurrences follow the device-gated CG: the
// recurrence residual triggers a check of the true residual; a check that
// fails replaces r and restarts the direction; three checks without a 10 %
// decrease end the solve.
constexpr int FZ_T = 512;
constexpr int FZ_W = FZ_T / 64;

__device__ __forceinline__ double fz_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < FZ_W; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// Level-wide vector passes over a thread's DOFs (or nodes, where the fixed
// DOFs matter: one mask byte per node), restrict-qualified and unrolled, so
// that the loads of several DOFs are in flight together (a workgroup has too
// few waves to hide a memory round trip per DOF).  acc: node sums in LDS,
// masked here (fixed rows return 0; the vectors vanish on fixed DOFs).
// n: DOFs (3 per node).
// r = f - A x; returns the thread's part of ||r||^2
__device__ __forceinline__ double fz_true_res(int n, const double* __restrict__ f,
                                              const double* __restrict__ acc,
                                              const uint8_t* __restrict__ m, double* __restrict__ r) {
  double s = 0.0;
#pragma unroll 4
  for (int node = threadIdx.x; node < n / 3; node += FZ_T) {
    const int mk = m[node];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int t = 3 * node + c;
      const double v = ((mk >> c) & 1) ? 0.0 : f[t] - acc[t];
      r[t] = v;
      s = fma(v, v, s);
    }
  }
  return s;
}
__device__ __forceinline__ double fz_dot(int n, const double* __restrict__ a, const double* __restrict__ b) {
  double s = 0.0;
#pragma unroll 8
  for (int t = threadIdx.x; t < n; t += FZ_T) s = fma(a[t], b[t], s);
  return s;
}
// p . (A p)
__device__ __forceinline__ double fz_dot_acc(int n, const double* __restrict__ p,
                                             const double* __restrict__ acc,
                                             const uint8_t* __restrict__ m) {
  double s = 0.0;
#pragma unroll 4
  for (int node = threadIdx.x; node < n / 3; node += FZ_T) {
    const int mk = m[node];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int t = 3 * node + c;
      s = fma(p[t], ((mk >> c) & 1) ? 0.0 : acc[t], s);
    }
  }
  return s;
}
// x += alpha p, r -= alpha A p; returns the thread's part of ||r||^2
__device__ __forceinline__ double fz_xr(int n, double alpha, const double* __restrict__ p,
                                        const double* __restrict__ acc,
                                        const uint8_t* __restrict__ m, double* __restrict__ x,
                                        double* __restrict__ r) {
  double s = 0.0;
#pragma unroll 4
  for (int node = threadIdx.x; node < n / 3; node += FZ_T) {
    const int mk = m[node];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int t = 3 * node + c;
      x[t] = fma(alpha, p[t], x[t]);
      const double v = r[t] - alpha * (((mk >> c) & 1) ? 0.0 : acc[t]);
      r[t] = v;
      s = fma(v, v, s);
    }
  }
  return s;
}
// p = z + beta p
__device__ __forceinline__ void fz_pz(int n, double beta, const double* __restrict__ z,
                                      double* __restrict__ p) {
#pragma unroll 8
  for (int t = threadIdx.x; t < n; t += FZ_T) p[t] = fma(beta, p[t], z[t]);
}
// x = w r
__device__ __forceinline__ void fz_scale(int n, const double* __restrict__ w,
                                         const double* __restrict__ r, double* __restrict__ x) {
#pragma unroll 8
  for (int t = threadIdx.x; t < n; t += FZ_T) x[t] = w[t] * r[t];
}
// out = r - A x
__device__ __forceinline__ void fz_res0(int n, const double* __restrict__ r,
                                        const double* __restrict__ acc,
                                        const uint8_t* __restrict__ m, double* __restrict__ out) {
#pragma unroll 4
  for (int node = threadIdx.x; node < n / 3; node += FZ_T) {
    const int mk = m[node];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int t = 3 * node + c;
      out[t] = ((mk >> c) & 1) ? 0.0 : r[t] - acc[t];
    }
  }
}
// x += w (b - A x), A x from LDS node sums (fine, masked) or a vector (coarse)
__device__ __forceinline__ void fz_jac(int n, const double* __restrict__ w, const double* __restrict__ b,
                                       const double* __restrict__ ax, const uint8_t* __restrict__ m,
                                       bool fine, double* __restrict__ x) {
#pragma unroll 4
  for (int node = threadIdx.x; node < n / 3; node += FZ_T) {
    const int mk = fine ? m[node] : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int t = 3 * node + c;
      const double a = ((mk >> c) & 1) ? 0.0 : ax[t];
      x[t] = fma(w[t], b[t] - a, x[t]);
    }
  }
}

// acc = K u on the finest level (before masking), in LDS.  A thread walks
// its elements colour by colour (a barrier after each colour) and loads the
// next element's 24 values and modulus before it computes the current one.
__device__ __attribute__((noinline)) void fz_mf_apply(const FzDesc& d, const double* __restrict__ u,
                                                      double* acc) {
  const Lat L = d.lv[0].L;
  const int nn = (int)L.nn();
  for (int t = threadIdx.x; t < 3 * nn; t += FZ_T) acc[t] = 0.0;
  __syncthreads();
  const int ex1 = L.nx - 1, ey1 = L.ny - 1, ez1 = L.nz - 1;
  const int P = L.nx * L.ny;
  const int tid = threadIdx.x;
  auto count = [&](int col) {  // this thread's elements of colour col
    const int cx = col & 1, cy = (col >> 1) & 1, cz = col >> 2;
    const int ne = ((ex1 - cx + 1) / 2) * ((ey1 - cy + 1) / 2) * ((ez1 - cz + 1) / 2);
    return ne > tid ? (ne - tid + FZ_T - 1) / FZ_T : 0;
  };
  auto advance = [&](int& col, int& k) {
    ++k;
    while (col < 8 && k >= count(col)) {
      ++col;
      k = 0;
    }
  };
  struct Item {
    double v[24];  // bottom face nodes (i, j), (i+1, j), (i, j+1), (i+1, j+1), then the top face
    double E;
    int n0;
  };
  // q = m quo + rem for q below 2^13 (the element count is at most 6,000):
  // the single-precision estimate is off by at most one
  auto divmod = [](int q, int m, int& quo, int& rem) {
    quo = (int)((float)q * __builtin_amdgcn_rcpf((float)m));
    rem = q - quo * m;
    if (rem < 0) {
      --quo;
      rem += m;
    } else if (rem >= m) {
      ++quo;
      rem -= m;
    }
  };
  auto load = [&](int col, int k, Item& it) {
    const int cx = col & 1, cy = (col >> 1) & 1, cz = col >> 2;
    const int mx = (ex1 - cx + 1) / 2, my = (ey1 - cy + 1) / 2;
    const int q = tid + k * FZ_T;
    int qy, ix, qz, iy;
    divmod(q, mx, qy, ix);
    divmod(qy, my, qz, iy);
    const int ex = cx + 2 * ix, ey = cy + 2 * iy, ez = cz + 2 * qz;
    it.n0 = ex + L.nx * ey + P * ez;
    it.E = d.E[ex + ex1 * (ey + ey1 * ez)];
#pragma unroll
    for (int zz = 0; zz < 2; ++zz)
#pragma unroll
      for (int cn = 0; cn < 4; ++cn) {
        const int nb = it.n0 + zz * P + (cn & 1) + L.nx * (cn >> 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) it.v[12 * zz + 3 * cn + c] = u[3 * nb + c];
      }
  };
  auto compute = [&](const Item& it) {
    // 2-D Haar transforms of the two faces (q = mx + 2 my)
    double fb[3][4], ft[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      {
        const double u00 = it.v[c], u10 = it.v[3 + c], u01 = it.v[6 + c], u11 = it.v[9 + c];
        const double a = u00 + u10, b = u10 - u00, cc = u01 + u11, dd = u11 - u01;
        fb[c][0] = a + cc;
        fb[c][1] = b + dd;
        fb[c][2] = cc - a;
        fb[c][3] = dd - b;
      }
      {
        const double u00 = it.v[12 + c], u10 = it.v[15 + c], u01 = it.v[18 + c], u11 = it.v[21 + c];
        const double a = u00 + u10, b = u10 - u00, cc = u01 + u11, dd = u11 - u01;
        ft[c][0] = a + cc;
        ft[c][1] = b + dd;
        ft[c][2] = cc - a;
        ft[c][3] = dd - b;
      }
    }
    double gb[3][4], gt[3][4];
    haar_element<double>(d.hv, fb, ft, it.E, gb, gt);
#pragma unroll
    for (int cn = 0; cn < 4; ++cn) {
      const int nb = it.n0 + (cn & 1) + L.nx * (cn >> 1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[3 * nb + c] += gb[c][cn];
        acc[3 * (nb + P) + c] += gt[c][cn];
      }
    }
  };
  Item cur, nxt;
  int pc = 0, pk = -1;
  advance(pc, pk);
  if (pc < 8) load(pc, pk, cur);
  for (int col = 0; col < 8; ++col) {
    const int n = count(col);
    for (int k = 0; k < n; ++k) {
      int nc = col, nk = k;
      advance(nc, nk);
      if (nc < 8) load(nc, nk, nxt);
      compute(cur);
      cur = nxt;
    }
    __syncthreads();
  }
}

// Level-wide steps of the V-cycle, each its own (not inlined) function so
// that the register budget of each is its own.
#define FZ_STEP __device__ __attribute__((noinline))

// y = A_l u (b null) or y = b - A_l u on a stencil level (identity rows
// baked into the stencil).  The 14 stored blocks are taken in 7 parts
// (blocks part and part + 7).  A work item is a node and two consecutive
// parts (the last item one part), so that a level of a few hundred nodes
// spreads over every thread and each thread waits for few rounds of loads;
// the node range of a pair is padded to whole waves, so a wave's items share
// their parts and the coefficient rows stay scalar.  The pair sums go to LDS
// (slot, the finest level's node sums, free while a stencil level runs; the
// host admits stencil levels of at most FZ_MAX_ST_NODES padded nodes) and
// each node adds its four in a fixed order.
FZ_STEP void fz_st_apply(const FzLevel& lv, const double* u, const double* b, double* y,
                         double* slot) {
  const int nn = (int)lv.L.nn();
  const OpST<double> op{lv.L, lv.coef};
  const InPlain<double> in{u, lv.L.ndof()};
  const int nnp = (nn + 63) & ~63;
  for (int q = threadIdx.x; q < 4 * nnp; q += FZ_T) {
    const int pr = __builtin_amdgcn_readfirstlane(q / nnp);  // whole waves per pair
    const int t = q - pr * nnp;
    if (t < nn) {
      int i, j, k;
      node_ijk(t, lv.L, i, j, k);
      double a[3], ap[3] = {0.0, 0.0, 0.0};
      ax_st_part<7, double, InPlain<double>>(op, in, 0, i, j, k, t, 2 * pr, a);
      if (pr < 3) ax_st_part<7, double, InPlain<double>>(op, in, 0, i, j, k, t, 2 * pr + 1, ap);
      for (int c = 0; c < 3; ++c) slot[(3 * pr + c) * nnp + t] = a[c] + ap[c];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nn; t += FZ_T)
    for (int c = 0; c < 3; ++c) {
      const double a = ((slot[c * nnp + t] + slot[(3 + c) * nnp + t]) + slot[(6 + c) * nnp + t]) +
                       slot[(9 + c) * nnp + t];
      y[3 * t + c] = b ? b[3 * t + c] - a : a;
    }
  __syncthreads();
}

// b_c = R r_f (0 on fixed coarse DOFs); x_c = W D^-1 b_c when x is given.
FZ_STEP void fz_restrict(const FzLevel& fl, const FzLevel& cl, double* b, double* x) {
  const int nd = (int)cl.L.ndof();
  const __amdgpu_buffer_rsrc_t rf = make_rsrc(fl.r, (size_t)fl.L.ndof() * sizeof(double));
  for (int t = threadIdx.x; t < nd; t += FZ_T) {
    const int node = t / 3, c = t - 3 * node;
    int I, J, K;
    node_ijk(node, cl.L, I, J, K);
    const double bv = ((cl.mask[node] >> c) & 1) ? 0.0 : restrict_at<double>(fl.L, rf, I, J, K, c);
    b[t] = bv;
    if (x) x[t] = cl.wD[t] * bv;
  }
  __syncthreads();
}

// x_f += P x_c on the free fine DOFs, two nodes per thread and pass (their
// gathers issued before the updates).
FZ_STEP void fz_prolong_add(const FzLevel& fl, const FzLevel& cl) {
  constexpr int U = 2;
  const __amdgpu_buffer_rsrc_t re = make_rsrc(cl.x, (size_t)cl.L.ndof() * sizeof(double));
  const int nn = (int)fl.L.nn();
  for (int t0 = threadIdx.x; t0 < nn; t0 += U * FZ_T) {
    double pe[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * FZ_T;
      int i, j, k;
      node_ijk(t < nn ? t : 0, fl.L, i, j, k);
      prolong_at<double>(cl.L, re, i, j, k, t < nn, pe[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * FZ_T;
      if (t >= nn) break;
      const int m = fl.mask[t];
      for (int c = 0; c < 3; ++c)
        if (!((m >> c) & 1)) fl.x[3 * t + c] += pe[u][c];
    }
  }
  __syncthreads();
}

// x = A_c^-1 b (b in LDS): a wave takes 8 rows at a time, the lanes split
// the columns, and all of a lane's loads for the 8 rows (columns lane,
// lane + 64, ...) are issued before the sums (past the row: offsets out of
// range read 0).
FZ_STEP void fz_coarse(const FzDesc& d, const FzLevel& cl, const double* sbc) {
  constexpr int RB = 8, CB = FZ_MAX_COARSE / 64;
  const int nd = (int)cl.L.ndof();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const __amdgpu_buffer_rsrc_t ra = make_rsrc(d.Ainv, (size_t)d.ld * d.ld * sizeof(double));
  const int ncb = (nd + 63) / 64;
  for (int r0 = wid * RB; r0 < nd; r0 += FZ_W * RB) {
    double s[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) s[q] = 0.0;
    for (int cb = 0; cb < ncb; cb += 4) {
      double a[4][RB], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = (cb + u) * 64 + lane;
        const bool okc = c < nd;
        bv[u] = okc ? sbc[c] : 0.0;
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const int row = r0 + q;
          const int off = (okc && row < nd) ? (row * d.ld + c) * (int)sizeof(double) : kBufOOB;
          a[u][q] = bload<double>(ra, off, 0);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < RB; ++q) s[q] = fma(a[u][q], bv[u], s[q]);
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const double t = wave_sum(s[q]);
      if (lane == 0 && r0 + q < nd) cl.x[r0 + q] = t;
    }
  }
  (void)CB;
  __syncthreads();
}

// x += W D^-1 (b - A x) over a level's DOFs; A x in t (coarse) or in the
// LDS node sums acc (fine)
FZ_STEP void fz_jacobi_update(const FzLevel& lv, const double* b, const double* t, bool fine,
                              const double* acc) {
  fz_jac((int)lv.L.ndof(), lv.wD, b, fine ? acc : t, lv.mask, fine, lv.x);
  __syncthreads();
}

// z = M r (Algorithm 1, V-cycle from a zero guess) into lv[0].x; r: the
// level-0 residual (zero on fixed DOFs).
FZ_STEP void fz_vcycle(const FzDesc& d, const double* r, double* acc, double* sbc) {
  const int L = d.nlev;
  const FzLevel& l0 = d.lv[0];
  {
    const int nd = (int)l0.L.ndof();
    fz_scale(nd, l0.wD, r, l0.x);
    __syncthreads();
    for (int s = 1; s < d.pre; ++s) {
      fz_mf_apply(d, l0.x, acc);
      fz_jacobi_update(l0, r, nullptr, true, acc);
    }
    fz_mf_apply(d, l0.x, acc);
    fz_res0(nd, r, acc, l0.mask, l0.r);
    __syncthreads();
  }
  for (int l = 1; l < L; ++l) {
    const FzLevel& fl = d.lv[l - 1];
    const FzLevel& cl = d.lv[l];
    if (l == L - 1) {
      fz_restrict(fl, cl, sbc, nullptr);
      fz_coarse(d, cl, sbc);
      break;
    }
    fz_restrict(fl, cl, cl.b, cl.x);
    for (int s = 1; s < d.pre; ++s) {
      fz_st_apply(cl, cl.x, nullptr, cl.r, acc);
      fz_jacobi_update(cl, cl.b, cl.r, false, nullptr);
    }
    fz_st_apply(cl, cl.x, cl.b, cl.r, acc);
  }
  for (int l = L - 2; l >= 0; --l) {
    const FzLevel& fl = d.lv[l];
    fz_prolong_add(fl, d.lv[l + 1]);
    for (int s = 0; s < d.post; ++s) {
      if (l == 0) {
        fz_mf_apply(d, fl.x, acc);
        fz_jacobi_update(fl, r, nullptr, true, acc);
      } else {
        fz_st_apply(fl, fl.x, nullptr, fl.r, acc);
        fz_jacobi_update(fl, fl.b, fl.r, false, nullptr);
      }
    }
  }
}

__global__ __launch_bounds__(FZ_T) void k_fused_pcg(const FzDesc* __restrict__ descs) {
  __shared__ double acc[3 * FZ_MAX_NODES];
  __shared__ double sbc[FZ_MAX_COARSE];
  __shared__ double sh[FZ_W];
  // the descriptor in LDS: read there, it cannot alias the vectors written
  __shared__ FzDesc sd;
  {
    const int* src = reinterpret_cast<const int*>(descs + blockIdx.x);
    int* dst = reinterpret_cast<int*>(&sd);
    for (int t = threadIdx.x; t < (int)(sizeof(FzDesc) / sizeof(int)); t += FZ_T) dst[t] = src[t];
    __syncthreads();
  }
  const FzDesc& d = sd;
  const int nd = (int)d.lv[0].L.ndof();
  const uint8_t* mask = d.lv[0].mask;
  double* x = d.x;
  double* r = d.r;
  double* p = d.p;
  const double* f = d.f;
  const double* z = d.lv[0].x;
  // true residual r = f - A x into r; returns ||r||^2
  auto true_residual = [&]() {
    fz_mf_apply(d, x, acc);
    return fz_sum(fz_true_res(nd, f, acc, mask, r), sh);
  };
  const double ff = fz_sum(fz_dot(nd, f, f), sh);
  const double tol2 = d.tol2 * ff;
  double rr = true_residual();
  if (d.scale_warm) {
    // x <- a x with a = f.x / x.K x, x.K x = x.(f - r)
    double s0 = 0.0, s1 = 0.0;
    for (int t = threadIdx.x; t < nd; t += FZ_T) {
      s0 = fma(f[t], x[t], s0);
      s1 = fma(x[t], f[t] - r[t], s1);
    }
    const double fx = fz_sum(s0, sh), xkx = fz_sum(s1, sh);
    if (xkx > 0.0 && isfinite(fx / xkx)) {
      const double a = fx / xkx;
      double s = 0.0;
      for (int t = threadIdx.x; t < nd; t += FZ_T) {
        x[t] *= a;
        const double v = (1.0 - a) * f[t] + a * r[t];
        r[t] = v;
        s = fma(v, v, s);
      }
      rr = fz_sum(s, sh);
    }
  }
  int state = CG_ACTIVE, it = 0, repl = 0, stall = 0;
  double rr_best = rr;
  if (!(rr <= tol2)) {
    fz_vcycle(d, r, acc, sbc);
    fz_pz(nd, 0.0, z, p);
    double rz = fz_sum(fz_dot(nd, r, z), sh);
    bool restart = false;
    while (true) {
      if (it >= d.maxit) {
        state = CG_MAXIT;
        break;
      }
      fz_mf_apply(d, p, acc);
      const double pq = fz_sum(fz_dot_acc(nd, p, acc, mask), sh);
      if (!(pq > 0.0) || !isfinite(rz)) {
        state = CG_BREAKDOWN;
        break;
      }
      const double alpha = rz / pq;
      rr = fz_sum(fz_xr(nd, alpha, p, acc, mask, x, r), sh);
      ++it;
      if (!isfinite(rr)) {
        state = CG_BREAKDOWN;
        break;
      }
      if (rr <= tol2) {
        const double rt = true_residual();
        if (rt <= tol2) {
          rr = rt;
          state = CG_DONE;
          break;
        }
        ++repl;
        restart = true;
        if (rt < 0.81 * rr_best) {
          rr_best = rt;
          stall = 0;
        } else if (++stall >= 3) {
          rr = rt;
          state = CG_MAXIT;
          break;
        }
        rr = rt;
      }
      fz_vcycle(d, r, acc, sbc);
      const double rzn = fz_sum(fz_dot(nd, r, z), sh);
      const double beta = restart ? 0.0 : rzn / rz;
      restart = false;
      fz_pz(nd, beta, z, p);
      __syncthreads();
      rz = rzn;
    }
  } else {
    state = CG_DONE;
  }
  if (threadIdx.x == 0) {
    CgScalars& c = *d.cs;
    c.ff = ff;
    c.tol2 = tol2;
    c.rr = rr;
    c.iters = it;
    c.state = state;
    c.replacements = repl;
  }
}

void fused_solve(const FzDesc* descs, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fused_pcg, dim3(n), dim3(FZ_T), 0, st, descs);
  MGCG_HIP(hipGetLastError());
}

// One workgroup per problem, one 32-bit word per thread.
__global__ void k_fz_gather(const FzGatherSrc* src, int n, FzRecord* out) {
  const FzGatherSrc g = src[blockIdx.x];
  const int nw = g.nrhs * (int)(sizeof(CgScalars) / sizeof(int));
  int* o = reinterpret_cast<int*>(out[blockIdx.x].cs);
  const int* c = reinterpret_cast<const int*>(g.cs);
  for (int t = threadIdx.x; t < nw; t += blockDim.x) o[t] = c[t];
  if (threadIdx.x < 4) out[blockIdx.x].bad[threadIdx.x] = g.bad[threadIdx.x];
}

void fused_gather(const FzGatherSrc* src, int n, FzRecord* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fz_gather, dim3(n), dim3(64), 0, st, src, n, out);
  MGCG_HIP(hipGetLastError());
}

}  // namespace mgcg
