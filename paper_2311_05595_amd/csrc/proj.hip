// Projection of design variables onto densities (Sec. 3.2 eq. (5)) with the
// weights of the density filter (Sec. 2.2 eq. (4)), and its transpose (the
// chain rule of Sec. 3.4).
//
// Both directions are gathers, so every output is a fixed-order sum (no
// atomics): a thread per density cell for rho = W x, a thread per design cell
// for W^T g.  The Gaussian weight is separable, exp(-c M) = e(m_x) e(m_y)
// e(m_z) with e(m) = exp(-c m^2) and c = 9 / (8 n^2 d^2 rmin^2) (M the integer
// squared centre offset in units of 1/(2nd)); the ball's cut-off is not, so
// the loops walk the candidate rows (z, y) and test the integer M of every
// candidate against (2 n d rmin)^2.  e(|m|) comes from a table computed once
// on the host.  The normalisation 1/(2 pi rmin/3) of eq. (4) cancels in
// omega_ij / omega_i and is left out.
#include <algorithm>
#include <cmath>
#include <array>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "proj.h"

namespace mgcg {

namespace {

struct ProjArgs {
  int nr[3];  // density lattice (x, y, z)
  int nx[3];  // design lattice
  int n, d;
  int kd;     // design cells searched on either side of a density centre's cell
  int kr;     // density cells searched on either side of a design centre's cell
  double R2;  // (2 n d rmin)^2
  const double* tab;  // e(|m|), |m| = 0 .. ntab - 1
};

constexpr int PROJ_BS = 256;

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }

// rho_i = (1/omega_i) sum_j omega_ij x_j, or, with NORM, 1/omega_i itself.
template <bool NORM>
__global__ __launch_bounds__(PROJ_BS) void k_proj_fwd(ProjArgs a, const double* __restrict__ x,
                                                       const double* __restrict__ invw,
                                                       double* __restrict__ out) {
  const long nrho = (long)a.nr[0] * a.nr[1] * a.nr[2];
  const long i = (long)blockIdx.x * PROJ_BS + threadIdx.x;
  if (i >= nrho) return;
  const int ix = (int)(i % a.nr[0]);
  const long t = i / a.nr[0];
  const int iy = (int)(t % a.nr[1]);
  const int iz = (int)(t / a.nr[1]);
  const int two_n = 2 * a.n;
  // the design cell holding the density centre, per axis; m(j) = A - 2n j
  const int cx = ((2 * ix + 1) * a.d) / two_n, cy = ((2 * iy + 1) * a.d) / two_n,
            cz = ((2 * iz + 1) * a.d) / two_n;
  const int Ax = (2 * ix + 1) * a.d - a.n, Ay = (2 * iy + 1) * a.d - a.n,
            Az = (2 * iz + 1) * a.d - a.n;
  const int xlo = max(cx - a.kd, 0), xhi = min(cx + a.kd, a.nx[0] - 1);
  const int ylo = max(cy - a.kd, 0), yhi = min(cy + a.kd, a.nx[1] - 1);
  const int zlo = max(cz - a.kd, 0), zhi = min(cz + a.kd, a.nx[2] - 1);
  double acc = 0.0;
  for (int jz = zlo; jz <= zhi; ++jz) {
    const int mz = Az - two_n * jz;
    const int sz = mz * mz;
    if ((double)sz > a.R2) continue;
    const double ez = a.tab[iabs(mz)];
    for (int jy = ylo; jy <= yhi; ++jy) {
      const int my = Ay - two_n * jy;
      const int syz = sz + my * my;
      if ((double)syz > a.R2) continue;
      const double eyz = ez * a.tab[iabs(my)];
      const double* xr = x + ((long)jz * a.nx[1] + jy) * a.nx[0];
      for (int jx = xlo; jx <= xhi; ++jx) {
        const int mx = Ax - two_n * jx;
        if ((double)(syz + mx * mx) > a.R2) continue;
        const double w = a.tab[iabs(mx)] * eyz;
        if constexpr (NORM)
          acc += w;
        else
          acc = fma(w, xr[jx], acc);
      }
    }
  }
  out[i] = NORM ? 1.0 / acc : acc * invw[i];
}

// (W^T g)_k = sum_i omega_ik (g_i / omega_i) over the density cells whose
// ball holds design cell k (the same integer test, the pair's m unchanged).
__global__ __launch_bounds__(PROJ_BS) void k_proj_t(ProjArgs a, const double* __restrict__ g,
                                                     const double* __restrict__ invw,
                                                     double* __restrict__ out) {
  const long nx = (long)a.nx[0] * a.nx[1] * a.nx[2];
  const long k = (long)blockIdx.x * PROJ_BS + threadIdx.x;
  if (k >= nx) return;
  const int kx = (int)(k % a.nx[0]);
  const long t = k / a.nx[0];
  const int ky = (int)(t % a.nx[1]);
  const int kz = (int)(t / a.nx[1]);
  const int two_d = 2 * a.d;
  // the density cell holding the design centre, per axis; m(i) = B + 2d i
  const int cx = ((2 * kx + 1) * a.n) / two_d, cy = ((2 * ky + 1) * a.n) / two_d,
            cz = ((2 * kz + 1) * a.n) / two_d;
  const int Bx = a.d - (2 * kx + 1) * a.n, By = a.d - (2 * ky + 1) * a.n,
            Bz = a.d - (2 * kz + 1) * a.n;
  const int xlo = max(cx - a.kr, 0), xhi = min(cx + a.kr, a.nr[0] - 1);
  const int ylo = max(cy - a.kr, 0), yhi = min(cy + a.kr, a.nr[1] - 1);
  const int zlo = max(cz - a.kr, 0), zhi = min(cz + a.kr, a.nr[2] - 1);
  double acc = 0.0;
  for (int iz = zlo; iz <= zhi; ++iz) {
    const int mz = Bz + two_d * iz;
    const int sz = mz * mz;
    if ((double)sz > a.R2) continue;
    const double ez = a.tab[iabs(mz)];
    for (int iy = ylo; iy <= yhi; ++iy) {
      const int my = By + two_d * iy;
      const int syz = sz + my * my;
      if ((double)syz > a.R2) continue;
      const double eyz = ez * a.tab[iabs(my)];
      const long row = ((long)iz * a.nr[1] + iy) * a.nr[0];
      for (int ix = xlo; ix <= xhi; ++ix) {
        const int mx = Bx + two_d * ix;
        if ((double)(syz + mx * mx) > a.R2) continue;
        const double w = a.tab[iabs(mx)] * eyz;
        acc = fma(w, g[row + ix] * invw[row + ix], acc);
      }
    }
  }
  out[k] = acc;
}

// ---- tiled kernels: n a multiple of d (q = n / d), the halo within 4 cells
//
// Density cell i = q j + p (per axis, p < q) has the design cell j under its
// centre, and the squared centre offsets to design cell j + o depend on p and
// o only: m = (2p + 1) d - n - 2 n o.  So each of the q^3 phases p has one
// stencil S_p, a list of (offset o, weight) shared by every cell of that
// phase.  Blocks stage a tile of the design lattice with an h-cell halo in
// LDS and gather from tables whose entries hold an LDS offset and G weights,
// one per output accumulated from that offset (zero where an output's
// stencil misses it):
// * forward: a thread owns PF_Z design cells along z and, for each, G
//   phases' densities at a time, the table the union of their stencils; one
//   entry feeds PF_Z LDS reads and PF_Z * G fused multiply-adds;
// * transpose: design cell k collects g_i / omega_i over the density cells
//   i = q (k - o) + p from the mirrored stencils, one phase's sub-lattice
//   staged at a time (its loads issued before the barrier that frees the
//   region).
// Table entries are read with wave-uniform indices (scalar loads) a batch
// ahead, so the wait for a batch's LDS reads does not also wait for them.
constexpr int PT_X = 8, PT_Y = 8, PT_Z = 4;  // threads of a block per axis
static_assert(PT_X * PT_Y * PT_Z == PROJ_BS, "one thread per tile column");
constexpr int PF_Z = 2;  // design cells per forward thread along z

struct ProjTileArgs {
  int nr[3], nx[3];
  int q, np, h;
  int S[3];          // staged region per axis: tile + 2h
  int P0;            // LDS row pitch of the region (>= S[0], = 8 mod 16)
  int ntile[3];      // tiles per axis
};

// LDS row pitch of a region S0 cells wide: 8 (mod 16) doubles, so that the
// two 8-lane rows of a 16-lane group of a wave land on disjoint halves of
// the 32 four-byte banks.
constexpr int lds_pitch(int S0) { return S0 <= 8 ? 8 : ((S0 + 7) / 16) * 16 + 8; }

__device__ __forceinline__ void tile_origin(const ProjTileArgs& a, int& bx, int& by, int& bz) {
  const int b = blockIdx.x;
  bx = b % a.ntile[0];
  by = (b / a.ntile[0]) % a.ntile[1];
  bz = b / (a.ntile[0] * a.ntile[1]);
}

template <int G>
struct PtBatch {
  static constexpr int value = G == 1 ? 8 : 4;
};

// One table entry read as whole 16-byte words (contiguous, so that the
// loads of a batch merge into wide scalar loads).
template <int G>
__device__ __forceinline__ ProjEntryG<G> load_entry(const ProjEntryG<G>* p) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  constexpr int NV = sizeof(ProjEntryG<G>) / 16;
  union {
    ProjEntryG<G> e;
    d2 v[NV];
  } u;
  const d2* s = reinterpret_cast<const d2*>(p);
#pragma unroll
  for (int i = 0; i < NV; ++i) u.v[i] = s[i];
  return u.e;
}

// acc[b][c] += sum_e w_e[c] * sh[base[b] + SIGN * rel_e] over the entries
// [e0, e1) (a multiple of the batch size, zero-weight padded).
template <int SIGN, int G, int NB>
__device__ __forceinline__ void grouped_gather(const ProjEntryG<G>* __restrict__ ent, int e0, int e1,
                                               const double* sh, const int (&base)[NB],
                                               double (&acc)[NB][G]) {
  constexpr int B = PtBatch<G>::value;
  e0 = __builtin_amdgcn_readfirstlane(e0);
  e1 = __builtin_amdgcn_readfirstlane(e1);
  if (e0 >= e1) return;
  ProjEntryG<G> cur[B];
#pragma unroll
  for (int k = 0; k < B; ++k) cur[k] = load_entry(ent + e0 + k);
  for (int e = e0; e < e1; e += B) {
    ProjEntryG<G> nxt[B];
    const int en = e + B < e1 ? e + B : e;
#pragma unroll
    for (int k = 0; k < B; ++k) nxt[k] = load_entry(ent + en + k);
    double xv[B][NB];
#pragma unroll
    for (int k = 0; k < B; ++k)
#pragma unroll
      for (int b = 0; b < NB; ++b) xv[k][b] = sh[base[b] + SIGN * cur[k].rel];
    // the next batch's entries are needed here: their loads are issued
    // before this batch's arithmetic and share its wait
#pragma unroll
    for (int k = 0; k < B; ++k) {
      asm volatile("" : : "s"(nxt[k].rel));
#pragma unroll
      for (int c = 0; c < G; ++c) asm volatile("" : : "s"(nxt[k].w[c]));
    }
#pragma unroll
    for (int k = 0; k < B; ++k)
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < G; ++c) acc[b][c] = fma(cur[k].w[c], xv[k][b], acc[b][c]);
#pragma unroll
    for (int k = 0; k < B; ++k) cur[k] = nxt[k];
  }
}

// Staging of the block's region (S[0] x S[1] x S[2] cells of the design
// lattice from (rx, ry, rz)): values of design cells x_j (TRANS false) or,
// for phase (px, py, pz), g_i / omega_i at the density cells i = q j + p
// (TRANS true); 0 outside the domain.  stage_load issues the loads of cells
// p0 + threadIdx.x + u * PROJ_BS (u < PT_STAGE) into registers, branch-free
// (cells outside the region or the domain load entry 0 and are masked), and
// stage_store writes them to LDS.
constexpr int PT_STAGE = 12;
template <bool TRANS>
__device__ __forceinline__ void stage_load(const ProjTileArgs& a, int p0, int rx, int ry, int rz,
                                           int px, int py, int pz, const double* __restrict__ src,
                                           const double* __restrict__ invw,
                                           double (&v)[PT_STAGE]) {
  const int nreg = a.S[0] * a.S[1] * a.S[2];
#pragma unroll
  for (int u = 0; u < PT_STAGE; ++u) {
    const int idx = p0 + (int)threadIdx.x + u * PROJ_BS;
    const int vx = idx % a.S[0], vy = (idx / a.S[0]) % a.S[1], vz = idx / (a.S[0] * a.S[1]);
    const int jx = rx + vx, jy = ry + vy, jz = rz + vz;
    const bool in = idx < nreg && (unsigned)jx < (unsigned)a.nx[0] &&
                    (unsigned)jy < (unsigned)a.nx[1] && (unsigned)jz < (unsigned)a.nx[2];
    if constexpr (TRANS) {
      const long i = in ? (long)(a.q * jx + px) +
                              (long)a.nr[0] * ((long)(a.q * jy + py) + (long)a.nr[1] * (a.q * jz + pz))
                        : 0L;
      const double gv = src[i], wv = invw[i];
      v[u] = in ? gv * wv : 0.0;
    } else {
      const long j = in ? jx + (long)a.nx[0] * (jy + (long)a.nx[1] * jz) : 0L;
      const double xv = src[j];
      v[u] = in ? xv : 0.0;
    }
  }
}
__device__ __forceinline__ int lds_index(const ProjTileArgs& a, int idx) {
  const int vx = idx % a.S[0], r = idx / a.S[0];
  return vx + a.P0 * r;  // r = vy + S[1] vz: rows of the region
}
__device__ __forceinline__ void stage_store(const ProjTileArgs& a, int p0, const double (&v)[PT_STAGE],
                                            double* sh) {
  const int nreg = a.S[0] * a.S[1] * a.S[2];
#pragma unroll
  for (int u = 0; u < PT_STAGE; ++u) {
    const int idx = p0 + (int)threadIdx.x + u * PROJ_BS;
    if (idx < nreg) sh[lds_index(a, idx)] = v[u];
  }
}

// (the tables are separate no-alias parameters: the compiler then reads them
// through the scalar cache, which it may not do for memory the kernel's
// stores might alias)
template <int G>
__global__ __launch_bounds__(PROJ_BS) void k_proj_fwd_tile(ProjTileArgs a,
                                                            const ProjEntryG<G>* __restrict__ ent,
                                                            const int* __restrict__ start,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ invw,
                                                            double* __restrict__ out) {
  extern __shared__ double sh[];
  int bx, by, bz;
  tile_origin(a, bx, by, bz);
  const int t = threadIdx.x;
  const int rx = bx * PT_X - a.h, ry = by * PT_Y - a.h, rz = bz * PT_Z * PF_Z - a.h;
  const int nreg = a.S[0] * a.S[1] * a.S[2];
  for (int p0 = 0; p0 < nreg; p0 += PT_STAGE * PROJ_BS) {
    double v[PT_STAGE];
    stage_load<false>(a, p0, rx, ry, rz, 0, 0, 0, x, nullptr, v);
    stage_store(a, p0, v, sh);
  }
  __syncthreads();
  const int lx = t % PT_X, ly = (t / PT_X) % PT_Y, lz = t / (PT_X * PT_Y);
  const int jx = bx * PT_X + lx, jy = by * PT_Y + ly;
  int jz[PF_Z], base[PF_Z];
  bool on[PF_Z];
#pragma unroll
  for (int b = 0; b < PF_Z; ++b) {
    const int zl = PF_Z * lz + b;
    jz[b] = bz * PT_Z * PF_Z + zl;
    on[b] = jx < a.nx[0] && jy < a.nx[1] && jz[b] < a.nx[2];
    base[b] = (lx + a.h) + a.P0 * ((ly + a.h) + a.S[1] * (zl + a.h));
  }
  for (int p0 = 0; p0 < a.np; p0 += G) {
    double acc[PF_Z][G];
#pragma unroll
    for (int b = 0; b < PF_Z; ++b)
#pragma unroll
      for (int c = 0; c < G; ++c) acc[b][c] = 0.0;
    grouped_gather<1, G, PF_Z>(ent, start[p0 / G], start[p0 / G + 1], sh, base, acc);
    // the group's 1/omega loads together, then its stores
    long idx[PF_Z][G];
    double w[PF_Z][G];
#pragma unroll
    for (int b = 0; b < PF_Z; ++b)
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const int p = p0 + c;
        const int px = p % a.q, py = (p / a.q) % a.q, pz = p / (a.q * a.q);
        idx[b][c] = on[b] ? (long)(a.q * jx + px) +
                                (long)a.nr[0] *
                                    ((long)(a.q * jy + py) + (long)a.nr[1] * (a.q * jz[b] + pz))
                          : 0L;
        w[b][c] = invw[idx[b][c]];
      }
#pragma unroll
    for (int b = 0; b < PF_Z; ++b)
      if (on[b]) {
#pragma unroll
        for (int c = 0; c < G; ++c) out[idx[b][c]] = acc[b][c] * w[b][c];
      }
  }
}

// Transpose: a thread owns PT_ZT design cells along z (each table entry then
// serves PT_ZT LDS reads).  The region's cells of this thread (cells
// threadIdx.x + u * PROJ_BS, one staging pass) are decomposed once; for phase
// p the density cell of region cell (vx, vy, vz) is cell0 + px + nr0 (py +
// nr1 pz) with cell0 = q (rx + vx) + nr0 (q (ry + vy) + nr1 q (rz + vz)).
constexpr int PT_ZT = 2;
constexpr int PT_STAGE_T = 16;  // region cells per thread: (8 + 2h)^2 (8 + 2h) <= 4096, h <= 4
__global__ __launch_bounds__(PROJ_BS) void k_proj_t_tile(ProjTileArgs a,
                                                          const ProjEntryG<1>* __restrict__ ent,
                                                          const int* __restrict__ start,
                                                          const double* __restrict__ g,
                                                          const double* __restrict__ invw,
                                                          double* __restrict__ out) {
  extern __shared__ double sh[];
  int bx, by, bz;
  tile_origin(a, bx, by, bz);
  const int t = threadIdx.x;
  const int rx = bx * PT_X - a.h, ry = by * PT_Y - a.h, rz = bz * PT_Z * PT_ZT - a.h;
  const int lx = t % PT_X, ly = (t / PT_X) % PT_Y, lz = t / (PT_X * PT_Y);
  const int kx = bx * PT_X + lx, ky = by * PT_Y + ly;
  const int nreg = a.S[0] * a.S[1] * a.S[2];
  int base[PT_ZT];
#pragma unroll
  for (int b = 0; b < PT_ZT; ++b)
    base[b] = (lx + a.h) + a.P0 * ((ly + a.h) + a.S[1] * (PT_ZT * lz + b + a.h));
  long cell0[PT_STAGE_T];
  int slot[PT_STAGE_T];
  unsigned inmask = 0;
#pragma unroll
  for (int u = 0; u < PT_STAGE_T; ++u) {
    const int idx = t + u * PROJ_BS;
    const int vx = idx % a.S[0], vy = (idx / a.S[0]) % a.S[1], vz = idx / (a.S[0] * a.S[1]);
    const int jx = rx + vx, jy = ry + vy, jz = rz + vz;
    const bool in = idx < nreg && (unsigned)jx < (unsigned)a.nx[0] &&
                    (unsigned)jy < (unsigned)a.nx[1] && (unsigned)jz < (unsigned)a.nx[2];
    cell0[u] = in ? (long)(a.q * jx) + (long)a.nr[0] * ((long)(a.q * jy) + (long)a.nr[1] * (a.q * jz))
                  : 0L;
    inmask |= in ? 1u << u : 0u;
    slot[u] = idx < nreg ? lds_index(a, idx) : -1;
  }
  double acc[PT_ZT][1];
#pragma unroll
  for (int b = 0; b < PT_ZT; ++b) acc[b][0] = 0.0;
  for (int p = 0; p < a.np; ++p) {
    const int px = p % a.q, py = (p / a.q) % a.q, pz = p / (a.q * a.q);
    const long poff = px + (long)a.nr[0] * (py + (long)a.nr[1] * pz);
    double v[PT_STAGE_T];
#pragma unroll
    for (int u = 0; u < PT_STAGE_T; ++u) {
      const bool in = (inmask >> u) & 1u;
      const long i = in ? cell0[u] + poff : 0L;
      const double gv = g[i], wv = invw[i];
      v[u] = in ? gv * wv : 0.0;
    }
    __syncthreads();  // the previous phase's reads are done
#pragma unroll
    for (int u = 0; u < PT_STAGE_T; ++u)
      if (slot[u] >= 0) sh[slot[u]] = v[u];
    __syncthreads();
    grouped_gather<-1, 1, PT_ZT>(ent, start[p], start[p + 1], sh, base, acc);
  }
#pragma unroll
  for (int b = 0; b < PT_ZT; ++b) {
    const int kz = bz * PT_Z * PT_ZT + PT_ZT * lz + b;
    if (kx < a.nx[0] && ky < a.nx[1] && kz < a.nx[2])
      out[kx + (long)a.nx[0] * (ky + (long)a.nx[1] * kz)] = acc[b][0];
  }
}

// Largest per-axis squared offset from a density centre to its nearest
// design centre over the axis (the ball of a cell is empty exactly when the
// three axes' nearest offsets already exceed the radius).
long worst_nearest(int ncr, int ncx, int n, int d) {
  long worst = 0;
  for (int i = 0; i < ncr; ++i) {
    long best = -1;
    const int c = ((2 * i + 1) * d) / (2 * n);
    for (int j = std::max(c - 1, 0); j <= std::min(c + 1, ncx - 1); ++j) {
      const long m = (long)(2 * i + 1) * d - (long)(2 * j + 1) * n;
      if (best < 0 || m * m < best) best = m * m;
    }
    worst = std::max(worst, best);
  }
  return worst;
}

}  // namespace

ProjGeom Proj::geometry(const mgcg_proj_desc& d) {
  if (d.nelx < 1 || d.nely < 1 || d.nelz < 1) throw Error(MGCG_EINVAL, "element counts must be >= 1");
  if (d.nsub < 1 || d.nsub > 64 || d.ndes < 1 || d.ndes > 64)
    throw Error(MGCG_EINVAL, "nsub and ndes must lie in 1..64");
  if (!(d.rmin > 0.0) || !std::isfinite(d.rmin)) throw Error(MGCG_EINVAL, "rmin must be positive");
  const double R = 2.0 * d.nsub * d.ndes * d.rmin;
  if (R > 4096.0) throw Error(MGCG_EINVAL, "rmin too large (2 n d rmin > 4096)");
  ProjGeom g;
  const int ne[3] = {d.nelx, d.nely, d.nelz};
  long nr = 1, nx = 1;
  for (int a = 0; a < 3; ++a) {
    const long lr = (long)ne[a] * d.nsub, lx = (long)ne[a] * d.ndes;
    // (2 i + 1) d stays far inside 32-bit integers
    if (lr > (1L << 20) || lx > (1L << 20)) throw Error(MGCG_EINVAL, "lattice axis above 2^20 cells");
    g.nr[a] = (int)lr;
    g.nx[a] = (int)lx;
    nr *= lr;
    nx *= lx;
  }
  if (nr > 0x7FFFFFFFL || nx > 0x7FFFFFFFL) throw Error(MGCG_EINVAL, "lattice above 2^31 - 1 cells");
  g.n = d.nsub;
  g.d = d.ndes;
  g.R2 = R * R;
  // every member has |m| <= 2ndr, i.e. its centre within d*rmin + 1/2 cells
  g.kd = (int)std::floor(d.ndes * d.rmin + 0.5) + 1;
  g.kr = (int)std::floor(d.nsub * d.rmin + 0.5) + 1;
  g.ntab = (int)std::floor(R) + 2;
  g.nrho = nr;
  g.nxv = nx;
  long worst = 0;
  for (int a = 0; a < 3; ++a) worst += worst_nearest(g.nr[a], g.nx[a], g.n, g.d);
  if ((double)worst > g.R2)
    throw Error(MGCG_EINVAL, "rmin leaves density cells without a design cell in their ball");
  const double c = 9.0 / (8.0 * (double)g.n * g.n * g.d * g.d * d.rmin * d.rmin);
  g.tab.resize(g.ntab);
  for (int m = 0; m < g.ntab; ++m) g.tab[m] = std::exp(-c * (double)m * (double)m);
  phase_tables(g);
  return g;
}

// The gather tables of the tiled kernels (left empty, q = 0, when d does not
// divide n, the phases are too many or a stencil reaches past 4 cells).
template <int G>
static void pad_batch(std::vector<ProjEntryG<G>>& v) {
  while (v.size() % PtBatch<G>::value) v.push_back(ProjEntryG<G>{});
}

void Proj::phase_tables(ProjGeom& g) {
  g.q = g.np = g.h = g.gf = 0;
  g.fwd1.clear();
  g.fwd4.clear();
  g.trg.clear();
  g.start_f.clear();
  g.start_t.clear();
  if (g.n % g.d != 0) return;
  const int q = g.n / g.d;
  if (q > 8) return;
  const int np = q * q * q;
  // stencil of each phase: offset (ordered z, y, x) -> weight
  using Key = std::array<int, 3>;  // (oz, oy, ox)
  std::vector<std::map<Key, double>> S(np);
  int h = 0;
  long total = 0;
  for (int p = 0; p < np; ++p) {
    const int pp[3] = {p % q, (p / q) % q, p / (q * q)};
    int m0[3];
    for (int a = 0; a < 3; ++a) m0[a] = (2 * pp[a] + 1) * g.d - g.n;  // m at o = 0
    for (int oz = -g.kd; oz <= g.kd; ++oz)
      for (int oy = -g.kd; oy <= g.kd; ++oy)
        for (int ox = -g.kd; ox <= g.kd; ++ox) {
          const long mx = m0[0] - 2L * g.n * ox, my = m0[1] - 2L * g.n * oy,
                     mz = m0[2] - 2L * g.n * oz;
          if ((double)(mx * mx + my * my + mz * mz) > g.R2) continue;
          // the generic kernels' product order: (e(mz) e(my)) e(mx)
          S[p][Key{oz, oy, ox}] =
              g.tab[std::labs(mx)] * (g.tab[std::labs(mz)] * g.tab[std::labs(my)]);
          h = std::max({h, std::abs(ox), std::abs(oy), std::abs(oz)});
        }
    total += (long)S[p].size();
  }
  if (h > 4 || total > 65536) return;
  g.q = q;
  g.np = np;
  g.h = h;
  g.gf = np % 4 == 0 ? 4 : 1;
  // forward: groups of gf consecutive phases, the union of their stencils
  const int SXf = lds_pitch(PT_X + 2 * h), SYf = PT_Y + 2 * h;
  g.start_f.push_back(0);
  for (int p0 = 0; p0 < np; p0 += g.gf) {
    std::set<Key> U;
    for (int c = 0; c < g.gf; ++c)
      for (const auto& kv : S[p0 + c]) U.insert(kv.first);
    for (const Key& u : U) {
      const int rel = u[2] + SXf * (u[1] + SYf * u[0]);
      if (g.gf == 4) {
        ProjEntryG<4> e{};
        for (int c = 0; c < 4; ++c) {
          auto it = S[p0 + c].find(u);
          e.w[c] = it == S[p0 + c].end() ? 0.0 : it->second;
        }
        e.rel = rel;
        g.fwd4.push_back(e);
      } else {
        ProjEntryG<1> e{};
        e.w[0] = S[p0].at(u);
        e.rel = rel;
        g.fwd1.push_back(e);
      }
    }
    if (g.gf == 4) {
      pad_batch(g.fwd4);
      g.start_f.push_back((int)g.fwd4.size());
    } else {
      pad_batch(g.fwd1);
      g.start_f.push_back((int)g.fwd1.size());
    }
  }
  // transpose: per phase, the mirrored stencil (read at k - o)
  const int SXt = lds_pitch(PT_X + 2 * h), SYt = PT_Y + 2 * h;
  g.start_t.push_back(0);
  for (int p = 0; p < np; ++p) {
    for (const auto& kv : S[p]) {
      ProjEntryG<1> e{};
      e.w[0] = kv.second;
      e.rel = kv.first[2] + SXt * (kv.first[1] + SYt * kv.first[0]);
      g.trg.push_back(e);
    }
    pad_batch(g.trg);
    g.start_t.push_back((int)g.trg.size());
  }
}

size_t Proj::device_bytes(const mgcg_proj_desc& d) {
  const ProjGeom g = geometry(d);
  return ((size_t)g.nrho + (size_t)g.ntab) * sizeof(double) + g.table_bytes();
}

Proj::Proj(const mgcg_proj_desc& d, int device) : g_(geometry(d)), device_(device) {
  MGCG_HIP(hipSetDevice(device_));
  (void)d;
  try {
    const size_t fwd_bytes = g_.gf == 4 ? g_.fwd4.size() * sizeof(ProjEntryG<4>)
                                        : g_.fwd1.size() * sizeof(ProjEntryG<1>);
    const size_t tr_bytes = g_.trg.size() * sizeof(ProjEntryG<1>);
    if (hipMalloc(&invw_, (size_t)g_.nrho * sizeof(double)) != hipSuccess ||
        hipMalloc(&tab_, g_.tab.size() * sizeof(double)) != hipSuccess ||
        (g_.q > 0 && (hipMalloc(&fwd_ent_, fwd_bytes) != hipSuccess ||
                      hipMalloc(&tr_ent_, tr_bytes) != hipSuccess ||
                      hipMalloc(&start_f_, g_.start_f.size() * sizeof(int)) != hipSuccess ||
                      hipMalloc(&start_t_, g_.start_t.size() * sizeof(int)) != hipSuccess))) {
      (void)hipGetLastError();
      throw Error(MGCG_ENOMEM, "projection allocation failed");
    }
    MGCG_HIP(hipMemcpyAsync(tab_, g_.tab.data(), g_.tab.size() * sizeof(double),
                            hipMemcpyHostToDevice, stream_));
    if (g_.q > 0) {
      const void* fsrc = g_.gf == 4 ? (const void*)g_.fwd4.data() : (const void*)g_.fwd1.data();
      MGCG_HIP(hipMemcpyAsync(fwd_ent_, fsrc, fwd_bytes, hipMemcpyHostToDevice, stream_));
      MGCG_HIP(hipMemcpyAsync(tr_ent_, g_.trg.data(), tr_bytes, hipMemcpyHostToDevice, stream_));
      MGCG_HIP(hipMemcpyAsync(start_f_, g_.start_f.data(), g_.start_f.size() * sizeof(int),
                              hipMemcpyHostToDevice, stream_));
      MGCG_HIP(hipMemcpyAsync(start_t_, g_.start_t.data(), g_.start_t.size() * sizeof(int),
                              hipMemcpyHostToDevice, stream_));
    }
    launch_norm();
    MGCG_HIP(hipStreamSynchronize(stream_));
  } catch (...) {
    release();
    throw;
  }
}

Proj::~Proj() { release(); }

void Proj::release() {
  (void)hipSetDevice(device_);
  (void)hipStreamSynchronize(stream_);
  if (invw_) (void)hipFree(invw_);
  if (tab_) (void)hipFree(tab_);
  for (void* q : {fwd_ent_, tr_ent_, (void*)start_f_, (void*)start_t_})
    if (q) (void)hipFree(q);
  invw_ = tab_ = nullptr;
  fwd_ent_ = tr_ent_ = nullptr;
  start_f_ = start_t_ = nullptr;
}

void Proj::set_stream(hipStream_t s) {
  MGCG_HIP(hipSetDevice(device_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  stream_ = s;
}

static ProjArgs args_of(const ProjGeom& g, const double* tab) {
  ProjArgs a;
  for (int i = 0; i < 3; ++i) {
    a.nr[i] = g.nr[i];
    a.nx[i] = g.nx[i];
  }
  a.n = g.n;
  a.d = g.d;
  a.kd = g.kd;
  a.kr = g.kr;
  a.R2 = g.R2;
  a.tab = tab;
  return a;
}

void Proj::launch_norm() {
  const int nb = (int)((g_.nrho + PROJ_BS - 1) / PROJ_BS);
  hipLaunchKernelGGL(k_proj_fwd<true>, dim3(nb), dim3(PROJ_BS), 0, stream_, args_of(g_, tab_),
                     (const double*)nullptr, (const double*)nullptr, invw_);
  MGCG_HIP(hipGetLastError());
}

namespace {
// Temporary device copies of host vectors for one call.
struct Staging {
  std::vector<void*> p;
  ~Staging() {
    for (void* q : p) (void)hipFree(q);
  }
  double* get(long n) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)std::max(n, 1L) * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(MGCG_ENOMEM, "projection staging allocation failed");
    }
    p.push_back(q);
    return (double*)q;
  }
};
}  // namespace

void Proj::run(bool transpose, const double* in, double* out, int mem) {
  if (!in || !out) throw Error(MGCG_EINVAL, "null vector");
  if (mem != MGCG_MEM_HOST && mem != MGCG_MEM_DEVICE) throw Error(MGCG_EINVAL, "bad mem flag");
  MGCG_HIP(hipSetDevice(device_));
  const long nin = transpose ? g_.nrho : g_.nxv, nout = transpose ? g_.nxv : g_.nrho;
  Staging st;
  const double* din = in;
  double* dout = out;
  if (mem == MGCG_MEM_HOST) {
    double* a = st.get(nin);
    MGCG_HIP(hipMemcpyAsync(a, in, (size_t)nin * sizeof(double), hipMemcpyHostToDevice, stream_));
    din = a;
    dout = st.get(nout);
  }
  if (g_.q > 0) {
    ProjTileArgs a;
    for (int i = 0; i < 3; ++i) {
      a.nr[i] = g_.nr[i];
      a.nx[i] = g_.nx[i];
    }
    a.q = g_.q;
    a.np = g_.np;
    a.h = g_.h;
    // design cells per block tile: PF_Z (forward) or PT_ZT (transpose) per
    // thread along z
    const int T[3] = {PT_X, PT_Y, PT_Z * (transpose ? PT_ZT : PF_Z)};
    long nb = 1;
    for (int i = 0; i < 3; ++i) {
      a.S[i] = T[i] + 2 * g_.h;
      a.ntile[i] = (g_.nx[i] + T[i] - 1) / T[i];
      nb *= a.ntile[i];
    }
    a.P0 = lds_pitch(a.S[0]);
    const size_t lds = (size_t)a.P0 * a.S[1] * a.S[2] * sizeof(double);
    if (transpose)
      hipLaunchKernelGGL(k_proj_t_tile, dim3((unsigned)nb), dim3(PROJ_BS), lds, stream_, a,
                         (const ProjEntryG<1>*)tr_ent_, (const int*)start_t_, din,
                         (const double*)invw_, dout);
    else if (g_.gf == 4)
      hipLaunchKernelGGL(k_proj_fwd_tile<4>, dim3((unsigned)nb), dim3(PROJ_BS), lds, stream_, a,
                         (const ProjEntryG<4>*)fwd_ent_, (const int*)start_f_, din,
                         (const double*)invw_, dout);
    else
      hipLaunchKernelGGL(k_proj_fwd_tile<1>, dim3((unsigned)nb), dim3(PROJ_BS), lds, stream_, a,
                         (const ProjEntryG<1>*)fwd_ent_, (const int*)start_f_, din,
                         (const double*)invw_, dout);
  } else {
    const int nb = (int)((nout + PROJ_BS - 1) / PROJ_BS);
    if (transpose)
      hipLaunchKernelGGL(k_proj_t, dim3(nb), dim3(PROJ_BS), 0, stream_, args_of(g_, tab_), din,
                         (const double*)invw_, dout);
    else
      hipLaunchKernelGGL(k_proj_fwd<false>, dim3(nb), dim3(PROJ_BS), 0, stream_,
                         args_of(g_, tab_), din, (const double*)invw_, dout);
  }
  MGCG_HIP(hipGetLastError());
  if (mem == MGCG_MEM_HOST) {
    MGCG_HIP(hipMemcpyAsync(out, dout, (size_t)nout * sizeof(double), hipMemcpyDeviceToHost,
                            stream_));
    MGCG_HIP(hipStreamSynchronize(stream_));
  }
}

}  // namespace mgcg
