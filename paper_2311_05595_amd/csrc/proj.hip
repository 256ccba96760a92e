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
#include <cstdlib>
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
// stencil, a list of (offset o, weight) shared by every cell of that phase.
// A block stages an 8 x 8 x 4 tile of design cells with an h-cell halo in LDS
// and each thread, one design cell, gathers the q^3 densities over it from
// the tables, read with wave-uniform indices.  The transpose is the sum over
// phases of the mirrored gather: design cell k collects g_i / omega_i from
// the density cells i = q (k - o) + p, staged phase by phase.
constexpr int PT_X = 8, PT_Y = 8, PT_Z = 4;  // design cells per block (one per thread)
static_assert(PT_X * PT_Y * PT_Z == PROJ_BS, "one design cell per thread");

struct ProjTileArgs {
  int nr[3], nx[3];
  int q, np, h;
  int S[3];          // staged region per axis: tile + 2h
  int ntile[3];      // tiles per axis
};

__device__ __forceinline__ void tile_origin(const ProjTileArgs& a, int& bx, int& by, int& bz) {
  const int b = blockIdx.x;
  bx = b % a.ntile[0];
  by = (b / a.ntile[0]) % a.ntile[1];
  bz = b / (a.ntile[0] * a.ntile[1]);
}

// Sum of w_e * sh[base + sign * rel_e] over the entries [e0, e1) of one phase
// (a multiple of PT_BATCH, zero-weight padded): table entries are read with
// wave-uniform indices (scalar loads) a batch ahead, so the wait for a batch's
// LDS reads does not also wait for its table loads.
constexpr int PT_BATCH = 8;
template <int SIGN>
__device__ __forceinline__ double phase_gather(const ProjEntry* __restrict__ ent, int e0, int e1,
                                               const double* sh, int base) {
  double acc0 = 0.0, acc1 = 0.0;
  e0 = __builtin_amdgcn_readfirstlane(e0);
  e1 = __builtin_amdgcn_readfirstlane(e1);
  if (e0 >= e1) return 0.0;
  ProjEntry cur[PT_BATCH];
#pragma unroll
  for (int k = 0; k < PT_BATCH; ++k) cur[k] = ent[e0 + k];
  for (int e = e0; e < e1; e += PT_BATCH) {
    ProjEntry nxt[PT_BATCH];
    const int en = e + PT_BATCH < e1 ? e + PT_BATCH : e;
#pragma unroll
    for (int k = 0; k < PT_BATCH; ++k) nxt[k] = ent[en + k];
    double xv[PT_BATCH];
#pragma unroll
    for (int k = 0; k < PT_BATCH; ++k) xv[k] = sh[base + SIGN * cur[k].rel];
    // the next batch's entries are needed here: their loads are issued
    // before this batch's arithmetic and share its wait
    asm volatile(""
                 :
                 : "s"(nxt[0].w), "s"(nxt[1].w), "s"(nxt[2].w), "s"(nxt[3].w), "s"(nxt[4].w),
                   "s"(nxt[5].w), "s"(nxt[6].w), "s"(nxt[7].w), "s"(nxt[0].rel), "s"(nxt[1].rel),
                   "s"(nxt[2].rel), "s"(nxt[3].rel), "s"(nxt[4].rel), "s"(nxt[5].rel),
                   "s"(nxt[6].rel), "s"(nxt[7].rel));
#pragma unroll
    for (int k = 0; k < PT_BATCH; k += 2) {
      acc0 = fma(cur[k].w, xv[k], acc0);
      acc1 = fma(cur[k + 1].w, xv[k + 1], acc1);
    }
#pragma unroll
    for (int k = 0; k < PT_BATCH; ++k) cur[k] = nxt[k];
  }
  return acc0 + acc1;
}

// Stages the block's region (tile + halo, S[0] x S[1] x S[2] cells of the
// design lattice starting at (rx, ry, rz)) in LDS, every load issued before
// the first store: design values x_j (TRANS false) or, for phase (px, py, pz),
// g_i / omega_i at the density cells i = q j + p (TRANS true); 0 outside the
// domain.  The region holds at most PT_STAGE * PROJ_BS cells (h <= 4).
constexpr int PT_STAGE = 12;
template <bool TRANS>
__device__ __forceinline__ void stage_region(const ProjTileArgs& a, int rx, int ry, int rz, int px,
                                             int py, int pz, const double* __restrict__ src,
                                             const double* __restrict__ invw, double* sh) {
  const int nreg = a.S[0] * a.S[1] * a.S[2];
  double v[PT_STAGE];
  // branch-free: cells outside the region or the domain load entry 0 and
  // are masked to 0, so every load of the thread is issued back to back
#pragma unroll
  for (int u = 0; u < PT_STAGE; ++u) {
    const int idx = (int)threadIdx.x + u * PROJ_BS;
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
#pragma unroll
  for (int u = 0; u < PT_STAGE; ++u) {
    const int idx = (int)threadIdx.x + u * PROJ_BS;
    if (idx < nreg) sh[idx] = v[u];
  }
}

// (the tables are separate no-alias parameters: the compiler then reads them
// through the scalar cache, which it may not do for memory the kernel's
// stores might alias)
__global__ __launch_bounds__(PROJ_BS) void k_proj_fwd_tile(ProjTileArgs a,
                                                            const ProjEntry* __restrict__ ent,
                                                            const int* __restrict__ start,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ invw,
                                                            double* __restrict__ out) {
  extern __shared__ double sh[];
  int bx, by, bz;
  tile_origin(a, bx, by, bz);
  const int t = threadIdx.x;
  const int rx = bx * PT_X - a.h, ry = by * PT_Y - a.h, rz = bz * PT_Z - a.h;
  stage_region<false>(a, rx, ry, rz, 0, 0, 0, x, nullptr, sh);
  __syncthreads();
  const int lx = t % PT_X, ly = (t / PT_X) % PT_Y, lz = t / (PT_X * PT_Y);
  const int jx = bx * PT_X + lx, jy = by * PT_Y + ly, jz = bz * PT_Z + lz;
  const bool on = jx < a.nx[0] && jy < a.nx[1] && jz < a.nx[2];
  const int base = (lx + a.h) + a.S[0] * ((ly + a.h) + a.S[1] * (lz + a.h));
  // phases in groups of 8: the gathers first, then the group's 1/omega loads
  // together, then its stores
  constexpr int G = 8;
  for (int p0 = 0; p0 < a.np; p0 += G) {
    double acc[G];
    long idx[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int p = p0 + u < a.np ? p0 + u : p0;
      const int px = p % a.q, py = (p / a.q) % a.q, pz = p / (a.q * a.q);
      acc[u] = p0 + u < a.np ? phase_gather<1>(ent, start[p], start[p + 1], sh, base) : 0.0;
      idx[u] = on ? (long)(a.q * jx + px) +
                        (long)a.nr[0] * ((long)(a.q * jy + py) + (long)a.nr[1] * (a.q * jz + pz))
                  : 0L;
    }
    double w[G];
#pragma unroll
    for (int u = 0; u < G; ++u) w[u] = invw[idx[u]];
    if (on) {
#pragma unroll
      for (int u = 0; u < G; ++u)
        if (p0 + u < a.np) out[idx[u]] = acc[u] * w[u];
    }
  }
}

__global__ __launch_bounds__(PROJ_BS) void k_proj_t_tile(ProjTileArgs a,
                                                          const ProjEntry* __restrict__ ent,
                                                          const int* __restrict__ start,
                                                          const double* __restrict__ g,
                                                          const double* __restrict__ invw,
                                                          double* __restrict__ out) {
  extern __shared__ double sh[];
  int bx, by, bz;
  tile_origin(a, bx, by, bz);
  const int t = threadIdx.x;
  const int rx = bx * PT_X - a.h, ry = by * PT_Y - a.h, rz = bz * PT_Z - a.h;
  const int lx = t % PT_X, ly = (t / PT_X) % PT_Y, lz = t / (PT_X * PT_Y);
  const int kx = bx * PT_X + lx, ky = by * PT_Y + ly, kz = bz * PT_Z + lz;
  const bool on = kx < a.nx[0] && ky < a.nx[1] && kz < a.nx[2];
  const int base = (lx + a.h) + a.S[0] * ((ly + a.h) + a.S[1] * (lz + a.h));
  double acc = 0.0;
  for (int p = 0; p < a.np; ++p) {
    const int px = p % a.q, py = (p / a.q) % a.q, pz = p / (a.q * a.q);
    __syncthreads();  // the previous phase's reads are done
    stage_region<true>(a, rx, ry, rz, px, py, pz, g, invw, sh);
    __syncthreads();
    acc += phase_gather<-1>(ent, start[p], start[p + 1], sh, base);
  }
  if (on) out[kx + (long)a.nx[0] * (ky + (long)a.nx[1] * kz)] = acc;
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

// The q^3 phase stencils of the tiled kernels (left empty, q = 0, when d does
// not divide n, the phases are too many or a stencil reaches past 4 cells).
void Proj::phase_tables(ProjGeom& g) {
  g.q = g.np = g.h = 0;
  g.ent.clear();
  g.start.clear();
  if (g.n % g.d != 0) return;
  const int q = g.n / g.d;
  if (q > 8) return;
  struct Raw {
    int o[3];
    double w;
  };
  std::vector<std::vector<Raw>> ph(q * q * q);
  int h = 0;
  long total = 0;
  for (int p = 0; p < q * q * q; ++p) {
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
          const double w = g.tab[std::labs(mx)] * (g.tab[std::labs(mz)] * g.tab[std::labs(my)]);
          ph[p].push_back(Raw{{ox, oy, oz}, w});
          h = std::max({h, std::abs(ox), std::abs(oy), std::abs(oz)});
        }
    total += (long)ph[p].size();
  }
  if (h > 4 || total > 65536) return;  // (h <= 4: the region fits PT_STAGE * PROJ_BS cells)
  g.q = q;
  g.np = q * q * q;
  g.h = h;
  const int SX = PT_X + 2 * h, SY = PT_Y + 2 * h;  // the tile's x and y extents with halo
  g.start.push_back(0);
  for (int p = 0; p < g.np; ++p) {
    for (const Raw& r : ph[p]) g.ent.push_back(ProjEntry{r.w, r.o[0] + SX * (r.o[1] + SY * r.o[2]), 0});
    // zero-weight padding to whole batches of the gather loop
    while (g.ent.size() % PT_BATCH) g.ent.push_back(ProjEntry{0.0, 0, 0});
    g.start.push_back((int)g.ent.size());
  }
}

size_t Proj::device_bytes(const mgcg_proj_desc& d) {
  const ProjGeom g = geometry(d);
  return ((size_t)g.nrho + (size_t)g.ntab) * sizeof(double) + g.ent.size() * sizeof(ProjEntry) +
         g.start.size() * sizeof(int);
}

Proj::Proj(const mgcg_proj_desc& d, int device) : g_(geometry(d)), device_(device) {
  MGCG_HIP(hipSetDevice(device_));
  (void)d;
  try {
    if (hipMalloc(&invw_, (size_t)g_.nrho * sizeof(double)) != hipSuccess ||
        hipMalloc(&tab_, g_.tab.size() * sizeof(double)) != hipSuccess ||
        (g_.q > 0 && (hipMalloc(&ent_, g_.ent.size() * sizeof(ProjEntry)) != hipSuccess ||
                      hipMalloc(&start_, g_.start.size() * sizeof(int)) != hipSuccess))) {
      (void)hipGetLastError();
      throw Error(MGCG_ENOMEM, "projection allocation failed");
    }
    MGCG_HIP(hipMemcpyAsync(tab_, g_.tab.data(), g_.tab.size() * sizeof(double),
                            hipMemcpyHostToDevice, stream_));
    if (g_.q > 0) {
      MGCG_HIP(hipMemcpyAsync(ent_, g_.ent.data(), g_.ent.size() * sizeof(ProjEntry),
                              hipMemcpyHostToDevice, stream_));
      MGCG_HIP(hipMemcpyAsync(start_, g_.start.data(), g_.start.size() * sizeof(int),
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
  if (ent_) (void)hipFree(ent_);
  if (start_) (void)hipFree(start_);
  invw_ = tab_ = nullptr;
  ent_ = nullptr;
  start_ = nullptr;
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
    const int T[3] = {PT_X, PT_Y, PT_Z};
    long nb = 1;
    for (int i = 0; i < 3; ++i) {
      a.S[i] = T[i] + 2 * g_.h;
      a.ntile[i] = (g_.nx[i] + T[i] - 1) / T[i];
      nb *= a.ntile[i];
    }
    const size_t lds = (size_t)a.S[0] * a.S[1] * a.S[2] * sizeof(double);
    if (transpose)
      hipLaunchKernelGGL(k_proj_t_tile, dim3((unsigned)nb), dim3(PROJ_BS), lds, stream_, a,
                         (const ProjEntry*)ent_, (const int*)start_, din, (const double*)invw_,
                         dout);
    else
      hipLaunchKernelGGL(k_proj_fwd_tile, dim3((unsigned)nb), dim3(PROJ_BS), lds, stream_, a,
                         (const ProjEntry*)ent_, (const int*)start_, din, (const double*)invw_,
                         dout);
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
