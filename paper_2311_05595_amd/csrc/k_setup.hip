// Operator refresh after a density update (Sec. 7.2: the smoother data,
// the system matrix of every mesh level and the Cholesky factor of the
// coarsest one are recomputed at each optimisation iteration), plus the
// compliance and sensitivity kernels (Sec. 3.4).
#include "devutil.h"

namespace mgcg {

// ------------------------------------------------------------ SIMP moduli
__global__ __launch_bounds__(BS) void k_simp(const double* __restrict__ rho, double* E, float* E32,
                                             long n, double E0, double Emin, double penal, int* bad) {
  for (long i = (long)blockIdx.x * BS + threadIdx.x; i < n; i += (long)gridDim.x * BS) {
    const double r = rho[i];
    if (!(r >= 0.0 && r <= 1.0)) {  // also catches NaN
      atomicOr(bad, 1);
      E[i] = Emin;
      if (E32) E32[i] = (float)Emin;
      continue;
    }
    const double e = Emin + pow(r, penal) * (E0 - Emin);
    E[i] = e;
    if (E32) E32[i] = (float)e;
  }
}

void setup_simp(const double* rho, double* E, float* E32, long n, double E0, double Emin,
                double penal, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_simp, dim3(vec_grid(n)), dim3(BS), 0, st, rho, E, E32, n, E0, Emin, penal,
                     bad);
  MGCG_HIP(hipGetLastError());
}

// ------------------------------------------------ effective element matrices
// Keff[e] = sum_s E[dens(e, s)] Ksub[s] for a batch of EB elements per block
// (the shared Ksub entry is read once per batch), supported rows/columns
// zeroed.
constexpr int EB = 16;

__device__ __forceinline__ bool dof_fixed(const uint8_t* mask, const Lat& L, int order, int ex,
                                          int ey, int ez, int ldof) {
  const int p1 = order + 1;
  const int a = ldof / 3, c = ldof % 3;
  const int ax = a % p1, ay = (a / p1) % p1, az = a / (p1 * p1);
  const long node = (order * ex + ax) + (long)L.nx * ((order * ey + ay) + (long)L.ny * (order * ez + az));
  return (mask[node] >> c) & 1;
}

__global__ __launch_bounds__(BS) void k_effective(int order, int nsub, int nelx, int nely, int nelz,
                                                  const double* __restrict__ E,
                                                  const double* __restrict__ Ksub,
                                                  const uint8_t* __restrict__ mask, Lat L,
                                                  double* Keff) {
  const int ns3 = nsub * nsub * nsub;
  const int nd = order == 1 ? 24 : 81;
  const int nd2 = nd * nd;
  const long nel = (long)nelx * nely * nelz;
  const long e0 = (long)blockIdx.y * EB;
  __shared__ double sE[EB][64];
  for (int t = threadIdx.x; t < EB * ns3; t += BS) {
    const int b = t / ns3, s = t % ns3;
    const long e = e0 + b;
    double v = 0.0;
    if (e < nel) {
      const int ex = (int)(e % nelx), ey = (int)((e / nelx) % nely), ez = (int)(e / ((long)nelx * nely));
      const int sx = s % nsub, sy = (s / nsub) % nsub, sz = s / (nsub * nsub);
      const long di = (nsub * ex + sx) + (long)(nsub * nelx) * ((nsub * ey + sy) + (long)(nsub * nely) * (nsub * ez + sz));
      v = E[di];
    }
    sE[b][s] = v;
  }
  __syncthreads();
  const int ij = blockIdx.x * BS + threadIdx.x;
  if (ij >= nd2) return;
  double acc[EB];
#pragma unroll
  for (int b = 0; b < EB; ++b) acc[b] = 0.0;
  for (int s = 0; s < ns3; ++s) {
    const double k = Ksub[(size_t)s * nd2 + ij];
#pragma unroll
    for (int b = 0; b < EB; ++b) acc[b] += sE[b][s] * k;
  }
  const int i = ij / nd, j = ij % nd;
  for (int b = 0; b < EB; ++b) {
    const long e = e0 + b;
    if (e >= nel) break;
    const int ex = (int)(e % nelx), ey = (int)((e / nelx) % nely), ez = (int)(e / ((long)nelx * nely));
    const bool fx = dof_fixed(mask, L, order, ex, ey, ez, i) || dof_fixed(mask, L, order, ex, ey, ez, j);
    Keff[(size_t)e * nd2 + ij] = fx ? 0.0 : acc[b];
  }
}

void setup_effective(int order, int nsub, int nelx, int nely, int nelz, const double* E,
                     const double* Ksub, const uint8_t* mask, Lat L, double* Keff, hipStream_t st) {
  const int nd = order == 1 ? 24 : 81;
  const long nel = (long)nelx * nely * nelz;
  if (nsub * nsub * nsub > 64) throw Error(-1, "nsub > 4 is not supported");
  dim3 grid((nd * nd + BS - 1) / BS, (unsigned)((nel + EB - 1) / EB));
  hipLaunchKernelGGL(k_effective, grid, dim3(BS), 0, st, order, nsub, nelx, nely, nelz, E, Ksub,
                     mask, L, Keff);
  MGCG_HIP(hipGetLastError());
}

// ------------------------------------------------------------ Galerkin
// One block per coarse element.  Children have nodes at coarse-local lattice
// positions in {0,1,2}^3; W[a][b] = trilinear weight of coarse vertex b at
// child node a.  KE += W^T (Z Kc Z) W, computed as T = Kc W then W^T T.
__device__ __forceinline__ double w1d(int pos, int bit) {
  return pos == 1 ? 0.5 : ((pos == 2 * bit) ? 1.0 : 0.0);
}

__global__ __launch_bounds__(BS) void k_galerkin(int src_kind, Lat F, const double* __restrict__ E,
                                                 const double* __restrict__ K0,
                                                 const double* __restrict__ Kc,
                                                 const uint8_t* __restrict__ mask_f, int ncx,
                                                 int ncy, int ncz, double* KE,
                                                 const int* __restrict__ elist) {
  __shared__ double sK[81 * 81];
  __shared__ double sT[81 * 24];
  __shared__ double sW[27 * 8];
  __shared__ uint8_t sFix[81];
  const long E_id = elist ? elist[blockIdx.x] : blockIdx.x;
  const int EX = (int)(E_id % ncx), EY = (int)((E_id / ncx) % ncy), EZ = (int)(E_id / ((long)ncx * ncy));
  const bool q2 = (src_kind == OP_EQ2);
  const int nen = q2 ? 27 : 8, nd = 3 * nen, p1 = q2 ? 3 : 2;
  const int nchild = q2 ? 1 : 8;
  // fine element grid (Q1-type children live on the fine lattice's element grid)
  const int fex = q2 ? (F.nx - 1) / 2 : F.nx - 1, fey = q2 ? (F.ny - 1) / 2 : F.ny - 1;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int ch = 0; ch < nchild; ++ch) {
    const int cx = q2 ? 0 : (ch & 1), cy = q2 ? 0 : ((ch >> 1) & 1), cz = q2 ? 0 : (ch >> 2);
    const int ex = q2 ? EX : 2 * EX + cx, ey = q2 ? EY : 2 * EY + cy, ez = q2 ? EZ : 2 * EZ + cz;
    const long fe = ex + (long)fex * (ey + (long)fey * ez);
    // child supports and interpolation weights
    for (int t = threadIdx.x; t < nd; t += BS) {
      const int a = t / 3, c = t % 3;
      const int ax = a % p1, ay = (a / p1) % p1, az = a / (p1 * p1);
      const int order = q2 ? 2 : 1;
      const long node = (order * ex + ax) + (long)F.nx * ((order * ey + ay) + (long)F.ny * (order * ez + az));
      sFix[t] = (mask_f[node] >> c) & 1;
    }
    for (int t = threadIdx.x; t < nen * 8; t += BS) {
      const int a = t / 8, b = t % 8;
      const int ax = a % p1, ay = (a / p1) % p1, az = a / (p1 * p1);
      const int px = q2 ? ax : cx + ax, py = q2 ? ay : cy + ay, pz = q2 ? az : cz + az;
      sW[t] = w1d(px, b & 1) * w1d(py, (b >> 1) & 1) * w1d(pz, b >> 2);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nd * nd; t += BS) {
      const int i = t / nd, j = t % nd;
      double v;
      if (src_kind == OP_MF_Q1)
        v = E[fe] * K0[t];
      else
        v = Kc[(size_t)fe * nd * nd + t];
      sK[t] = (sFix[i] || sFix[j]) ? 0.0 : v;
    }
    __syncthreads();
    // T[(a,i)][(b,j)] = sum_a' Kc[(a,i)][(a',j)] W[a'][b]
    for (int t = threadIdx.x; t < nd * 24; t += BS) {
      const int row = t / 24, col = t % 24;
      const int b = col / 3, j = col % 3;
      double s = 0.0;
      for (int a2 = 0; a2 < nen; ++a2) {
        const double w = sW[a2 * 8 + b];
        if (w != 0.0) s += sK[row * nd + 3 * a2 + j] * w;
      }
      sT[t] = s;
    }
    __syncthreads();
    // KE[(b,i)][(b',j)] += sum_a W[a][b] T[(a,i)][(b',j)]
    for (int q = 0; q < 3; ++q) {
      const int t = threadIdx.x + q * BS;
      if (t >= 576) break;
      const int row = t / 24, col = t % 24;
      const int b = row / 3, i = row % 3;
      double s = 0.0;
      for (int a = 0; a < nen; ++a) {
        const double w = sW[a * 8 + b];
        if (w != 0.0) s += w * sT[(3 * a + i) * 24 + col];
      }
      acc[q] += s;
    }
    __syncthreads();
  }
  for (int q = 0; q < 3; ++q) {
    const int t = threadIdx.x + q * BS;
    if (t < 576) KE[(size_t)E_id * 576 + t] = acc[q];
  }
}

void setup_galerkin(int src_kind, Lat fine, const double* E, const double* K0, const double* Kc,
                    const uint8_t* mask_f, int ncx, int ncy, int ncz, double* KE,
                    const int* elist, int n_elist, hipStream_t st) {
  const long nce = elist ? n_elist : (long)ncx * ncy * ncz;
  if (nce <= 0) return;
  hipLaunchKernelGGL(k_galerkin, dim3((unsigned)nce), dim3(BS), 0, st, src_kind, fine, E, K0, Kc,
                     mask_f, ncx, ncy, ncz, KE, elist);
  MGCG_HIP(hipGetLastError());
}

// One block = 576 threads (one per matrix entry) x GB coarse elements; the
// moduli of the GB elements sit in LDS, every G entry is read once per block.
constexpr int GB = 8;
__global__ __launch_bounds__(576) void k_galerkin_lin(const double* __restrict__ E,
                                                      const double* __restrict__ G, int B,
                                                      int nsub, int nelx, int nely, int ncx,
                                                      int ncy, int ncz, double* KE) {
  extern __shared__ double sE[];  // [GB][M]
  const int M = B * B * B;
  const long nce = (long)ncx * ncy * ncz;
  const long e0 = (long)blockIdx.x * GB;
  const long ndx = (long)nsub * nelx, ndy = (long)nsub * nely;
  for (int t = threadIdx.x; t < GB * M; t += 576) {
    const int b = t / M, m = t % M;
    const long e = e0 + b;
    double v = 0.0;
    if (e < nce) {
      const int EX = (int)(e % ncx), EY = (int)((e / ncx) % ncy), EZ = (int)(e / ((long)ncx * ncy));
      const int px = m % B, py = (m / B) % B, pz = m / (B * B);
      v = E[(B * (long)EX + px) + ndx * ((B * (long)EY + py) + ndy * (B * (long)EZ + pz))];
    }
    sE[t] = v;
  }
  __syncthreads();
  const int q = threadIdx.x;
  double acc[GB];
#pragma unroll
  for (int b = 0; b < GB; ++b) acc[b] = 0.0;
  for (int m = 0; m < M; ++m) {
    const double g = G[(size_t)m * 576 + q];
#pragma unroll
    for (int b = 0; b < GB; ++b) acc[b] += sE[b * M + m] * g;
  }
#pragma unroll
  for (int b = 0; b < GB; ++b) {
    const long e = e0 + b;
    if (e < nce) KE[(size_t)e * 576 + q] = acc[b];
  }
}

void setup_galerkin_lin(const double* E, const double* G, int B, int nsub, int nelx, int nely,
                        int ncx, int ncy, int ncz, double* KE, hipStream_t st) {
  const long nce = (long)ncx * ncy * ncz;
  const int M = B * B * B;
  hipLaunchKernelGGL(k_galerkin_lin, dim3((unsigned)((nce + GB - 1) / GB)), dim3(576),
                     (size_t)GB * M * sizeof(double), st, E, G, B, nsub, nelx, nely, ncx, ncy, ncz,
                     KE);
  MGCG_HIP(hipGetLastError());
}

// ------------------------------------------------------------ stencils
// Index of the stored (forward) block of offset d, or -1 for a backward one.
__device__ __forceinline__ int fwd_block(int dx, int dy, int dz) {
#pragma unroll
  for (int b = 0; b < ST_BLOCKS; ++b) {
    const Off3 o = st_offset(b);
    if (o.dx == dx && o.dy == dy && o.dz == dz) return b;
  }
  return -1;
}

// Jacobi data of one DOF row from its diagonal and absolute row sum: the
// weight is min(omega, theta * A_ii / sum_j |A_ij|) (a Gershgorin bound of
// theta < 2 on every row of W D^{-1} A), stored pre-divided by A_ii.
template <typename T>
__device__ __forceinline__ void jacobi_row(bool fixed, double dg, double rs, double omega,
                                           double theta, T* wD, double* diag64, long idx) {
  if (diag64) diag64[idx] = fixed ? 1.0 : dg;
  if (fixed || !(dg > 0.0)) {
    wD[idx] = T(0);
    return;
  }
  const double w = fmin(omega, theta * dg / rs);
  wD[idx] = T(w / dg);
}

// Node-parallel assembly of the half stencil from Q1-type element matrices
// KE [nel][24*24] on lattice L (elements (nx-1)(ny-1)(nz-1)); all 27 blocks
// of the node's rows are formed for the row sums, the 14 forward ones stored.
template <typename T>
__global__ __launch_bounds__(BS) void k_stencil(Lat L, const double* __restrict__ KE,
                                                const uint8_t* __restrict__ mask, T* coef, T* wD,
                                                double* diag64, double omega, double theta) {
  const long node = (long)blockIdx.x * BS + threadIdx.x;
  const long nn = L.nn();
  if (node >= nn) return;
  const int i = (int)(node % L.nx), j = (int)((node / L.nx) % L.ny), k = (int)(node / ((long)L.nx * L.ny));
  const int ex1 = L.nx - 1, ey1 = L.ny - 1, ez1 = L.nz - 1;
  const uint8_t mi = mask[node];
  double rs[3] = {0.0, 0.0, 0.0}, dg[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 27; ++q) {
    const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
    const int b = fwd_block(dx, dy, dz);
    const int ii = i + dx, jj = j + dy, kk = k + dz;
    const bool nbok = (unsigned)ii < (unsigned)L.nx && (unsigned)jj < (unsigned)L.ny &&
                      (unsigned)kk < (unsigned)L.nz;
    const uint8_t mj = nbok ? mask[ii + (long)L.nx * (jj + (long)L.ny * kk)] : 7;
    double blk[9];
    for (int t = 0; t < 9; ++t) blk[t] = 0.0;
    if (nbok) {
      for (int oz = 0; oz < 2; ++oz)
        for (int oy = 0; oy < 2; ++oy)
          for (int ox = 0; ox < 2; ++ox) {
            const int ex = i - 1 + ox, ey = j - 1 + oy, ez = k - 1 + oz;
            if ((unsigned)ex >= (unsigned)ex1 || (unsigned)ey >= (unsigned)ey1 || (unsigned)ez >= (unsigned)ez1)
              continue;
            const int ax = 1 - ox, ay = 1 - oy, az = 1 - oz;
            const int bx = ax + dx, by = ay + dy, bz = az + dz;
            if ((unsigned)bx > 1u || (unsigned)by > 1u || (unsigned)bz > 1u) continue;
            const int a = ax + 2 * (ay + 2 * az), bb = bx + 2 * (by + 2 * bz);
            const double* K = KE + (size_t)(ex + (long)ex1 * (ey + (long)ey1 * ez)) * 576;
            for (int c = 0; c < 3; ++c)
              for (int e = 0; e < 3; ++e) blk[3 * c + e] += K[(3 * a + c) * 24 + 3 * bb + e];
          }
    }
    for (int c = 0; c < 3; ++c)
      for (int e = 0; e < 3; ++e) {
        double v = blk[3 * c + e];
        if (((mi >> c) & 1) || ((mj >> e) & 1)) v = 0.0;
        if (q == 13 && c == e && ((mi >> c) & 1)) v = 1.0;
        rs[c] += fabs(v);
        if (q == 13 && c == e) dg[c] = v;
        if (b >= 0) coef[(size_t)(b * 9 + 3 * c + e) * nn + node] = (T)v;
      }
  }
  for (int c = 0; c < 3; ++c)
    jacobi_row<T>((mi >> c) & 1, dg[c], rs[c], omega, theta, wD, diag64, 3 * node + c);
}

template <typename T>
void setup_stencil(Lat L, const double* KE, const uint8_t* mask, T* coef, T* wD, double* diag64,
                   double omega, double theta, hipStream_t st) {
  hipLaunchKernelGGL(k_stencil<T>, dim3(nblocks(L.nn())), dim3(BS), 0, st, L, KE, mask, coef, wD,
                     diag64, omega, theta);
  MGCG_HIP(hipGetLastError());
}
template void setup_stencil<double>(Lat, const double*, const uint8_t*, double*, double*, double*,
                                    double, double, hipStream_t);
template void setup_stencil<float>(Lat, const double*, const uint8_t*, float*, float*, double*,
                                   double, double, hipStream_t);

// Jacobi data of the matrix-free trilinear operator (E_e K0 per element).
template <typename T>
__global__ __launch_bounds__(BS) void k_diag_mf(Lat L, const double* __restrict__ E,
                                                const double* __restrict__ K0,
                                                const uint8_t* __restrict__ mask, T* wD,
                                                double* diag64, double omega, double theta) {
  const long node = (long)blockIdx.x * BS + threadIdx.x;
  if (node >= L.nn()) return;
  const int i = (int)(node % L.nx), j = (int)((node / L.nx) % L.ny), k = (int)(node / ((long)L.nx * L.ny));
  const int ex1 = L.nx - 1, ey1 = L.ny - 1, ez1 = L.nz - 1;
  const uint8_t mi = mask[node];
  double rs[3] = {0.0, 0.0, 0.0}, dg[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 27; ++q) {
    const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
    const int ii = i + dx, jj = j + dy, kk = k + dz;
    if ((unsigned)ii >= (unsigned)L.nx || (unsigned)jj >= (unsigned)L.ny || (unsigned)kk >= (unsigned)L.nz)
      continue;
    const uint8_t mj = mask[ii + (long)L.nx * (jj + (long)L.ny * kk)];
    double blk[9];
    for (int t = 0; t < 9; ++t) blk[t] = 0.0;
    for (int o = 0; o < 8; ++o) {
      const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
      const int ex = i - 1 + ox, ey = j - 1 + oy, ez = k - 1 + oz;
      if ((unsigned)ex >= (unsigned)ex1 || (unsigned)ey >= (unsigned)ey1 || (unsigned)ez >= (unsigned)ez1)
        continue;
      const int ax = 1 - ox, ay = 1 - oy, az = 1 - oz;
      const int bx = ax + dx, by = ay + dy, bz = az + dz;
      if ((unsigned)bx > 1u || (unsigned)by > 1u || (unsigned)bz > 1u) continue;
      const int a = ax + 2 * (ay + 2 * az), bb = bx + 2 * (by + 2 * bz);
      const double Ee = E[ex + (long)ex1 * (ey + (long)ey1 * ez)];
      for (int c = 0; c < 3; ++c)
        for (int e = 0; e < 3; ++e) blk[3 * c + e] += Ee * K0[(3 * a + c) * 24 + 3 * bb + e];
    }
    for (int c = 0; c < 3; ++c)
      for (int e = 0; e < 3; ++e) {
        double v = blk[3 * c + e];
        if (((mi >> c) & 1) || ((mj >> e) & 1)) v = 0.0;
        if (q == 13 && c == e && ((mi >> c) & 1)) v = 1.0;
        rs[c] += fabs(v);
        if (q == 13 && c == e) dg[c] = v;
      }
  }
  for (int c = 0; c < 3; ++c)
    jacobi_row<T>((mi >> c) & 1, dg[c], rs[c], omega, theta, wD, diag64, 3 * node + c);
}

template <typename T>
void setup_diag_mf(Lat L, const double* E, const double* K0, const uint8_t* mask, T* wD,
                   double* diag64, double omega, double theta, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_mf<T>, dim3(nblocks(L.nn())), dim3(BS), 0, st, L, E, K0, mask, wD,
                     diag64, omega, theta);
  MGCG_HIP(hipGetLastError());
}
template void setup_diag_mf<double>(Lat, const double*, const double*, const uint8_t*, double*,
                                    double*, double, double, hipStream_t);
template void setup_diag_mf<float>(Lat, const double*, const double*, const uint8_t*, float*,
                                   double*, double, double, hipStream_t);

// Jacobi data of the stored triquadratic operator: the row of a node couples
// the nodes within two lattice steps; entries shared by several elements
// are summed before taking absolute values.
template <typename T>
__global__ __launch_bounds__(BS) void k_diag_eq2(Lat L, const double* __restrict__ Ke,
                                                 const uint8_t* __restrict__ mask, T* wD,
                                                 double* diag64, double omega, double theta) {
  const long node = (long)blockIdx.x * BS + threadIdx.x;
  if (node >= L.nn()) return;
  const int i = (int)(node % L.nx), j = (int)((node / L.nx) % L.ny), k = (int)(node / ((long)L.nx * L.ny));
  const int nex = (L.nx - 1) / 2, ney = (L.ny - 1) / 2, nez = (L.nz - 1) / 2;
  int exs[2], axs[2], nxe = 0, eys[2], ays[2], nye = 0, ezs[2], azs[2], nze = 0;
  auto axis = [](int p, int ne, int* es, int* as, int& n) {
    n = 0;
    if (p & 1) { es[0] = (p - 1) / 2; as[0] = 1; n = 1; }
    else {
      if (p / 2 - 1 >= 0) { es[n] = p / 2 - 1; as[n] = 2; ++n; }
      if (p / 2 < ne) { es[n] = p / 2; as[n] = 0; ++n; }
    }
  };
  axis(i, nex, exs, axs, nxe);
  axis(j, ney, eys, ays, nye);
  axis(k, nez, ezs, azs, nze);
  const uint8_t mi = mask[node];
  double rs[3] = {0.0, 0.0, 0.0}, dg[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 125; ++q) {
    const int dx = q % 5 - 2, dy = (q / 5) % 5 - 2, dz = q / 25 - 2;
    double blk[9];
    for (int t = 0; t < 9; ++t) blk[t] = 0.0;
    bool any = false;
    for (int cz = 0; cz < nze; ++cz)
      for (int cy = 0; cy < nye; ++cy)
        for (int cx = 0; cx < nxe; ++cx) {
          const int bx = axs[cx] + dx, by = ays[cy] + dy, bz = azs[cz] + dz;
          if ((unsigned)bx > 2u || (unsigned)by > 2u || (unsigned)bz > 2u) continue;
          any = true;
          const long e = exs[cx] + (long)nex * (eys[cy] + (long)ney * ezs[cz]);
          const int a = axs[cx] + 3 * (ays[cy] + 3 * azs[cz]), bb = bx + 3 * (by + 3 * bz);
          for (int c = 0; c < 3; ++c)
            for (int e2 = 0; e2 < 3; ++e2)
              blk[3 * c + e2] += Ke[(size_t)e * 6561 + (3 * a + c) * 81 + 3 * bb + e2];
        }
    if (!any) continue;
    for (int c = 0; c < 3; ++c)
      for (int e2 = 0; e2 < 3; ++e2) {
        double v = blk[3 * c + e2];  // supported rows/columns are zero in Ke
        if (q == 62 && c == e2 && ((mi >> c) & 1)) v = 1.0;
        rs[c] += fabs(v);
        if (q == 62 && c == e2) dg[c] = v;
      }
  }
  for (int c = 0; c < 3; ++c)
    jacobi_row<T>((mi >> c) & 1, dg[c], rs[c], omega, theta, wD, diag64, 3 * node + c);
}

template <typename T>
void setup_diag_eq2(Lat L, const double* Ke, const uint8_t* mask, T* wD, double* diag64,
                    double omega, double theta, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_eq2<T>, dim3(nblocks(L.nn())), dim3(BS), 0, st, L, Ke, mask, wD,
                     diag64, omega, theta);
  MGCG_HIP(hipGetLastError());
}
template void setup_diag_eq2<double>(Lat, const double*, const uint8_t*, double*, double*, double,
                                     double, hipStream_t);
template void setup_diag_eq2<float>(Lat, const double*, const uint8_t*, float*, double*, double,
                                    double, hipStream_t);

// ------------------------------------------------------------ coarsest level
// Dense A_ff (row-major, nc x nc) from Q1-type FP64 element matrices of the
// level (src OP_MF_Q1: E_e K0; otherwise KE[e]); one thread per row
// accumulates the contributions of the elements around its node, so every
// entry has a single writer (A must be zeroed before).
__global__ __launch_bounds__(BS) void k_dense(int src_kind, Lat L, const double* __restrict__ E,
                                              const double* __restrict__ K0,
                                              const double* __restrict__ KE,
                                              const int* __restrict__ freedof,
                                              const int* __restrict__ dofpos, int nc, double* A) {
  const int I = blockIdx.x * BS + threadIdx.x;
  if (I >= nc) return;
  const int gdof = freedof[I];
  const long node = gdof / 3;
  const int c = gdof % 3;
  const int i = (int)(node % L.nx), j = (int)((node / L.nx) % L.ny), k = (int)(node / ((long)L.nx * L.ny));
  const int ex1 = L.nx - 1, ey1 = L.ny - 1, ez1 = L.nz - 1;
  for (int o = 0; o < 8; ++o) {
    const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
    const int ex = i - 1 + ox, ey = j - 1 + oy, ez = k - 1 + oz;
    if ((unsigned)ex >= (unsigned)ex1 || (unsigned)ey >= (unsigned)ey1 || (unsigned)ez >= (unsigned)ez1)
      continue;
    const long e = ex + (long)ex1 * (ey + (long)ey1 * ez);
    const int a = (1 - ox) + 2 * ((1 - oy) + 2 * (1 - oz));
    for (int b = 0; b < 8; ++b) {
      const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
      const long nb = (ex + bx) + (long)L.nx * ((ey + by) + (long)L.ny * (ez + bz));
      for (int e2 = 0; e2 < 3; ++e2) {
        const int J = dofpos[3 * nb + e2];
        if (J < 0) continue;
        const int kk = (3 * a + c) * 24 + 3 * b + e2;
        const double v = src_kind == OP_MF_Q1 ? E[e] * K0[kk] : KE[(size_t)e * 576 + kk];
        A[(size_t)I * nc + J] += v;
      }
    }
  }
}

void setup_dense(int src_kind, Lat L, const double* E, const double* K0, const double* KE,
                 const int* freedof, const int* dofpos, int nc, double* A, hipStream_t st) {
  fill<double>(A, 0.0, (long)nc * nc, st);
  if (nc == 0) return;
  hipLaunchKernelGGL(k_dense, dim3(nblocks(nc)), dim3(BS), 0, st, src_kind, L, E, K0, KE, freedof,
                     dofpos, nc, A);
  MGCG_HIP(hipGetLastError());
}

// Right-looking Cholesky A = L L^T in place (lower triangle), one workgroup.
__global__ __launch_bounds__(1024) void k_cholesky(double* A, int n, int* bad) {
  __shared__ double sd;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      double d = A[(size_t)k * n + k];
      if (!(d > 0.0) || !isfinite(d)) {
        atomicOr(bad, 2);
        d = 1.0;
      }
      d = sqrt(d);
      A[(size_t)k * n + k] = d;
      sd = d;
    }
    __syncthreads();
    const double inv = 1.0 / sd;
    for (int i = k + 1 + threadIdx.x; i < n; i += 1024) A[(size_t)i * n + k] *= inv;
    __syncthreads();
    const int m = n - k - 1;
    for (long idx = threadIdx.x; idx < (long)m * m; idx += 1024) {
      const int i = k + 1 + (int)(idx / m), j = k + 1 + (int)(idx % m);
      if (j <= i) A[(size_t)i * n + j] -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
    }
    __syncthreads();
  }
}

// Left-looking panel Cholesky A = L L^T (lower triangle, in place), one
// workgroup: each panel of NB columns is first updated with the finished
// columns to its left (a parallel dot-product pass over L2-resident rows),
// then factored column by column inside LDS.  Dynamic LDS: rows x NB doubles.
template <int NB>
__global__ __launch_bounds__(1024) void k_cholesky_panel(double* A, int n, int* bad) {
  extern __shared__ double P[];  // [n - p0][NB], row-major
  __shared__ double sd;
  const int tid = threadIdx.x;
  for (int p0 = 0; p0 < n; p0 += NB) {
    const int w = min(NB, n - p0), rows = n - p0;
    // load + left-looking update of the panel (lower part r >= c)
    for (int t = tid; t < rows * NB; t += 1024) {
      const int r = t / NB, c = t % NB;
      double v = 0.0;
      if (c < w && r >= c) {
        const double* ai = A + (size_t)(p0 + r) * n;
        const double* aj = A + (size_t)(p0 + c) * n;
        v = ai[p0 + c];
        double s0 = 0.0, s1 = 0.0;
        int k = 0;
        for (; k + 1 < p0; k += 2) {
          s0 += ai[k] * aj[k];
          s1 += ai[k + 1] * aj[k + 1];
        }
        if (k < p0) s0 += ai[k] * aj[k];
        v -= s0 + s1;
      }
      P[t] = v;
    }
    __syncthreads();
    for (int c = 0; c < w; ++c) {
      if (tid == 0) {
        double d = P[c * NB + c];
        if (!(d > 0.0) || !isfinite(d)) {
          atomicOr(bad, 2);
          d = 1.0;
        }
        d = sqrt(d);
        P[c * NB + c] = d;
        sd = d;
      }
      __syncthreads();
      const double inv = 1.0 / sd;
      for (int r = c + 1 + tid; r < rows; r += 1024) P[r * NB + c] *= inv;
      __syncthreads();
      const int wc = w - c - 1;
      if (wc > 0) {
        for (int t = tid; t < (rows - c - 1) * wc; t += 1024) {
          const int r = c + 1 + t / wc, c2 = c + 1 + t % wc;
          if (r >= c2) P[r * NB + c2] -= P[r * NB + c] * P[c2 * NB + c];
        }
      }
      __syncthreads();
    }
    for (int t = tid; t < rows * NB; t += 1024) {
      const int r = t / NB, c = t % NB;
      if (c < w && r >= c) A[(size_t)(p0 + r) * n + p0 + c] = P[t];
    }
    __syncthreads();
  }
}

// Column j of L^{-1} by forward substitution (one workgroup per column).
__global__ __launch_bounds__(BS) void k_trinv(const double* __restrict__ Lf, double* Linv, int n) {
  extern __shared__ double w[];
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += BS) w[i] = (i == j) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = j; k < n; ++k) {
    const double wk = w[k] / Lf[(size_t)k * n + k];
    __syncthreads();
    if (threadIdx.x == 0) w[k] = wk;
    for (int i = k + 1 + threadIdx.x; i < n; i += BS) w[i] -= Lf[(size_t)i * n + k] * wk;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += BS) Linv[(size_t)i * n + j] = (i >= j) ? w[i] : 0.0;
}

// Ainv = Linv^T Linv.
__global__ __launch_bounds__(BS) void k_ltl(const double* __restrict__ Linv, double* Ainv, int n) {
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  if (t >= (long)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  double s = 0.0;
  for (int k = (i > j ? i : j); k < n; ++k) s += Linv[(size_t)k * n + i] * Linv[(size_t)k * n + j];
  Ainv[t] = s;
}

void setup_cholesky_inverse(double* A, double* Linv, double* Ainv, int nc, int* bad,
                            hipStream_t st) {
  if (nc == 0) return;
  // panel in at most 64 KB of LDS
  const size_t lim = 64 * 1024;
  if ((size_t)nc * 32 * sizeof(double) <= lim)
    hipLaunchKernelGGL(k_cholesky_panel<32>, dim3(1), dim3(1024), (size_t)nc * 32 * sizeof(double),
                       st, A, nc, bad);
  else if ((size_t)nc * 16 * sizeof(double) <= lim)
    hipLaunchKernelGGL(k_cholesky_panel<16>, dim3(1), dim3(1024), (size_t)nc * 16 * sizeof(double),
                       st, A, nc, bad);
  else if ((size_t)nc * 8 * sizeof(double) <= lim)
    hipLaunchKernelGGL(k_cholesky_panel<8>, dim3(1), dim3(1024), (size_t)nc * 8 * sizeof(double),
                       st, A, nc, bad);
  else
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, st, A, nc, bad);
  MGCG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_trinv, dim3(nc), dim3(BS), nc * sizeof(double), st, A, Linv, nc);
  MGCG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_ltl, dim3(nblocks((long)nc * nc)), dim3(BS), 0, st, Linv, Ainv, nc);
  MGCG_HIP(hipGetLastError());
}

// ------------------------------------------------------------ compliance
__global__ __launch_bounds__(BS) void k_comp(const double* __restrict__ f, const double* __restrict__ u,
                                             long ndof, int nrhs, double* part) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (r >= nrhs) continue;
    const size_t o = (size_t)r * ndof;
    double s = 0.0;
    for (long i = (long)blockIdx.x * BS + threadIdx.x; i < ndof; i += (long)gridDim.x * BS)
      s += f[o + i] * u[o + i];
    block_partial1(s, part + (size_t)r * MAX_BLOCKS + blockIdx.x);
  }
}

__global__ void k_comp_fin(const double* part, int nb, int nrhs, double* out) {
  __shared__ double sh[BS / 64];
  for (int r = 0; r < nrhs; ++r) {
    const double s = block_sum(part + (size_t)r * MAX_BLOCKS, nb, sh);
    if (threadIdx.x == 0) out[r] = s;
  }
}

void comp_dot(const double* f, const double* u, long ndof, int nrhs, double* out, RedBuf red,
              hipStream_t st) {
  double* part = red.partials + RED_COMP * RED_REGION;
  const int g = vec_grid(ndof);
  hipLaunchKernelGGL(k_comp, dim3(g), dim3(BS), 0, st, f, u, ndof, nrhs, part);
  MGCG_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_comp_fin, dim3(1), dim3(BS), 0, st, part, g, nrhs, out);
  MGCG_HIP(hipGetLastError());
}

// ------------------------------------------------------------ sensitivity
// One thread per (sub-element s, displacement element e), threads of a
// wavefront share s (uniform Ksub[s] reads):
//   dc = -p rho^{p-1} (E0 - Emin) sum_l u_{l,e}^T K^(e_s) u_{l,e}.
template <int ORDER>
__global__ __launch_bounds__(BS) void k_sens(int nsub, int nelx, int nely, int nelz, Lat L,
                                             const double* __restrict__ rho,
                                             const double* __restrict__ u, long ndof, int nrhs,
                                             const double* __restrict__ Ksub, double E0mEmin,
                                             double penal, double* dc) {
  constexpr int P1 = ORDER + 1, NEN = P1 * P1 * P1, ND = 3 * NEN;
  const long nel = (long)nelx * nely * nelz;
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  const int ns3 = nsub * nsub * nsub;
  if (t >= nel * ns3) return;
  const int s = (int)(t / nel);
  const long e = t % nel;
  const int ex = (int)(e % nelx), ey = (int)((e / nelx) % nely), ez = (int)(e / ((long)nelx * nely));
  const double* K = Ksub + (size_t)s * ND * ND;
  double w = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    double ue[ND];
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
      const int ax = a % P1, ay = (a / P1) % P1, az = a / (P1 * P1);
      const long node = (ORDER * ex + ax) + (long)L.nx * ((ORDER * ey + ay) + (long)L.ny * (ORDER * ez + az));
#pragma unroll
      for (int c = 0; c < 3; ++c) ue[3 * a + c] = u[(size_t)r * ndof + 3 * node + c];
    }
    for (int i = 0; i < ND; ++i) {
      double ti = 0.0;
#pragma unroll
      for (int jj = 0; jj < ND; ++jj) ti += K[i * ND + jj] * ue[jj];
      w += ue[i] * ti;
    }
  }
  const int sx = s % nsub, sy = (s / nsub) % nsub, sz = s / (nsub * nsub);
  const long di = (nsub * ex + sx) + (long)(nsub * nelx) * ((nsub * ey + sy) + (long)(nsub * nely) * (nsub * ez + sz));
  const double r = rho[di];
  dc[di] = -penal * pow(r, penal - 1.0) * E0mEmin * w;
}

void sens_kernel(int order, int nsub, int nelx, int nely, int nelz, Lat L, const double* rho,
                 const double* u, long ndof, int nrhs, const double* Ksub, double /*scale_p*/,
                 double E0mEmin, double penal, double* dc, hipStream_t st) {
  const long n = (long)nelx * nely * nelz * nsub * nsub * nsub;
  if (order == 1)
    hipLaunchKernelGGL(k_sens<1>, dim3(nblocks(n)), dim3(BS), 0, st, nsub, nelx, nely, nelz, L, rho,
                       u, ndof, nrhs, Ksub, E0mEmin, penal, dc);
  else
    hipLaunchKernelGGL(k_sens<2>, dim3(nblocks(n)), dim3(BS), 0, st, nsub, nelx, nely, nelz, L, rho,
                       u, ndof, nrhs, Ksub, E0mEmin, penal, dc);
  MGCG_HIP(hipGetLastError());
}

}  // namespace mgcg
