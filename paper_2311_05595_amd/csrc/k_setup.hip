// Operator refresh after a density update (Sec. 7.2: the smoother data,
// the system matrix of every mesh level and the exact coarsest solve are
// recomputed at each optimisation iteration; the paper factors the coarsest
// matrix by Cholesky, here its explicit inverse is built by blocked
// Gauss-Jordan elimination), plus the
// compliance and sensitivity kernels (Sec. 3.4).
#include <utility>

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
  const int nd = 3 * (order + 1) * (order + 1) * (order + 1);
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
  const int nd = 3 * (order + 1) * (order + 1) * (order + 1);
  const long nel = (long)nelx * nely * nelz;
  if (nsub * nsub * nsub > 64) throw Error(-1, "nsub > 4 is not supported");
  dim3 grid((nd * nd + BS - 1) / BS, (unsigned)((nel + EB - 1) / EB));
  hipLaunchKernelGGL(k_effective, grid, dim3(BS), 0, st, order, nsub, nelx, nely, nelz, E, Ksub,
                     mask, L, Keff);
  MGCG_HIP(hipGetLastError());
}

// Wrapped-diagonal copy of symmetric Q2 element matrices: D[e][s][i] =
// K[e][i][(i + s) mod 81], s = 0..40 (one thread per stored value; writes
// coalesced, reads within the element's matrix).
template <typename T>
__global__ __launch_bounds__(BS) void k_pack_q2(const double* __restrict__ K, T* D, long nel) {
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  if (t >= nel * Q2_PACKED) return;
  const long e = t / Q2_PACKED;
  const int q = (int)(t - e * Q2_PACKED), s = q / 81, i = q - 81 * s;
  int j = i + s;
  j -= j >= 81 ? 81 : 0;
  D[t] = (T)K[(size_t)e * 6561 + 81 * i + j];
}

template <typename T>
void setup_pack_q2(const double* K, T* D, long nel, hipStream_t st) {
  const long n = nel * Q2_PACKED;
  hipLaunchKernelGGL(k_pack_q2<T>, dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, st, K, D,
                     nel);
  MGCG_HIP(hipGetLastError());
}
template void setup_pack_q2<double>(const double*, double*, long, hipStream_t);
template void setup_pack_q2<float>(const double*, float*, long, hipStream_t);

// The same for serendipity elements: the 60 rows and columns of their DOFs
// (DOF 3k + c of serendipity node k is DOF 3 s2_node(k) + c of the 27-node
// layout), D[e][s][i] = K[e][i][(i + s) mod 60], s = 0..30.
template <typename T>
__global__ __launch_bounds__(BS) void k_pack_s2(const double* __restrict__ K, T* D, long nel) {
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  if (t >= nel * S2_PACKED) return;
  const long e = t / S2_PACKED;
  const int q = (int)(t - e * S2_PACKED), s = q / 60, i = q - 60 * s;
  int j = i + s;
  j -= j >= 60 ? 60 : 0;
  const int di = 3 * s2_node(i / 3) + i % 3, dj = 3 * s2_node(j / 3) + j % 3;
  D[t] = (T)K[(size_t)e * 6561 + 81 * di + dj];
}

template <typename T>
void setup_pack_s2(const double* K, T* D, long nel, hipStream_t st) {
  const long n = nel * S2_PACKED;
  hipLaunchKernelGGL(k_pack_s2<T>, dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, st, K, D,
                     nel);
  MGCG_HIP(hipGetLastError());
}
template void setup_pack_s2<double>(const double*, double*, long, hipStream_t);
template void setup_pack_s2<float>(const double*, float*, long, hipStream_t);

// The same for tricubic elements: N = 192 DOFs of the 64-node element, or
// the 96 of the 32-node serendipity one (DOF 3k + c of serendipity node k is
// DOF 3 s3_node(k) + c of the 64-node layout), D[e][s][i] = K[e][i][(i + s)
// mod N], s = 0..N/2.
template <typename T, int N>
__global__ __launch_bounds__(BS) void k_pack_e3(const double* __restrict__ K, T* D, long nel) {
  constexpr int PK = (N / 2 + 1) * N;
  const long t = (long)blockIdx.x * BS + threadIdx.x;
  if (t >= nel * PK) return;
  const long e = t / PK;
  const int q = (int)(t - e * PK), s = q / N, i = q - N * s;
  int j = i + s;
  j -= j >= N ? N : 0;
  const int di = N == L3_ND ? i : 3 * s3_node(i / 3) + i % 3;
  const int dj = N == L3_ND ? j : 3 * s3_node(j / 3) + j % 3;
  D[t] = (T)K[(size_t)e * L3_ND * L3_ND + (size_t)L3_ND * di + dj];
}

template <typename T>
void setup_pack_e3(const double* K, T* D, long nel, int serendipity, hipStream_t st) {
  const long n = nel * (serendipity ? S3_PACKED : L3_PACKED);
  if (serendipity)
    hipLaunchKernelGGL((k_pack_e3<T, S3_ND>), dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, st,
                       K, D, nel);
  else
    hipLaunchKernelGGL((k_pack_e3<T, L3_ND>), dim3((unsigned)((n + BS - 1) / BS)), dim3(BS), 0, st,
                       K, D, nel);
  MGCG_HIP(hipGetLastError());
}
template void setup_pack_e3<double>(const double*, double*, long, int, hipStream_t);
template void setup_pack_e3<float>(const double*, float*, long, int, hipStream_t);

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

// A cubic fine element onto its own 8 vertices: W[a][b] = trilinear weight
// of vertex b at local node a (positions 0..3 of 3 per axis), KE = W^T Kc W
// with Kc (192x192, supported rows and columns already zero) read from
// global memory: T = Kc W (192 x 24) in LDS, then W^T T.
__global__ __launch_bounds__(BS) void k_galerkin_e3(const double* __restrict__ Kc, int ncx, int ncy,
                                                    double* KE, const int* __restrict__ elist) {
  __shared__ double sT[L3_ND * 24];
  __shared__ double sW[64 * 8];
  const long E_id = elist ? elist[blockIdx.x] : blockIdx.x;
  for (int t = threadIdx.x; t < 64 * 8; t += BS) {
    const int a = t / 8, b = t % 8;
    const int ax = a % 4, ay = (a / 4) % 4, az = a / 16;
    auto w1 = [](int pos, int bit) { return bit ? pos / 3.0 : (3 - pos) / 3.0; };
    sW[t] = w1(ax, b & 1) * w1(ay, (b >> 1) & 1) * w1(az, b >> 2);
  }
  __syncthreads();
  const double* K = Kc + (size_t)E_id * L3_ND * L3_ND;
  for (int t = threadIdx.x; t < L3_ND * 24; t += BS) {
    const int row = t / 24, col = t % 24;
    const int b = col / 3, j = col % 3;
    double acc = 0.0;
    for (int a2 = 0; a2 < 64; ++a2) acc += K[(size_t)row * L3_ND + 3 * a2 + j] * sW[a2 * 8 + b];
    sT[t] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 576; t += BS) {
    const int row = t / 24, col = t % 24;
    const int b = row / 3, i = row % 3;
    double acc = 0.0;
    for (int a = 0; a < 64; ++a) acc += sW[a * 8 + b] * sT[(3 * a + i) * 24 + col];
    KE[(size_t)E_id * 576 + t] = acc;
  }
  (void)ncx;
  (void)ncy;
}

void setup_galerkin(int src_kind, Lat fine, const double* E, const double* K0, const double* Kc,
                    const uint8_t* mask_f, int ncx, int ncy, int ncz, double* KE,
                    const int* elist, int n_elist, hipStream_t st) {
  const long nce = elist ? n_elist : (long)ncx * ncy * ncz;
  if (nce <= 0) return;
  if (src_kind == OP_EQ3)
    hipLaunchKernelGGL(k_galerkin_e3, dim3((unsigned)nce), dim3(BS), 0, st, Kc, ncx, ncy, KE, elist);
  else
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

// Jacobi data of the stored operators of degree P = 2 or 3: the row of a
// node couples the nodes within P lattice steps; entries shared by several
// elements are summed before taking absolute values.
template <typename T, int P>
__global__ __launch_bounds__(BS) void k_diag_ep(Lat L, const double* __restrict__ Ke,
                                                const uint8_t* __restrict__ mask, T* wD,
                                                double* diag64, double omega, double theta) {
  constexpr int P1 = P + 1, ND = 3 * P1 * P1 * P1, W = 2 * P + 1, CENTER = (W * W * W) / 2;
  const long node = (long)blockIdx.x * BS + threadIdx.x;
  if (node >= L.nn()) return;
  const int i = (int)(node % L.nx), j = (int)((node / L.nx) % L.ny), k = (int)(node / ((long)L.nx * L.ny));
  const int nex = (L.nx - 1) / P, ney = (L.ny - 1) / P, nez = (L.nz - 1) / P;
  int exs[2], axs[2], nxe = 0, eys[2], ays[2], nye = 0, ezs[2], azs[2], nze = 0;
  auto axis = [](int p, int ne, int* es, int* as, int& n) {
    n = 0;
    const int q = p / P, m = p - P * q;
    if (m) { es[0] = q; as[0] = m; n = 1; }
    else {
      if (q - 1 >= 0) { es[n] = q - 1; as[n] = P; ++n; }
      if (q < ne) { es[n] = q; as[n] = 0; ++n; }
    }
  };
  axis(i, nex, exs, axs, nxe);
  axis(j, ney, eys, ays, nye);
  axis(k, nez, ezs, azs, nze);
  const uint8_t mi = mask[node];
  double rs[3] = {0.0, 0.0, 0.0}, dg[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < W * W * W; ++q) {
    const int dx = q % W - P, dy = (q / W) % W - P, dz = q / (W * W) - P;
    double blk[9];
    for (int t = 0; t < 9; ++t) blk[t] = 0.0;
    bool any = false;
    for (int cz = 0; cz < nze; ++cz)
      for (int cy = 0; cy < nye; ++cy)
        for (int cx = 0; cx < nxe; ++cx) {
          const int bx = axs[cx] + dx, by = ays[cy] + dy, bz = azs[cz] + dz;
          if ((unsigned)bx > (unsigned)P || (unsigned)by > (unsigned)P || (unsigned)bz > (unsigned)P)
            continue;
          any = true;
          const long e = exs[cx] + (long)nex * (eys[cy] + (long)ney * ezs[cz]);
          const int a = axs[cx] + P1 * (ays[cy] + P1 * azs[cz]), bb = bx + P1 * (by + P1 * bz);
          for (int c = 0; c < 3; ++c)
            for (int e2 = 0; e2 < 3; ++e2)
              blk[3 * c + e2] += Ke[(size_t)e * ND * ND + (size_t)(3 * a + c) * ND + 3 * bb + e2];
        }
    if (!any) continue;
    for (int c = 0; c < 3; ++c)
      for (int e2 = 0; e2 < 3; ++e2) {
        double v = blk[3 * c + e2];  // supported rows/columns are zero in Ke
        if (q == CENTER && c == e2 && ((mi >> c) & 1)) v = 1.0;
        rs[c] += fabs(v);
        if (q == CENTER && c == e2) dg[c] = v;
      }
  }
  for (int c = 0; c < 3; ++c)
    jacobi_row<T>((mi >> c) & 1, dg[c], rs[c], omega, theta, wD, diag64, 3 * node + c);
}

template <typename T>
void setup_diag_eq2(Lat L, const double* Ke, const uint8_t* mask, T* wD, double* diag64,
                    double omega, double theta, hipStream_t st) {
  hipLaunchKernelGGL((k_diag_ep<T, 2>), dim3(nblocks(L.nn())), dim3(BS), 0, st, L, Ke, mask, wD,
                     diag64, omega, theta);
  MGCG_HIP(hipGetLastError());
}
template void setup_diag_eq2<double>(Lat, const double*, const uint8_t*, double*, double*, double,
                                     double, hipStream_t);
template void setup_diag_eq2<float>(Lat, const double*, const uint8_t*, float*, double*, double,
                                    double, hipStream_t);

template <typename T>
void setup_diag_e3(Lat L, const double* Ke, const uint8_t* mask, T* wD, double* diag64,
                   double omega, double theta, hipStream_t st) {
  hipLaunchKernelGGL((k_diag_ep<T, 3>), dim3(nblocks(L.nn())), dim3(BS), 0, st, L, Ke, mask, wD,
                     diag64, omega, theta);
  MGCG_HIP(hipGetLastError());
}
template void setup_diag_e3<double>(Lat, const double*, const uint8_t*, double*, double*, double,
                                    double, hipStream_t);
template void setup_diag_e3<float>(Lat, const double*, const uint8_t*, float*, double*, double,
                                   double, hipStream_t);

// ------------------------------------------------------------ coarsest level
// Dense operator of the coarsest level (row-major, stride ld) from its
// Q1-type FP64 element matrices (src OP_MF_Q1: E_e K0; otherwise KE[e]): one
// thread per free DOF accumulates the contributions of the elements around
// its node into its row, so every entry has a single writer; columns of
// fixed DOFs are skipped (A must be zeroed before).
__global__ __launch_bounds__(BS) void k_dense(int src_kind, Lat L, const double* __restrict__ E,
                                              const double* __restrict__ K0,
                                              const double* __restrict__ KE,
                                              const int* __restrict__ freedof,
                                              const int* __restrict__ dofpos, int nfree, int ld,
                                              double* A) {
  const int I = blockIdx.x * BS + threadIdx.x;
  if (I >= nfree) return;
  const int gdof = freedof[I];
  const long node = gdof / 3;
  const int c = gdof % 3;
  const int i = (int)(node % L.nx), j = (int)((node / L.nx) % L.ny), k = (int)(node / ((long)L.nx * L.ny));
  const int ex1 = L.nx - 1, ey1 = L.ny - 1, ez1 = L.nz - 1;
  double* row = A + (size_t)gdof * ld;
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
        if (dofpos[3 * nb + e2] < 0) continue;  // fixed column
        const int kk = (3 * a + c) * 24 + 3 * b + e2;
        const double v = src_kind == OP_MF_Q1 ? E[e] * K0[kk] : KE[(size_t)e * 576 + kk];
        row[3 * nb + e2] += v;
      }
    }
  }
}

// Unit diagonal on fixed DOFs and on the padding rows.
__global__ void k_dense_unit(const int* __restrict__ dofpos, long ndof, int ld, double* A) {
  const int g = blockIdx.x * BS + threadIdx.x;
  if (g >= ld) return;
  if (g >= ndof || dofpos[g] < 0) A[(size_t)g * ld + g] = 1.0;
}

void setup_dense(int src_kind, Lat L, const double* E, const double* K0, const double* KE,
                 const int* freedof, const int* dofpos, int nfree, int ld, double* A,
                 hipStream_t st) {
  fill<double>(A, 0.0, (long)ld * ld, st);
  if (nfree > 0) {
    hipLaunchKernelGGL(k_dense, dim3(nblocks(nfree)), dim3(BS), 0, st, src_kind, L, E, K0, KE,
                       freedof, dofpos, nfree, ld, A);
    MGCG_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_dense_unit, dim3(nblocks(ld)), dim3(BS), 0, st, dofpos, L.ndof(), ld, A);
  MGCG_HIP(hipGetLastError());
}

// ------------------------------------------------------------ coarsest inverse
// Blocked Gauss-Jordan elimination: sweeping pivot block k maps
//   A_kk -> D = A_kk^{-1},  A_kj -> D A_kj,  A_ik -> -A_ik D,
//   A_ij -> A_ij - A_ik D A_kj          (i, j != k),
// and after all blocks the matrix holds A^{-1}.  For a symmetric positive
// definite A every pivot block is a Schur complement of A, hence SPD itself:
// no pivoting is needed, and a pivot that is not clearly positive (relative
// to the original diagonal entry) means A is singular or indefinite.

__global__ void k_diag0(const double* __restrict__ A, int ld, double* diag0) {
  const int g = blockIdx.x * BS + threadIdx.x;
  if (g < ld) diag0[g] = A[(size_t)g * ld + g];
}

// D = A_kk^{-1} by unblocked Gauss-Jordan in LDS (one thread per entry).
__global__ __launch_bounds__(GJ_B * GJ_B) void k_gj_diag(const double* __restrict__ A, int ld,
                                                          int k, const double* __restrict__ diag0,
                                                          double* D, int* bad) {
  __shared__ double M[GJ_B][GJ_B + 1];
  const int r = threadIdx.x / GJ_B, c = threadIdx.x % GJ_B;
  const int k0 = k * GJ_B;
  M[r][c] = A[(size_t)(k0 + r) * ld + k0 + c];
  __syncthreads();
  for (int p = 0; p < GJ_B; ++p) {
    double piv = M[p][p];
    if (!(piv > 1e-13 * diag0[k0 + p]) || !isfinite(piv)) {
      if (threadIdx.x == 0) atomicOr(bad, 2);
      piv = 1.0;
    }
    const double ip = 1.0 / piv;
    double v;
    if (r == p && c == p)
      v = ip;
    else if (r == p)
      v = ip * M[p][c];
    else if (c == p)
      v = -M[r][p] * ip;
    else
      v = M[r][c] - M[r][p] * ip * M[p][c];
    __syncthreads();
    M[r][c] = v;
    __syncthreads();
  }
  D[r * GJ_B + c] = M[r][c];
}

// Tile (I, J) of the matrix after sweeping block k: reads A, writes B.
__global__ __launch_bounds__(BS) void k_gj_update(const double* __restrict__ A, double* B, int ld,
                                                  int k, const double* __restrict__ D) {
  __shared__ double sD[GJ_B][GJ_B + 1], sR[GJ_B][GJ_B + 1], sC[GJ_B][GJ_B + 1],
      sT[GJ_B][GJ_B + 1];
  const int I = blockIdx.y, J = blockIdx.x;
  const int c = threadIdx.x % GJ_B, r0 = threadIdx.x / GJ_B;  // rows r0 + 8 q
  constexpr int RS = BS / GJ_B;
  const size_t k0 = (size_t)k * GJ_B, i0 = (size_t)I * GJ_B, j0 = (size_t)J * GJ_B;
  for (int q = 0; q < GJ_B / RS; ++q) {
    const int r = r0 + RS * q;
    sD[r][c] = D[r * GJ_B + c];
    sR[r][c] = A[(k0 + r) * ld + j0 + c];  // A_kJ
    sC[r][c] = A[(i0 + r) * ld + k0 + c];  // A_Ik
  }
  __syncthreads();
  if (I == k && J == k) {
    for (int q = 0; q < GJ_B / RS; ++q) {
      const int r = r0 + RS * q;
      B[(i0 + r) * ld + j0 + c] = sD[r][c];
    }
    return;
  }
  if (I == k) {  // D A_kJ
    for (int q = 0; q < GJ_B / RS; ++q) {
      const int r = r0 + RS * q;
      double s = 0.0;
      for (int m = 0; m < GJ_B; ++m) s += sD[r][m] * sR[m][c];
      B[(i0 + r) * ld + j0 + c] = s;
    }
    return;
  }
  if (J == k) {  // -A_Ik D
    for (int q = 0; q < GJ_B / RS; ++q) {
      const int r = r0 + RS * q;
      double s = 0.0;
      for (int m = 0; m < GJ_B; ++m) s += sC[r][m] * sD[m][c];
      B[(i0 + r) * ld + j0 + c] = -s;
    }
    return;
  }
  // A_IJ - A_Ik (D A_kJ)
  double aij[GJ_B / RS];
  for (int q = 0; q < GJ_B / RS; ++q) aij[q] = A[(i0 + r0 + RS * q) * ld + j0 + c];
  for (int q = 0; q < GJ_B / RS; ++q) {
    const int r = r0 + RS * q;
    double s = 0.0;
    for (int m = 0; m < GJ_B; ++m) s += sD[r][m] * sR[m][c];
    sT[r][c] = s;
  }
  __syncthreads();
  for (int q = 0; q < GJ_B / RS; ++q) {
    const int r = r0 + RS * q;
    double s = 0.0;
    for (int m = 0; m < GJ_B; ++m) s += sC[r][m] * sT[m][c];
    B[(i0 + r) * ld + j0 + c] = aij[q] - s;
  }
}

double* setup_coarse_inverse(double* A, double* B, double* D, double* diag0, int ld, int* bad,
                             hipStream_t st) {
  const int nb = ld / GJ_B;
  hipLaunchKernelGGL(k_diag0, dim3(nblocks(ld)), dim3(BS), 0, st, A, ld, diag0);
  MGCG_HIP(hipGetLastError());
  for (int k = 0; k < nb; ++k) {
    hipLaunchKernelGGL(k_gj_diag, dim3(1), dim3(GJ_B * GJ_B), 0, st, A, ld, k, diag0, D, bad);
    MGCG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gj_update, dim3(nb, nb), dim3(BS), 0, st, A, B, ld, k, D);
    MGCG_HIP(hipGetLastError());
    std::swap(A, B);
  }
  return A;
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
// One thread per (sub-element s, displacement element e); s = blockIdx.y is
// uniform, so the sub-element matrix Ksub[s] is read through scalar loads:
//   dc = -p rho^{p-1} (E0 - Emin) sum_l u_{l,e}^T K^(e_s) u_{l,e}.
// ue[i] for a run-time i without dynamic register indexing.
template <int N>
__device__ __forceinline__ double select_row(const double (&v)[N], int i) {
  double out = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) out = (k == i) ? v[k] : out;
  return out;
}

template <int ORDER>
__global__ __launch_bounds__(BS) void k_sens(int nsub, int nelx, int nely, int nelz, Lat L,
                                             const double* __restrict__ rho,
                                             const double* __restrict__ u, long ndof, int nrhs,
                                             const double* __restrict__ Ksub, double E0mEmin,
                                             double penal, double* dc) {
  constexpr int P1 = ORDER + 1, NEN = P1 * P1 * P1, ND = 3 * NEN;
  const long nel = (long)nelx * nely * nelz;
  const long e = (long)blockIdx.x * BS + threadIdx.x;
  if (e >= nel) return;
  const int s = blockIdx.y;
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
    // rows one at a time (a row of K in scalar registers), u^T (K u)
#pragma unroll 1
    for (int i = 0; i < ND; ++i) {
      double ti = 0.0;
#pragma unroll
      for (int jj = 0; jj < ND; ++jj) ti += K[i * ND + jj] * ue[jj];
      w += select_row(ue, i) * ti;
    }
  }
  const int sx = s % nsub, sy = (s / nsub) % nsub, sz = s / (nsub * nsub);
  const long di = (nsub * ex + sx) + (long)(nsub * nelx) * ((nsub * ey + sy) + (long)(nsub * nely) * (nsub * ez + sz));
  const double r = rho[di];
  dc[di] = -penal * pow(r, penal - 1.0) * E0mEmin * w;
}

// With 4^3 sub-elements (and for cubic elements with any n^3 <= 64, the
// columns past n^3 zero) the quadratic forms of an element are one
// contraction: w_s = sum_l u_l^T K_s u_l = sum_{i <= j} U[k(i,j)] Kp[k(i,j)][s]
// with U = sum_l u_l u_l^T (symmetric, packed row by row, i <= j) and Kp[k][s]
// = K_s[i][j] times 2 off the diagonal (built once per mesh, sens_pack).
// Over a block of SP_EL = 16 elements this is a (16 x NK) by (NK x 64)
// product, run on the FP64 matrix cores (16x16x4 MFMA): the elements are the
// rows, the 64 sub-elements four column tiles (tile t, column n holds
// s = 4 n + t, so a lane's four B values are one 32-byte segment of a Kp
// row), four packed pairs per step.  A lane forms its A value U[e][k] from
// u_e staged in LDS, at the LDS offsets of (i, j) that a table beside Kp
// holds; Kp streams from L2 (1.7 MB for Q2) in chunks of SP_PF steps, one
// chunk ahead, in two register sets that alternate.  For Q2 the block's
// WPB = 4 waves split the packed pairs and add their tiles in a fixed order.
// Kp and the table are padded (zero rows, offset 0) to an even number of
// chunks per wave plus the prefetch overrun.  For cubic elements (18,528
// pairs) the table stays in global memory and each chunk's offsets are
// fetched with its Kp values: with u_e of four load cases staged, LDS could
// not hold both.
constexpr int SP_EL = 16;  // elements per block
constexpr int SP_PF = 4;   // steps per Kp chunk
template <int ORDER>
struct SensShape {
  static constexpr int ND = 3 * (ORDER + 1) * (ORDER + 1) * (ORDER + 1);
  static constexpr int NK = ND * (ND + 1) / 2;
  static constexpr int WPB = ORDER == 1 ? 1 : 4;
  static constexpr int QUANT = 4 * WPB * SP_PF * 2;
  static constexpr int NKP = (NK + QUANT - 1) / QUANT * QUANT;  // pairs the waves walk
  static constexpr int STEPS = NKP / (4 * WPB);                 // steps per wave
  static constexpr int ROWS = NKP + 4 * SP_PF;                  // + the prefetch overrun
};

static long sens_rows(int order) {
  return order == 1 ? SensShape<1>::ROWS : order == 2 ? SensShape<2>::ROWS : SensShape<3>::ROWS;
}

long sens_packed_doubles(int order) {
  const long rows = sens_rows(order);
  return rows * 64 + rows / 2;  // Kp rows, then one 32-bit offset pair per row
}

void sens_pack(int order, int nsub, const double* Ksub, std::vector<double>& out) {
  const int nd = order == 1 ? SensShape<1>::ND : order == 2 ? SensShape<2>::ND : SensShape<3>::ND;
  const long rows = sens_rows(order);
  const int ns3 = nsub * nsub * nsub;
  if (ns3 > 64) throw Error(-1, "at most 64 sub-elements");
  out.assign((size_t)sens_packed_doubles(order), 0.0);
  uint32_t* tab = reinterpret_cast<uint32_t*>(out.data() + rows * 64);
  long k = 0;
  for (int i = 0; i < nd; ++i)
    for (int j = i; j < nd; ++j, ++k) {
      for (int s = 0; s < ns3; ++s)
        out[(size_t)k * 64 + s] = (i == j ? 1.0 : 2.0) * Ksub[(size_t)s * nd * nd + (size_t)i * nd + j];
      // byte offsets of u[i] and u[j] in the staged [DOF][element] block
      tab[k] = (uint32_t)(i * SP_EL * 8) | ((uint32_t)(j * SP_EL * 8) << 16);
    }
}

typedef double v4d __attribute__((ext_vector_type(4)));

template <int ORDER, int NRHS>
__global__ __launch_bounds__(64 * SensShape<ORDER>::WPB) void k_sens_mfma(
    int nelx, int nely, int nelz, int nsub, Lat L, const double* __restrict__ rho,
    const double* __restrict__ u, long ndof, const double* __restrict__ Kp, double E0mEmin,
    double penal, double* __restrict__ dc) {
  using S = SensShape<ORDER>;
  constexpr int P1 = ORDER + 1, ND = S::ND, WPB = S::WPB, NT = 64 * WPB;
  constexpr int NU = NRHS * ND * SP_EL, NR = WPB * SP_EL * 64;
  constexpr int NCH = S::STEPS / SP_PF;  // chunks per wave (even)
  constexpr bool TAB_LDS = ORDER < 3;
  static_assert(NCH % 2 == 0, "two alternating register sets");
  static_assert(ND * SP_EL * 8 < 65536, "16-bit LDS offsets");
  __shared__ double sh[NU > NR ? NU : NR];
  __shared__ uint32_t tab[TAB_LDS ? S::NKP : 1];
  const long nel = (long)nelx * nely * nelz;
  const long e0 = (long)blockIdx.x * SP_EL;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint32_t* tabg = reinterpret_cast<const uint32_t*>(Kp + (size_t)S::ROWS * 64);
  if constexpr (TAB_LDS)
    for (int q = t; q < S::NKP; q += NT) tab[q] = tabg[q];
  // u_e of the block's elements, [load case][local DOF][element]; elements
  // past the mesh read 0
  for (int q = t; q < NU; q += NT) {
    const int m = q & (SP_EL - 1), d = (q / SP_EL) % ND, r = q / (SP_EL * ND);
    const long e = e0 + m;
    double v = 0.0;
    if (e < nel) {
      const int ex = (int)(e % nelx), ey = (int)((e / nelx) % nely),
                ez = (int)(e / ((long)nelx * nely));
      const int a = d / 3, c = d % 3;
      const int ax = a % P1, ay = (a / P1) % P1, az = a / (P1 * P1);
      const long node =
          (ORDER * ex + ax) + (long)L.nx * ((ORDER * ey + ay) + (long)L.ny * (ORDER * ez + az));
      v = u[(size_t)r * ndof + 3 * node + c];
    }
    sh[q] = v;
  }
  __syncthreads();
  // lane (m, kk): A row m (element e0 + m) and B column m (sub-elements
  // 4 m .. 4 m + 3, one per tile) at pair k0 + 4 step + kk
  const int m = lane & 15, kk = lane >> 4;
  const int k0 = w * S::STEPS * 4 + kk;
  const char* ub = reinterpret_cast<const char*>(sh) + m * 8;
  const double4* kb = reinterpret_cast<const double4*>(Kp) + (size_t)k0 * 16 + m;
  v4d acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  auto fetch = [&](double4* b, uint32_t* ijg, int c) {
#pragma unroll
    for (int p = 0; p < SP_PF; ++p) {
      b[p] = kb[(size_t)(c * SP_PF + p) * 64];
      if constexpr (!TAB_LDS) ijg[p] = tabg[k0 + 4 * (c * SP_PF + p)];
    }
  };
  auto run = [&](const double4* b, const uint32_t* ijg, int c) {
#pragma unroll
    for (int p = 0; p < SP_PF; ++p) {
      const uint32_t ij = TAB_LDS ? tab[k0 + 4 * (c * SP_PF + p)] : ijg[p];
      const int oi = (int)(ij & 0xffffu), oj = (int)(ij >> 16);
      double a = 0.0;
#pragma unroll
      for (int r = 0; r < NRHS; ++r)
        a = fma(*reinterpret_cast<const double*>(ub + oi + r * ND * SP_EL * 8),
                *reinterpret_cast<const double*>(ub + oj + r * ND * SP_EL * 8), a);
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[p].x, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[p].y, acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[p].z, acc[2], 0, 0, 0);
      acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[p].w, acc[3], 0, 0, 0);
    }
  };
  double4 b0[SP_PF], b1[SP_PF];
  uint32_t i0[SP_PF], i1[SP_PF];
  fetch(b0, i0, 0);
  for (int c = 0; c < NCH; c += 2) {
    fetch(b1, i1, c + 1);
    run(b0, i0, c);
    fetch(b0, i0, c + 2);  // (the last one reads the zero overrun rows)
    run(b1, i1, c + 1);
  }
  __syncthreads();  // every wave is done with the staged u
  // result value v of a lane is row kk + 4 v, column m of its tile (the
  // FP64 16x16x4 output layout): w[s][element] per wave
  double* red = sh + w * SP_EL * 64;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[(4 * m + q) * SP_EL + kk + 4 * v] = acc[q][v];
  __syncthreads();
  // outputs in density-lattice order within each (sy, sz) row: sub-element
  // x fastest, then element
  const int n = nsub;
  for (int q = t; q < SP_EL * n * n * n; q += NT) {
    const int sx = q % n, mm = (q / n) % SP_EL, syz = q / (n * SP_EL);
    const int s = sx + n * syz;
    double v = 0.0;
#pragma unroll
    for (int ww = 0; ww < WPB; ++ww) v += sh[ww * SP_EL * 64 + s * SP_EL + mm];
    const long e = e0 + mm;
    if (e >= nel) continue;
    const int ex = (int)(e % nelx), ey = (int)((e / nelx) % nely), ez = (int)(e / ((long)nelx * nely));
    const int sy = syz % n, sz = syz / n;
    const long di =
        (n * ex + sx) + (long)(n * nelx) * ((n * ey + sy) + (long)(n * nely) * (n * ez + sz));
    dc[di] = -penal * pow(rho[di], penal - 1.0) * E0mEmin * v;
  }
}

template <int ORDER>
static void launch_sens_mfma(int nelx, int nely, int nelz, int nsub, Lat L, const double* rho,
                             const double* u, long ndof, int nrhs, const double* Kp,
                             double E0mEmin, double penal, double* dc, hipStream_t st) {
  const dim3 g(nblocks((long)nelx * nely * nelz, SP_EL)), b(64 * SensShape<ORDER>::WPB);
  auto kern = nrhs == 1   ? k_sens_mfma<ORDER, 1>
              : nrhs == 2 ? k_sens_mfma<ORDER, 2>
              : nrhs == 3 ? k_sens_mfma<ORDER, 3>
                          : k_sens_mfma<ORDER, 4>;
  hipLaunchKernelGGL(kern, g, b, 0, st, nelx, nely, nelz, nsub, L, rho, u, ndof, Kp, E0mEmin,
                     penal, dc);
}

void sens_kernel(int order, int nsub, int nelx, int nely, int nelz, Lat L, const double* rho,
                 const double* u, long ndof, int nrhs, const double* Ksub, const double* Kp,
                 double E0mEmin, double penal, double* dc, hipStream_t st) {
  if (order == 3) {
    if (!Kp) throw Error(-1, "cubic elements need the packed sub-element matrices");
    launch_sens_mfma<3>(nelx, nely, nelz, nsub, L, rho, u, ndof, nrhs, Kp, E0mEmin, penal, dc, st);
    MGCG_HIP(hipGetLastError());
    return;
  }
  if (nsub == 4 && Kp) {
    if (order == 1)
      launch_sens_mfma<1>(nelx, nely, nelz, 4, L, rho, u, ndof, nrhs, Kp, E0mEmin, penal, dc, st);
    else
      launch_sens_mfma<2>(nelx, nely, nelz, 4, L, rho, u, ndof, nrhs, Kp, E0mEmin, penal, dc, st);
    MGCG_HIP(hipGetLastError());
    return;
  }
  const dim3 grid(nblocks((long)nelx * nely * nelz), nsub * nsub * nsub);
  if (order == 1)
    hipLaunchKernelGGL(k_sens<1>, grid, dim3(BS), 0, st, nsub, nelx, nely, nelz, L, rho, u, ndof,
                       nrhs, Ksub, E0mEmin, penal, dc);
  else
    hipLaunchKernelGGL(k_sens<2>, grid, dim3(BS), 0, st, nsub, nelx, nely, nelz, L, rho, u, ndof,
                       nrhs, Ksub, E0mEmin, penal, dc);
  MGCG_HIP(hipGetLastError());
}

}  // namespace mgcg
