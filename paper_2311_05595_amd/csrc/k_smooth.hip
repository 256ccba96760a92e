// Multicolour Gauss-Seidel smoothing on a quadratic or cubic finest level.
//
// Sec. 7.5 smooths quadratic and cubic elements by SSOR.  Its sweeps are
// sequential; here the nodes of the lattice of degree P are coloured by
// (i mod (P+1), j mod (P+1), k mod (P+1)).  Two nodes of one colour are
// P + 1 or more lattice steps apart along some axis, while an element spans
// P, so they share no element, their rows do not couple, and all nodes of a
// colour are updated at once from the latest values.  A forward sweep takes
// colours 0 .. (P+1)^3 - 1 (colour c = ci + (P+1) cj + (P+1)^2 ck) and a
// node's components x, y, z in that order; the backward sweep reverses
// both.  The result is a Gauss-Seidel sweep (relaxation 1) in that ordering
// of the DOFs.
//
// A group of lanes per node (32 for the 27-node element, a wave for the
// 64-node one): its 1, 2, 4 or 8 elements' rows of the node (3 x ND values
// each, ND = 81 or 192, stored by node so that they are contiguous) times
// the element's ND values of x, split over the lanes, one local node per
// lane; the three row sums are summed across the group, then one lane
// updates the node's components in order, each from the sums corrected by
// the components already updated (with the node's 3x3 diagonal block,
// precomputed at refresh).  Fixed DOFs (zero rows and columns in the element
// matrices) are skipped and stay 0.
#include "devutil.h"
#include "kernels.h"

namespace mgcg {

template <int P>
struct GsShape {
  static constexpr int M = P + 1;                  // colours per axis
  static constexpr int NEN = M * M * M;            // nodes per element
  static constexpr int ND = 3 * NEN;               // DOFs per element
  static constexpr int LPN = NEN <= 32 ? 32 : 64;  // lanes per node
};
constexpr int GS_WAVES = 4;  // waves per block

template <typename T, int P>
__global__ __launch_bounds__(BS) void k_rows_by_node(const double* __restrict__ Keff, T* Kn,
                                                     long nel) {
  constexpr int ND = GsShape<P>::ND, ND2 = ND * ND;
  const long n = nel * ND2;
  for (long q = (long)blockIdx.x * BS + threadIdx.x; q < n; q += (long)gridDim.x * BS) {
    const long e = q / ND2;
    const int w = (int)(q - e * ND2);
    const int a = w / (3 * ND), rem = w - 3 * ND * a, j = rem / 3, c = rem - 3 * j;
    Kn[q] = (T)Keff[e * ND2 + (3 * a + c) * ND + j];
  }
}

template <typename T>
void setup_rows_by_node(int order, const double* Keff, T* Kn, long nel, hipStream_t st) {
  const int nd = order == 3 ? GsShape<3>::ND : GsShape<2>::ND;
  long nb = (nel * nd * nd + BS - 1) / BS;
  if (nb > 65536) nb = 65536;
  if (order == 3)
    hipLaunchKernelGGL((k_rows_by_node<T, 3>), dim3((int)nb), dim3(BS), 0, st, Keff, Kn, nel);
  else
    hipLaunchKernelGGL((k_rows_by_node<T, 2>), dim3((int)nb), dim3(BS), 0, st, Keff, Kn, nel);
  MGCG_HIP(hipGetLastError());
}
template void setup_rows_by_node<double>(int, const double*, double*, long, hipStream_t);
template void setup_rows_by_node<float>(int, const double*, float*, long, hipStream_t);

// Sum over the LPN lanes of a node's group (every lane of the group gets it).
template <int LPN, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = LPN / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LPN);
  return v;
}

// Elements along one axis that contain node index i of a lattice of degree
// P with ne elements: the first one and how many (1 or 2).
template <int P>
__device__ __forceinline__ void gs_axis(int i, int ne, int& e0, int& cnt) {
  const int q = i / P;
  if (i - P * q) {
    e0 = q;
    cnt = 1;
  } else {
    e0 = q - 1;
    cnt = 2;
    if (e0 < 0) {
      e0 = 0;
      cnt = 1;
    }
    if (e0 + cnt > ne) cnt = ne - e0;
  }
}

// Each node's 3x3 diagonal block, summed over its elements:
// Dn[node * 9 + 3 c + c'] = A[3 node + c][3 node + c'].
template <typename T, int P>
__global__ __launch_bounds__(BS) void k_gs_diag(Lat L, const T* __restrict__ Kn, T* Dn) {
  using S = GsShape<P>;
  const int node = blockIdx.x * BS + threadIdx.x;
  if (node >= (int)L.nn()) return;
  const int i = node % L.nx, j = (node / L.nx) % L.ny, k = node / (L.nx * L.ny);
  const int nex = (L.nx - 1) / P, ney = (L.ny - 1) / P, nez = (L.nz - 1) / P;
  int ex0, cx, ey0, cy, ez0, cz;
  gs_axis<P>(i, nex, ex0, cx);
  gs_axis<P>(j, ney, ey0, cy);
  gs_axis<P>(k, nez, ez0, cz);
  T d[9];
#pragma unroll
  for (int v = 0; v < 9; ++v) d[v] = T(0);
  for (int ez = ez0; ez < ez0 + cz; ++ez)
    for (int ey = ey0; ey < ey0 + cy; ++ey)
      for (int ex = ex0; ex < ex0 + cx; ++ex) {
        const int e = ex + nex * (ey + ney * ez);
        const int an = (i - P * ex) + S::M * ((j - P * ey) + S::M * (k - P * ez));
        const T* kr = Kn + ((size_t)(e * S::NEN + an) * S::ND + 3 * an) * 3;  // [column c'][row c]
#pragma unroll
        for (int cp = 0; cp < 3; ++cp)
#pragma unroll
          for (int c = 0; c < 3; ++c) d[3 * c + cp] += kr[3 * cp + c];
      }
#pragma unroll
  for (int v = 0; v < 9; ++v) Dn[(size_t)node * 9 + v] = d[v];
}

template <typename T>
void setup_gs_diag(int order, const Lat& L, const T* Kn, T* Dn, hipStream_t st) {
  if (order == 3)
    hipLaunchKernelGGL((k_gs_diag<T, 3>), dim3(nblocks(L.nn())), dim3(BS), 0, st, L, Kn, Dn);
  else
    hipLaunchKernelGGL((k_gs_diag<T, 2>), dim3(nblocks(L.nn())), dim3(BS), 0, st, L, Kn, Dn);
  MGCG_HIP(hipGetLastError());
}
template void setup_gs_diag<double>(int, const Lat&, const double*, double*, hipStream_t);
template void setup_gs_diag<float>(int, const Lat&, const float*, float*, hipStream_t);

// One colour of a sweep.  Lane gl < NEN of the node's group takes the
// elements' local node aj = gl: for each element of the node (slot (dx, dy,
// dz), up to 8) a 3x3 block of the node's rows (9 contiguous values of Kn)
// against local node aj's 3 values of x.  The loads of SB slots are issued
// before their products (all 8 in FP32); slots past the node's elements,
// and lanes past NEN, read valid data and count 0.
template <typename T, int NR, int P>
__global__ __launch_bounds__(64 * GS_WAVES) void k_gs_colour(Lat L, const T* __restrict__ Kn,
                                                             const T* __restrict__ Dn,
                                                             const uint8_t* __restrict__ mask,
                                                             const T* __restrict__ b, T* x, int ci,
                                                             int cj, int ck, int backward,
                                                             const CgScalars* cs) {
  using S = GsShape<P>;
  constexpr int M = S::M, LPN = S::LPN, NPB = GS_WAVES * 64 / LPN;
  constexpr int SB = sizeof(T) == 4 ? 8 : 4;  // slots per load batch
  const Gate g = gate_load(cs, NR, CG_ACTIVE);
  const int lane = threadIdx.x & 63, gl = lane & (LPN - 1);
  const int mx = (L.nx - ci + M - 1) / M, my = (L.ny - cj + M - 1) / M, mz = (L.nz - ck + M - 1) / M;
  const int nnodes = mx * my * mz;
  const int q0 = blockIdx.x * NPB + (int)threadIdx.x / LPN;
  const bool live = q0 < nnodes;  // the group's node exists (uniform per group)
  const int q = live ? q0 : 0;
  const int qx = q % mx, qy = (q / mx) % my, qz = q / (mx * my);
  const int i = ci + M * qx, j = cj + M * qy, k = ck + M * qz;
  const int nex = (L.nx - 1) / P, ney = (L.ny - 1) / P, nez = (L.nz - 1) / P;
  int ex0, cx, ey0, cy, ez0, cz;
  gs_axis<P>(i, nex, ex0, cx);
  gs_axis<P>(j, ney, ey0, cy);
  gs_axis<P>(k, nez, ez0, cz);
  const long ndof = L.ndof();
  const int node = i + L.nx * (j + L.ny * k);
  const int sxy = L.nx * L.ny;
  // the leader's own operands, loaded with the first batch
  T bo[NR][3], xo[NR][3], dn[9];
  uint8_t m = 0;
  if (gl == 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        bo[r][c] = b[r * ndof + 3 * node + c];
        xo[r][c] = x[r * ndof + 3 * node + c];
      }
#pragma unroll
    for (int v = 0; v < 9; ++v) dn[v] = Dn[(size_t)node * 9 + v];
    m = mask[node];
  }
  // this lane's local node and its offset from an element's first node
  const bool has = gl < S::NEN;
  const int aj = has ? gl : 0;
  const int offn = aj % M + L.nx * ((aj / M) % M) + sxy * (aj / (M * M));
  T acc[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = T(0);
#pragma unroll
  for (int s0 = 0; s0 < 8; s0 += SB) {
    T kv[SB][9], xv[SB][NR][3];
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int sl = s0 + u, dx = sl & 1, dy = (sl >> 1) & 1, dz = sl >> 2;
      const bool sok = dx < cx && dy < cy && dz < cz;
      const int ex = ex0 + (sok ? dx : 0), ey = ey0 + (sok ? dy : 0), ez = ez0 + (sok ? dz : 0);
      const int e = ex + nex * (ey + ney * ez);
      const int an = (i - P * ex) + M * ((j - P * ey) + M * (k - P * ez));  // the node in e
      const int n0 = P * ex + L.nx * P * ey + sxy * P * ez;                 // e's first node
      const T* kb = Kn + (size_t)(e * S::NEN + an) * (3 * S::ND);           // [aj][c'][c]
      const T z = (sok && has) ? T(1) : T(0);
      const T* kr = kb + 9 * aj;
#pragma unroll
      for (int v = 0; v < 9; ++v) kv[u][v] = kr[v] * z;
      const int nj = n0 + offn;
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) xv[u][r][c] = x[r * ndof + 3 * nj + c];
    }
#pragma unroll
    for (int u = 0; u < SB; ++u)
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int cp = 0; cp < 3; ++cp) {
          acc[r][0] = fma(kv[u][3 * cp + 0], xv[u][r][cp], acc[r][0]);
          acc[r][1] = fma(kv[u][3 * cp + 1], xv[u][r][cp], acc[r][1]);
          acc[r][2] = fma(kv[u][3 * cp + 2], xv[u][r][cp], acc[r][2]);
        }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = group_sum<LPN>(acc[r][c]);
  if (!gate_open(g)) return;  // uniform: before the first store
  if (gl == 0 && live) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T s0 = acc[r][0], s1 = acc[r][1], s2 = acc[r][2];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int c = backward ? 2 - t : t;
        if ((m >> c) & 1) continue;
        const T sc = c == 0 ? s0 : c == 1 ? s1 : s2;
        const T dl = (bo[r][c] - sc) / dn[4 * c];
        xo[r][c] += dl;
        s0 = fma(dn[c], dl, s0);
        s1 = fma(dn[3 + c], dl, s1);
        s2 = fma(dn[6 + c], dl, s2);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) x[r * ndof + 3 * node + c] = xo[r][c];
    }
  }
}

template <typename T, int P>
static void gs_sweep(const Lat& L, const T* Kn, const T* Dn, const uint8_t* mask, const T* b, T* x,
                     bool backward, int nrhs, const CgScalars* cs, hipStream_t st) {
  constexpr int M = P + 1, NC = M * M * M, NPB = GS_WAVES * 64 / GsShape<P>::LPN;
  auto kern = nrhs == 1   ? k_gs_colour<T, 1, P>
              : nrhs == 2 ? k_gs_colour<T, 2, P>
              : nrhs == 3 ? k_gs_colour<T, 3, P>
                          : k_gs_colour<T, 4, P>;
  for (int t = 0; t < NC; ++t) {
    const int c = backward ? NC - 1 - t : t;
    const int ci = c % M, cj = (c / M) % M, ck = c / (M * M);
    const long nodes = (long)((L.nx - ci + M - 1) / M) * ((L.ny - cj + M - 1) / M) *
                       ((L.nz - ck + M - 1) / M);
    if (nodes == 0) continue;
    const int nb = (int)((nodes + NPB - 1) / NPB);
    hipLaunchKernelGGL(kern, dim3(nb), dim3(64 * GS_WAVES), 0, st, L, Kn, Dn, mask, b, x, ci, cj,
                       ck, backward ? 1 : 0, cs);
    MGCG_HIP(hipGetLastError());
  }
}

template <typename T>
void v_gauss_seidel(int order, const Lat& L, const T* Kn, const T* Dn, const uint8_t* mask,
                    const T* b, T* x, bool backward, int nrhs, const CgScalars* cs,
                    hipStream_t st) {
  if (order == 3)
    gs_sweep<T, 3>(L, Kn, Dn, mask, b, x, backward, nrhs, cs, st);
  else
    gs_sweep<T, 2>(L, Kn, Dn, mask, b, x, backward, nrhs, cs, st);
}
template void v_gauss_seidel<double>(int, const Lat&, const double*, const double*, const uint8_t*,
                                     const double*, double*, bool, int, const CgScalars*,
                                     hipStream_t);
template void v_gauss_seidel<float>(int, const Lat&, const float*, const float*, const uint8_t*,
                                    const float*, float*, bool, int, const CgScalars*, hipStream_t);

}  // namespace mgcg
