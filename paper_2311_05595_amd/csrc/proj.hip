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
#include <cmath>
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
  return g;
}

size_t Proj::device_bytes(const mgcg_proj_desc& d) {
  const ProjGeom g = geometry(d);
  return ((size_t)g.nrho + (size_t)g.ntab) * sizeof(double);
}

Proj::Proj(const mgcg_proj_desc& d, int device) : g_(geometry(d)), device_(device) {
  MGCG_HIP(hipSetDevice(device_));
  const double c = 9.0 / (8.0 * (double)g_.n * g_.n * g_.d * g_.d * d.rmin * d.rmin);
  std::vector<double> tab(g_.ntab);
  for (int m = 0; m < g_.ntab; ++m) tab[m] = std::exp(-c * (double)m * (double)m);
  try {
    if (hipMalloc(&invw_, (size_t)g_.nrho * sizeof(double)) != hipSuccess ||
        hipMalloc(&tab_, tab.size() * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(MGCG_ENOMEM, "projection allocation failed");
    }
    MGCG_HIP(hipMemcpyAsync(tab_, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice,
                            stream_));
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
  invw_ = tab_ = nullptr;
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
  const int nb = (int)((nout + PROJ_BS - 1) / PROJ_BS);
  if (transpose)
    hipLaunchKernelGGL(k_proj_t, dim3(nb), dim3(PROJ_BS), 0, stream_, args_of(g_, tab_), din,
                       (const double*)invw_, dout);
  else
    hipLaunchKernelGGL(k_proj_fwd<false>, dim3(nb), dim3(PROJ_BS), 0, stream_, args_of(g_, tab_),
                       din, (const double*)invw_, dout);
  MGCG_HIP(hipGetLastError());
  if (mem == MGCG_MEM_HOST) {
    MGCG_HIP(hipMemcpyAsync(out, dout, (size_t)nout * sizeof(double), hipMemcpyDeviceToHost,
                            stream_));
    MGCG_HIP(hipStreamSynchronize(stream_));
  }
}

}  // namespace mgcg
