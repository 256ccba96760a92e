// Choice of the variables fixed before the degree of the elements is raised
// (Sec. 6.1).  An element is void when all its densities are <= rho_l and all
// its design-gradient components >= -eps, solid when all densities are
// >= rho_u and all gradient components <= eps; it is fixed when every
// element sharing a node with it (inside the domain) is of its kind.  The
// design variables of fixed elements are fixed, and the nodes of the raised
// degree's lattice whose elements are all fixed void elements lose their
// DOFs.  One thread per element, per design cell and per node; the counts
// come from fixed-order block partials.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fix.h"

namespace mgcg {

namespace {

constexpr int FX_BS = 256;
enum : unsigned char { FX_MIXED = 0, FX_VOID = 1, FX_SOLID = 2 };

struct FixGeom {
  int nelx, nely, nelz, n, d, p;
  __host__ __device__ long nel() const { return (long)nelx * nely * nelz; }
  __host__ __device__ long nrho() const { return nel() * n * n * n; }
  __host__ __device__ long nx() const { return nel() * d * d * d; }
  __host__ __device__ long nnx() const { return (long)p * nelx + 1; }
  __host__ __device__ long nny() const { return (long)p * nely + 1; }
  __host__ __device__ long nnz() const { return (long)p * nelz + 1; }
  __host__ __device__ long nn() const { return nnx() * nny() * nnz(); }
};

// Block partial of one count (thread 0 writes it).
__device__ __forceinline__ long long block_count(int v, long long* sh) {
  long long s = v;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = s;
  __syncthreads();
  long long t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < FX_BS / 64; ++i) t += sh[i];
  return t;
}

__global__ __launch_bounds__(FX_BS) void k_fix_classify(FixGeom g, const double* __restrict__ rho,
                                                        const double* __restrict__ grad,
                                                        double rho_l, double rho_u, double eps,
                                                        unsigned char* __restrict__ kind) {
  const long e = (long)blockIdx.x * FX_BS + threadIdx.x;
  if (e >= g.nel()) return;
  const int ex = (int)(e % g.nelx), ey = (int)((e / g.nelx) % g.nely), ez = (int)(e / ((long)g.nelx * g.nely));
  bool lo = true, hi = true;
  const long X = (long)g.n * g.nelx, Y = (long)g.n * g.nely;
  for (int kz = 0; kz < g.n; ++kz)
    for (int ky = 0; ky < g.n; ++ky) {
      const double* row = rho + ((long)g.n * ex) + X * ((long)g.n * ey + ky + Y * ((long)g.n * ez + kz));
      for (int kx = 0; kx < g.n; ++kx) {
        const double r = row[kx];
        lo = lo && r <= rho_l;
        hi = hi && r >= rho_u;
      }
    }
  const long XD = (long)g.d * g.nelx, YD = (long)g.d * g.nely;
  for (int kz = 0; kz < g.d; ++kz)
    for (int ky = 0; ky < g.d; ++ky) {
      const double* row = grad + ((long)g.d * ex) + XD * ((long)g.d * ey + ky + YD * ((long)g.d * ez + kz));
      for (int kx = 0; kx < g.d; ++kx) {
        const double v = row[kx];
        lo = lo && v >= -eps;
        hi = hi && v <= eps;
      }
    }
  kind[e] = lo ? FX_VOID : (hi ? FX_SOLID : FX_MIXED);
}

__global__ __launch_bounds__(FX_BS) void k_fix_surround(FixGeom g, const unsigned char* __restrict__ kind,
                                                        unsigned char* __restrict__ fixed,
                                                        long long* __restrict__ part) {
  __shared__ long long sh[FX_BS / 64];
  const long e = (long)blockIdx.x * FX_BS + threadIdx.x;
  int isv = 0, iss = 0;
  if (e < g.nel()) {
    const int ex = (int)(e % g.nelx), ey = (int)((e / g.nelx) % g.nely),
              ez = (int)(e / ((long)g.nelx * g.nely));
    const unsigned char k = kind[e];
    bool same = k != FX_MIXED;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int x = ex + dx, y = ey + dy, z = ez + dz;
          if (x < 0 || y < 0 || z < 0 || x >= g.nelx || y >= g.nely || z >= g.nelz) continue;
          same = same && kind[x + (long)g.nelx * (y + (long)g.nely * z)] == k;
        }
    const unsigned char f = same ? k : FX_MIXED;
    fixed[e] = f;
    isv = f == FX_VOID;
    iss = f == FX_SOLID;
  }
  const long long cv = block_count(isv, sh);
  const long long cs = block_count(iss, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = cv;
    part[2 * blockIdx.x + 1] = cs;
  }
}

__global__ __launch_bounds__(FX_BS) void k_fix_design(FixGeom g, const unsigned char* __restrict__ fixed,
                                                      unsigned char* __restrict__ out,
                                                      long long* __restrict__ part) {
  __shared__ long long sh[FX_BS / 64];
  const long i = (long)blockIdx.x * FX_BS + threadIdx.x;
  int v = 0;
  if (i < g.nx()) {
    const long XD = (long)g.d * g.nelx, YD = (long)g.d * g.nely;
    const long x = i % XD, y = (i / XD) % YD, z = i / (XD * YD);
    const long e = x / g.d + g.nelx * (y / g.d + (long)g.nely * (z / g.d));
    v = fixed[e] != FX_MIXED;
    out[i] = (unsigned char)v;
  }
  const long long c = block_count(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = c;
}

// A node's elements along one axis: (i - 1) / p and i / p when i is a
// multiple of p (those inside the domain), i / p otherwise.
__global__ __launch_bounds__(FX_BS) void k_fix_nodes(FixGeom g, const unsigned char* __restrict__ fixed,
                                                     unsigned char* __restrict__ mask,
                                                     long long* __restrict__ part) {
  __shared__ long long sh[FX_BS / 64];
  const long nd = (long)blockIdx.x * FX_BS + threadIdx.x;
  int v = 0;
  if (nd < g.nn()) {
    const long i = nd % g.nnx(), j = (nd / g.nnx()) % g.nny(), k = nd / (g.nnx() * g.nny());
    const int p = g.p;
    const int x0 = (int)(i % p ? i / p : i / p - 1), x1 = (int)(i / p);
    const int y0 = (int)(j % p ? j / p : j / p - 1), y1 = (int)(j / p);
    const int z0 = (int)(k % p ? k / p : k / p - 1), z1 = (int)(k / p);
    bool all = true;
    for (int z = z0; z <= z1; ++z)
      for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
          if (x < 0 || y < 0 || z < 0 || x >= g.nelx || y >= g.nely || z >= g.nelz) continue;
          all = all && fixed[x + (long)g.nelx * (y + (long)g.nely * z)] == FX_VOID;
        }
    if (all) {
      mask[3 * nd] = 1;
      mask[3 * nd + 1] = 1;
      mask[3 * nd + 2] = 1;
    }
    v = all;
  }
  const long long c = block_count(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = c;
}

// Sums of the block partials (stride `stride`, `nb` blocks), in block order.
__global__ __launch_bounds__(FX_BS) void k_fix_sum(int nb, int stride, int ofs,
                                                   const long long* __restrict__ part,
                                                   long long* __restrict__ out) {
  __shared__ long long sh[FX_BS / 64];
  long long s = 0;
  for (int j = threadIdx.x; j < nb; j += FX_BS) s += part[(long)j * stride + ofs];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int i = 0; i < FX_BS / 64; ++i) t += sh[i];
    *out = t;
  }
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void* get(size_t bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw Error(MGCG_ENOMEM, "scratch allocation failed");
    }
    return p;
  }
};

int nblocks(long items) { return (int)((items + FX_BS - 1) / FX_BS); }

}  // namespace

namespace {

FixGeom check_geometry(const mgcg_fix_desc& d) {
  if (d.nelx < 1 || d.nely < 1 || d.nelz < 1 || d.nsub < 1 || d.nsub > 64 || d.ndes < 1 ||
      d.ndes > 64 || d.order < 1 || d.order > 3)
    throw Error(MGCG_EINVAL, "bad fixing geometry (mesh >= 1, n and d in 1..64, order 1..3)");
  if (!std::isfinite(d.rho_l) || !std::isfinite(d.rho_u) || !std::isfinite(d.eps_grad))
    throw Error(MGCG_EINVAL, "non-finite thresholds");
  FixGeom g{d.nelx, d.nely, d.nelz, d.nsub, d.ndes, d.order};
  const double lim = 2147483647.0;
  if ((double)g.nel() * d.nsub * d.nsub * d.nsub > lim || (double)g.nel() * d.ndes * d.ndes * d.ndes > lim ||
      3.0 * g.nn() > lim)
    throw Error(MGCG_EINVAL, "fixing lattices above 2^31 - 1 entries");
  return g;
}

// Device scratch of one call: the raw kinds (a byte per element), the block
// partials of the four counts and the counts themselves, 256-byte slots.
struct FixScratch {
  size_t o_raw, o_part, o_cnt, bytes;
  int be, bx, bn;
};
FixScratch scratch_plan(const FixGeom& g) {
  FixScratch s{};
  s.be = nblocks(g.nel());
  s.bx = nblocks(g.nx());
  s.bn = nblocks(g.nn());
  size_t off = 0;
  auto slot = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  s.o_raw = slot((size_t)g.nel());
  s.o_part = slot(8 * (size_t)(2 * s.be + s.bx + s.bn));
  s.o_cnt = slot(32);
  s.bytes = off;
  return s;
}

// The kernels of one call, on stream st, all arrays on the device; base: the
// scratch of scratch_plan(g); counts (4 int64) written to cnt.
void fix_launch(const FixGeom& g, const mgcg_fix_desc& d, const FixScratch& sp, char* base,
                const double* drho, const double* dgrad, unsigned char* dkind, unsigned char* ddes,
                unsigned char* dmask, long long* cnt, hipStream_t st) {
  unsigned char* raw = (unsigned char*)(base + sp.o_raw);
  long long* part = (long long*)(base + sp.o_part);
  const int be = sp.be, bx = sp.bx, bn = sp.bn;
  long long* pv = part;               // 2 per element block
  long long* pd = part + 2 * be;      // design blocks
  long long* pn = pd + bx;            // node blocks
  hipLaunchKernelGGL(k_fix_classify, dim3(be), dim3(FX_BS), 0, st, g, drho, dgrad, d.rho_l, d.rho_u,
                     d.eps_grad, raw);
  hipLaunchKernelGGL(k_fix_surround, dim3(be), dim3(FX_BS), 0, st, g, (const unsigned char*)raw,
                     dkind, pv);
  hipLaunchKernelGGL(k_fix_design, dim3(bx), dim3(FX_BS), 0, st, g, (const unsigned char*)dkind,
                     ddes, pd);
  hipLaunchKernelGGL(k_fix_nodes, dim3(bn), dim3(FX_BS), 0, st, g, (const unsigned char*)dkind,
                     dmask, pn);
  hipLaunchKernelGGL(k_fix_sum, dim3(1), dim3(FX_BS), 0, st, be, 2, 0, (const long long*)pv, cnt);
  hipLaunchKernelGGL(k_fix_sum, dim3(1), dim3(FX_BS), 0, st, be, 2, 1, (const long long*)pv, cnt + 1);
  hipLaunchKernelGGL(k_fix_sum, dim3(1), dim3(FX_BS), 0, st, bx, 1, 0, (const long long*)pd, cnt + 2);
  hipLaunchKernelGGL(k_fix_sum, dim3(1), dim3(FX_BS), 0, st, bn, 1, 0, (const long long*)pn, cnt + 3);
  MGCG_HIP(hipGetLastError());
}

// Scratch of the entry point that allocates nothing: one array per GPU, held
// until the process ends.  Every call on a GPU shares it (calls that overlap
// on one GPU race); each call writes all of what it reads back, so nothing
// needs clearing between calls.
static __device__ __align__(256) unsigned char scratch[MGCG_FIX_SCRATCH_BYTES];

// Device address of that GPU's array (the host-side name is only a stand-in
// for the symbol), looked up once per device with the device current.
char* scratch_address(int dev) {
  static std::mutex mu;
  static std::vector<char*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if (dev < 0) throw Error(MGCG_EDEVICE, "no current device");
  if ((size_t)dev >= addr.size()) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(MGCG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[dev] = (char*)p;
  }
  return addr[dev];
}

}  // namespace

void fix_variables(const mgcg_fix_desc& d, const double* rho, const double* grad,
                   unsigned char* kind_out, unsigned char* design_out, unsigned char* mask,
                   mgcg_fix_counts* counts, int mem) {
  if (mem != MGCG_MEM_HOST && mem != MGCG_MEM_DEVICE) throw Error(MGCG_EINVAL, "bad mem flag");
  if (!rho || !grad || !kind_out || !design_out || !mask) throw Error(MGCG_EINVAL, "null array");
  const FixGeom g = check_geometry(d);
  const long nel = g.nel(), nrho = g.nrho(), nx = g.nx(), nn = g.nn();
  hipStream_t st = nullptr;
  // scratch: raw kinds, block partials, the four counts; host inputs and
  // outputs staged behind them
  const FixScratch sp = scratch_plan(g);
  size_t off = sp.bytes;
  auto slot = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) / 256 * 256;
    return o;
  };
  size_t o_rho = 0, o_grad = 0, o_kind = 0, o_des = 0, o_mask = 0;
  if (mem == MGCG_MEM_HOST) {
    o_rho = slot(8 * (size_t)nrho);
    o_grad = slot(8 * (size_t)nx);
    o_kind = slot(nel);
    o_des = slot(nx);
    o_mask = slot(3 * (size_t)nn);
  }
  DevBuf buf;
  char* base = (char*)buf.get(off);
  long long* cnt = (long long*)(base + sp.o_cnt);
  const double *drho = rho, *dgrad = grad;
  unsigned char *dkind = kind_out, *ddes = design_out, *dmask = mask;
  if (mem == MGCG_MEM_HOST) {
    drho = (const double*)(base + o_rho);
    dgrad = (const double*)(base + o_grad);
    dkind = (unsigned char*)(base + o_kind);
    ddes = (unsigned char*)(base + o_des);
    dmask = (unsigned char*)(base + o_mask);
    MGCG_HIP(hipMemcpyAsync((void*)drho, rho, 8 * (size_t)nrho, hipMemcpyHostToDevice, st));
    MGCG_HIP(hipMemcpyAsync((void*)dgrad, grad, 8 * (size_t)nx, hipMemcpyHostToDevice, st));
    MGCG_HIP(hipMemcpyAsync(dmask, mask, 3 * (size_t)nn, hipMemcpyHostToDevice, st));
  }
  fix_launch(g, d, sp, base, drho, dgrad, dkind, ddes, dmask, cnt, st);
  if (mem == MGCG_MEM_HOST) {
    MGCG_HIP(hipMemcpyAsync(kind_out, dkind, nel, hipMemcpyDeviceToHost, st));
    MGCG_HIP(hipMemcpyAsync(design_out, ddes, nx, hipMemcpyDeviceToHost, st));
    MGCG_HIP(hipMemcpyAsync(mask, dmask, 3 * (size_t)nn, hipMemcpyDeviceToHost, st));
  }
  long long hc[4];
  MGCG_HIP(hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, st));
  MGCG_HIP(hipStreamSynchronize(st));
  if (counts) {
    counts->void_elems = hc[0];
    counts->solid_elems = hc[1];
    counts->fixed_design = hc[2];
    counts->suppressed_nodes = hc[3];
  }
}

void fix_variables_noalloc(const mgcg_fix_desc& d, const double* rho, const double* grad,
                           unsigned char* kind_out, unsigned char* design_out, unsigned char* mask,
                           int64_t* counts_dev, hipStream_t st) {
  if (!rho || !grad || !kind_out || !design_out || !mask || !counts_dev)
    throw Error(MGCG_EINVAL, "null array");
  const FixGeom g = check_geometry(d);
  const FixScratch sp = scratch_plan(g);
  if (sp.bytes > (size_t)MGCG_FIX_SCRATCH_BYTES)
    throw Error(MGCG_EINVAL, "mesh needs " + std::to_string(sp.bytes) +
                                 " bytes of scratch, above the static limit of " +
                                 std::to_string((long long)MGCG_FIX_SCRATCH_BYTES));
  int dev = -1;
  MGCG_HIP(hipGetDevice(&dev));
  char* base = scratch_address(dev);
  // the counts are summed into the scratch, then copied device to device
  // into the caller's array, in stream order
  long long* cnt = (long long*)(base + sp.o_cnt);
  fix_launch(g, d, sp, base, rho, grad, kind_out, design_out, mask, cnt, st);
  MGCG_HIP(hipMemcpyAsync(counts_dev, cnt, 4 * sizeof(long long), hipMemcpyDeviceToDevice, st));
}

}  // namespace mgcg
