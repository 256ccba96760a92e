// Host runtime of one problem: hierarchy plan, a single device arena sized
// exactly as mgcg_problem_device_bytes reports, the operator refresh, the
// V-cycle (Algorithm 1 applied recursively) and a device-gated PCG whose
// convergence test never needs a host round trip inside a chunk.
#include "problem.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "element.h"

namespace mgcg {

namespace {

// Gershgorin cap of the per-DOF Jacobi weights (every row sum of W D^-1 A
// stays below 2, so the smoother converges for any densities).
constexpr double kTheta = 1.9;
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Arena {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    size_t o = align256(off);
    off = o + n * sizeof(T);
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

void validate(const mgcg_desc& d) {
  auto bad = [](const char* m) { throw Error(MGCG_EINVAL, m); };
  if (d.nelx < 1 || d.nely < 1 || d.nelz < 1) bad("element counts must be >= 1");
  if (d.order < 1 || d.order > 3) bad("order must be 1, 2 or 3");
  if (d.nsub < 1 || d.nsub > 4) bad("nsub must be 1..4");
  if (d.nlevels < 1 || d.nlevels > 12) bad("nlevels must be 1..12");
  if (d.nrhs < 1 || d.nrhs > 4) bad("nrhs must be 1..4");
  if (d.precision != MGCG_FP64 && d.precision != MGCG_MIXED) bad("precision must be FP64 or MIXED");
  if (d.pre < 1 || d.pre > 8 || d.post < 0 || d.post > 8) bad("pre must be 1..8, post 0..8");
  if (!(d.omega > 0.0 && d.omega < 2.0)) bad("omega must be in (0, 2)");
  if (!(d.E0 > 0.0) || !(d.Emin >= 0.0) || !(d.Emin < d.E0)) bad("need E0 > Emin >= 0");
  if (!(d.nu > -1.0 && d.nu < 0.5)) bad("nu must be in (-1, 0.5)");
  if (!(d.penal >= 1.0 && d.penal <= 10.0)) bad("penal must be in [1, 10]");
  if (d.order >= 2 && d.nlevels < 2) bad("quadratic and cubic elements need nlevels >= 2");
  if (d.family != MGCG_LAGRANGE && !(d.family == MGCG_SERENDIPITY && d.order >= 2))
    bad("family must be Lagrange, or serendipity with order 2 or 3");
  if (d.smoother != MGCG_SMOOTH_JACOBI && !(d.smoother == MGCG_SMOOTH_GAUSS_SEIDEL && d.order >= 2))
    bad("smoother must be Jacobi, or Gauss-Seidel with order 2 or 3");
}

}  // namespace

// ------------------------------------------------------------------ planning
void Problem::plan_levels(const mgcg_desc& d, std::vector<LevelPlan>& lv) {
  validate(d);
  lv.clear();
  LevelPlan l0;
  const int p = d.order;
  l0.L = Lat{p * d.nelx + 1, p * d.nely + 1, p * d.nelz + 1};
  l0.kind = d.order == 3 ? OP_EQ3 : d.order == 2 ? OP_EQ2 : (d.nsub == 1 ? OP_MF_Q1 : OP_ST27);
  l0.ncx = d.nelx;
  l0.ncy = d.nely;
  l0.ncz = d.nelz;
  lv.push_back(l0);
  int cx = d.nelx, cy = d.nely, cz = d.nelz;
  for (int l = 1; l < d.nlevels; ++l) {
    if (!(l == 1 && d.order >= 2)) {  // degree >= 2: first onto the vertex lattice
      if (cx % 2 || cy % 2 || cz % 2)
        throw Error(MGCG_EINVAL, "too many levels: element counts must be even to coarsen");
      cx /= 2;
      cy /= 2;
      cz /= 2;
    }
    LevelPlan lp;
    lp.L = Lat{cx + 1, cy + 1, cz + 1};
    lp.kind = OP_ST27;
    lp.ncx = cx;
    lp.ncy = cy;
    lp.ncz = cz;
    lv.push_back(lp);
  }
  // kernels address a level vector (per load case), a stencil block's nine
  // coefficient rows and the element moduli through 32-bit buffer offsets
  for (const LevelPlan& l : lv) {
    if (l.L.ndof() * 8 >= kMaxBufferBytes)
      throw Error(MGCG_EINVAL, "mesh too large: a level vector would exceed 2 GiB");
    if (l.kind == OP_ST27 && 9 * l.L.nn() * 8 >= kMaxBufferBytes)
      throw Error(MGCG_EINVAL, "mesh too large: stencil coefficient rows would exceed 2 GiB");
  }
  if ((long)d.nelx * d.nely * d.nelz * d.nsub * d.nsub * d.nsub * 8 >= kMaxBufferBytes)
    throw Error(MGCG_EINVAL, "mesh too large: the density field would exceed 2 GiB");
  // the finest level's reducing applies write one partial sum per block
  if (!lv.empty() && (apply_blocks(lv[0].kind, lv[0].L, true) > MAX_BLOCKS ||
                      apply_blocks(lv[0].kind, lv[0].L, false) > MAX_BLOCKS))
    throw Error(MGCG_EINVAL, "mesh too large: the finest level exceeds the reduction buffer's blocks");
}

// One layout routine serves both the byte count and the pointer assignment.
size_t Problem::layout(const mgcg_desc& d, const std::vector<LevelPlan>& lv, char* base, Problem* s) {
  Arena A{base};
  const int R = d.nrhs;
  const bool mixed = d.precision == MGCG_MIXED;
  const size_t vb = mixed ? 4 : 8;
  const long nd0 = lv[0].L.ndof();
  const long nel0 = (long)d.nelx * d.nely * d.nelz;
  const long ns3 = (long)d.nsub * d.nsub * d.nsub;
  const long nrho = nel0 * ns3;
  const int ndl = 3 * (d.order + 1) * (d.order + 1) * (d.order + 1);
  const int L = (int)lv.size();
#define TAKE(member, T, n)          \
  do {                              \
    auto p_ = A.take<T>((size_t)(n)); \
    if (s) s->member = p_;          \
  } while (0)
  TAKE(f_, double, R * nd0);
  TAKE(rho_, double, nrho);
  TAKE(E_, double, nrho);
  if (mixed && lv[0].kind == OP_MF_Q1) TAKE(E32_, float, nrho);
  TAKE(Ksub_, double, ns3 * ndl * ndl);
  if (d.nsub == 4 || d.order == 3) TAKE(Kp_, double, sens_packed_doubles(d.order));
  TAKE(K0_, double, 576);
  if (mixed) TAKE(K032_, float, 576);
  TAKE(x_, double, R * nd0);
  TAKE(r_, double, R * nd0);
  TAKE(p_, double, R * nd0);
  TAKE(q_, double, R * nd0);
  TAKE(tmp64_, double, R * nd0);
  TAKE(cs_, CgScalars, 4);
  if (fused_ok(d, lv)) TAKE(fz_, FzDesc, R);
  TAKE(red_.partials, double, (size_t)RED_NREGIONS * RED_REGION);
  TAKE(compout_, double, 16);
  TAKE(bad_, int, 4);
  TAKE(dcbuf_, double, nrho);
  if (lv[0].kind == OP_ST27) TAKE(Keff_, double, nel0 * 576);
  if (lv[0].kind == OP_EQ3) {
    const long pk = d.family == MGCG_SERENDIPITY ? S3_PACKED : L3_PACKED;
    TAKE(Keff_, double, nel0 * L3_ND * L3_ND);  // full matrices (setup)
    TAKE(Kq2_, double, nel0 * pk);              // wrapped diagonals (applies)
    if (mixed) TAKE(Keff32_, float, nel0 * pk);
    TAKE(Yeq_, double, R * nel0 * L3_ND);
    if (d.smoother == MGCG_SMOOTH_GAUSS_SEIDEL) {
      TAKE(Kn_, char, nel0 * L3_ND * L3_ND * (mixed ? sizeof(float) : sizeof(double)));
      TAKE(Dn_, char, lv[0].L.nn() * 9 * (mixed ? sizeof(float) : sizeof(double)));
    }
  }
  if (lv[0].kind == OP_EQ2) {
    TAKE(Keff_, double, nel0 * 6561);           // full matrices (setup)
    TAKE(Kq2_, double, nel0 * Q2_PACKED);       // wrapped diagonals (applies)
    if (mixed) TAKE(Keff32_, float, nel0 * Q2_PACKED);
    TAKE(Yeq_, double, R * nel0 * 81);
    // the Gauss-Seidel smoother's rows by node, in the V-cycle precision
    if (d.smoother == MGCG_SMOOTH_GAUSS_SEIDEL) {
      TAKE(Kn_, char, nel0 * 6561 * (mixed ? sizeof(float) : sizeof(double)));
      TAKE(Dn_, char, lv[0].L.nn() * 9 * (mixed ? sizeof(float) : sizeof(double)));
    }
  }
  for (int l = 0; l < L; ++l) {
    const long nn = lv[l].L.nn(), nd = lv[l].L.ndof();
    const long nel = (long)lv[l].ncx * lv[l].ncy * lv[l].ncz;
    LevelBufs* b = s ? &s->B_[l] : nullptr;
    auto take_to = [&](auto*& dst, auto tag, size_t n) {
      using T = decltype(tag);
      T* p = A.take<T>(n);
      if (b) dst = p;
    };
    uint8_t* um = nullptr;
    double* dd = nullptr;
    char* cv = nullptr;
    take_to(um, uint8_t{}, nn);
    if (b) b->mask = um;
    if (l >= 1) {
      take_to(dd, double{}, nel * 576);
      if (b) b->KE = dd;
    }
    if (l >= 1 || lv[0].kind == OP_ST27) {
      take_to(cv, char{}, (size_t)ST_COEF * nn * vb);
      if (b) b->coefV = cv;
      if (l == 0 && mixed) {
        take_to(dd, double{}, (size_t)ST_COEF * nn);
        if (b) b->coef64 = dd;
      }
    }
    take_to(cv, char{}, nd * vb);
    if (b) b->invD = cv;
    take_to(dd, double{}, nd);
    if (b) b->diag64 = dd;
    take_to(cv, char{}, R * nd * vb);
    if (b) b->b = cv;
    take_to(cv, char{}, R * nd * vb);
    if (b) b->xa = cv;
    take_to(cv, char{}, R * nd * vb);
    if (b) b->xb = cv;
    take_to(cv, char{}, R * nd * vb);
    if (b) b->r = cv;
  }
  if (L >= 2) {
    const int B = d.order >= 2 ? d.nsub : 2 * d.nsub;
    TAKE(G_, double, (size_t)B * B * B * 576);
    TAKE(dmasked_, int, (long)lv[1].ncx * lv[1].ncy * lv[1].ncz);
  }
  const long ndc = lv[L - 1].L.ndof();  // upper bound of the coarsest free DOFs
  TAKE(dfree_, int, ndc);
  TAKE(ddofpos_, int, ndc);
  const long ldc = coarse_ld(ndc);  // dense coarsest operator and its inverse, padded
  TAKE(Ad_, double, ldc * ldc);
  TAKE(Ad2_, double, ldc * ldc);
  TAKE(Dgj_, double, GJ_B * GJ_B);
  TAKE(diag0_, double, ldc);
#undef TAKE
  return align256(A.off);
}

size_t Problem::device_bytes(const mgcg_desc& d) {
  std::vector<LevelPlan> lv;
  plan_levels(d, lv);
  return layout(d, lv, nullptr, nullptr);
}

long Problem::nrho() const {
  return (long)d_.nelx * d_.nely * d_.nelz * d_.nsub * d_.nsub * d_.nsub;
}

// ------------------------------------------------------------------ lifetime
Problem::Problem(const mgcg_desc& d, const uint8_t* mask, const double* f, int device)
    : d_(d), device_(device) {
  plan_levels(d_, lv_);
  vbytes_ = d_.precision == MGCG_MIXED ? 4 : 8;
  const long nd0 = lv_[0].L.ndof();
  if (!mask || !f) throw Error(MGCG_EINVAL, "mask and f are required");
  // node masks per level: bit c set when DOF c of the node is fixed; a coarse
  // node inherits the mask of the fine node it coincides with.
  hmask_off_.assign(lv_.size() + 1, 0);
  for (size_t l = 0; l < lv_.size(); ++l) hmask_off_[l + 1] = hmask_off_[l] + lv_[l].L.nn();
  hmask_.assign(hmask_off_.back(), 0);
  for (long n = 0; n < lv_[0].L.nn(); ++n) {
    uint8_t m = 0;
    for (int c = 0; c < 3; ++c)
      if (mask[3 * n + c]) m |= (uint8_t)(1 << c);
    hmask_[n] = m;
  }
  if (d_.family == MGCG_SERENDIPITY) {
    // face- and body-interior nodes of the lattice (two or three indices
    // off the vertex lattice)
    const Lat L0 = lv_[0].L;
    const int p = d_.order;
    for (long n = 0; n < L0.nn(); ++n) {
      const long i = n % L0.nx, j = (n / L0.nx) % L0.ny, k = n / ((long)L0.nx * L0.ny);
      if ((i % p != 0) + (j % p != 0) + (k % p != 0) >= 2) hmask_[n] = 7;
    }
  }
  for (size_t l = 1; l < lv_.size(); ++l) {
    const Lat F = lv_[l - 1].L, C = lv_[l].L;
    // Q1 halving and the Q2 -> vertex lattice step take every second node,
    // the cubic -> vertex lattice step every third
    const int stride = (l == 1 && d_.order == 3) ? 3 : 2;
    for (int k = 0; k < C.nz; ++k)
      for (int j = 0; j < C.ny; ++j)
        for (int i = 0; i < C.nx; ++i) {
          const long fn = (long)stride * i + (long)F.nx * ((long)stride * j + (long)F.ny * stride * k);
          hmask_[hmask_off_[l] + i + (long)C.nx * (j + (long)C.ny * k)] = hmask_[hmask_off_[l - 1] + fn];
        }
  }
  hf_.assign(f, f + (size_t)d_.nrhs * nd0);
  for (int r = 0; r < d_.nrhs; ++r)
    for (long i = 0; i < nd0; ++i)
      if ((hmask_[i / 3] >> (i % 3)) & 1) hf_[(size_t)r * nd0 + i] = 0.0;
  for (double v : hf_)
    if (!std::isfinite(v)) throw Error(MGCG_EINVAL, "non-finite load");
  // coarsest free DOF list
  const LevelPlan& lc = lv_.back();
  hdofpos_.assign(lc.L.ndof(), -1);
  for (long n = 0; n < lc.L.nn(); ++n)
    for (int c = 0; c < 3; ++c)
      if (!((hmask_[hmask_off_[lv_.size() - 1] + n] >> c) & 1)) {
        hdofpos_[3 * n + c] = (int)hfree_.size();
        hfree_.push_back((int)(3 * n + c));
      }
  nc_ = (int)hfree_.size();
  hKsub_ = sub_element_matrices(d_.order, d_.nsub, d_.nu, d_.family);
  B_.resize(lv_.size());
  if (lv_.size() >= 2) build_linear_galerkin();
  // unit trilinear element in its Haar basis as class values; must
  // reproduce the quadrature
  {
    const double nu = d_.nu;
    const std::vector<double> k0 = sub_element_matrices(1, 1, nu);
    double mx = 0.0;
    for (int q = 0; q < 576; ++q) mx = std::max(mx, std::fabs(k0[q]));
    // the Haar-basis form: T^T K0 T / 64 from the quadrature matrix must
    // match the class values on the structure, and vanish off it
    hv64_ = q1_haar_values(nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), 1.0 / (2.0 * (1.0 + nu)));
    for (int k = 0; k < 16; ++k) hv32_.v[k] = (float)hv64_.v[k];
    auto Th = [](int a, int m) {
      int p = 1;
      for (int d = 0; d < 3; ++d) p *= (((m >> d) & 1) && !((a >> d) & 1)) ? -1 : 1;
      return p;
    };
    double herr = 0.0;
    for (int i = 0; i < 24; ++i)
      for (int j = 0; j < 24; ++j) {
        double h = 0.0;
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b)
            h += Th(a, i / 3) * Th(b, j / 3) * k0[(3 * a + i % 3) * 24 + 3 * b + j % 3];
        h /= 64.0;
        const int q = i * 24 + j;
        const double v = kQ1H.cls[q] < 0 ? 0.0 : kQ1H.sgn[q] * hv64_.v[kQ1H.cls[q]];
        herr = std::max(herr, std::fabs(v - h));
      }
    if (herr > 1e-14 * mx) throw Error(MGCG_EINVAL, "Haar element table does not match the quadrature");
  }
}

Problem::~Problem() {
  try {
    release();
  } catch (...) {
  }
  if (budget_) budget_->attach(-1);
}

void Problem::attach_budget(Budget* b) {
  if (arena_) throw Error(MGCG_EINVAL, "the problem already holds device memory");
  if (budget_) budget_->attach(-1);
  budget_ = b;
  if (b) b->attach(1);
}

void Problem::release() {
  if (!arena_) return;
  hipSetDevice(device_);
  if (stream_) hipStreamSynchronize(stream_);
  drop_iter_graph();
  for (auto& e : timer_.pool) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  timer_.pool.clear();
  if (ev_chunk_) hipEventDestroy(ev_chunk_);
  if (ev_s0_) hipEventDestroy(ev_s0_);
  if (ev_s1_) hipEventDestroy(ev_s1_);
  ev_chunk_ = ev_s0_ = ev_s1_ = nullptr;
  if (hcs_) hipHostFree(hcs_);
  hcs_ = nullptr;
  hipFree(arena_);
  arena_ = nullptr;
  if (budget_) budget_->refund(bytes_);
  if (own_stream_) {
    if (stream_ == own_stream_) stream_ = nullptr;
    hipStreamDestroy(own_stream_);
    own_stream_ = nullptr;
  }
  have_ops_ = have_u_ = false;
  for (auto& b : B_) b = LevelBufs{};
}

void Problem::set_stream(hipStream_t s) {
  MGCG_HIP(hipSetDevice(device_));
  if (stream_) MGCG_HIP(hipStreamSynchronize(stream_));
  stream_ = s;
  ensure_stream();
}

hipStream_t Problem::ensure_stream() {
  MGCG_HIP(hipSetDevice(device_));
  if (!own_stream_) MGCG_HIP(hipStreamCreateWithFlags(&own_stream_, hipStreamNonBlocking));
  if (!stream_) stream_ = own_stream_;
  return stream_;
}

void Problem::allocate() {
  if (arena_) return;
  ensure_stream();
  bytes_ = layout(d_, lv_, nullptr, nullptr);
  if (budget_ && !budget_->charge(bytes_))
    throw Error(MGCG_EBUDGET, "the context's HBM budget cannot hold " + std::to_string(bytes_) +
                                  " more bytes");
  char* base = nullptr;
  if (hipMalloc(&base, bytes_) != hipSuccess) {
    (void)hipGetLastError();
    if (budget_) budget_->refund(bytes_);
    throw Error(MGCG_ENOMEM, "device allocation of " + std::to_string(bytes_) + " bytes failed");
  }
  arena_ = base;
  layout(d_, lv_, base, this);
  MGCG_HIP(hipMemsetAsync(arena_, 0, bytes_, stream_));
  MGCG_HIP(hipHostMalloc((void**)&hcs_, 4 * sizeof(CgScalars), hipHostMallocDefault));
  MGCG_HIP(hipEventCreateWithFlags(&ev_chunk_, hipEventDisableTiming));
  MGCG_HIP(hipEventCreate(&ev_s0_));
  MGCG_HIP(hipEventCreate(&ev_s1_));
  // static data
  const long nd0 = lv_[0].L.ndof();
  for (size_t l = 0; l < lv_.size(); ++l)
    MGCG_HIP(hipMemcpyAsync(B_[l].mask, &hmask_[hmask_off_[l]], lv_[l].L.nn(), hipMemcpyHostToDevice,
                            stream_));
  MGCG_HIP(hipMemcpyAsync(f_, hf_.data(), hf_.size() * sizeof(double), hipMemcpyHostToDevice, stream_));
  if (Kp_) {
    // the 64 sub-element matrices packed for the sensitivity contraction
    sens_pack(d_.order, d_.nsub, hKsub_.data(), hKp_);
    MGCG_HIP(hipMemcpyAsync(Kp_, hKp_.data(), hKp_.size() * sizeof(double), hipMemcpyHostToDevice,
                            stream_));
  }
  MGCG_HIP(hipMemcpyAsync(Ksub_, hKsub_.data(), hKsub_.size() * sizeof(double), hipMemcpyHostToDevice,
                          stream_));
  {
    std::vector<double> k0 = sub_element_matrices(1, 1, d_.nu);
    MGCG_HIP(hipMemcpyAsync(K0_, k0.data(), 576 * sizeof(double), hipMemcpyHostToDevice, stream_));
    if (K032_) convert<double, float>(K0_, K032_, 576, stream_);
  }
  if (G_) {
    MGCG_HIP(hipMemcpyAsync(G_, hG_.data(), hG_.size() * sizeof(double), hipMemcpyHostToDevice, stream_));
    if (!hmasked_.empty())
      MGCG_HIP(hipMemcpyAsync(dmasked_, hmasked_.data(), hmasked_.size() * sizeof(int),
                              hipMemcpyHostToDevice, stream_));
  }
  if (nc_ > 0) {
    MGCG_HIP(hipMemcpyAsync(dfree_, hfree_.data(), hfree_.size() * sizeof(int), hipMemcpyHostToDevice,
                            stream_));
    MGCG_HIP(hipMemcpyAsync(ddofpos_, hdofpos_.data(), hdofpos_.size() * sizeof(int),
                            hipMemcpyHostToDevice, stream_));
  }
  (void)nd0;
  MGCG_HIP(hipStreamSynchronize(stream_));
}

void Problem::sync() { MGCG_HIP(hipStreamSynchronize(stream_)); }

// ------------------------------------------------------------------ operators
// First coarse level as K_E = sum_m E_m G_m: G_m = P^T K^(e_s) P for the
// density cell m of the coarse element (child c, sub-element s), where P
// interpolates the coarse element's 8 vertices trilinearly onto the child's
// nodes (Sec. 2.3).  Elements with a supported child DOF are listed for the
// explicit masked product.
void Problem::build_linear_galerkin() {
  const int n = d_.nsub, p = d_.order;
  const bool q2 = p >= 2;  // one fine element of degree p per coarse element
  const int B = q2 ? n : 2 * n;
  gB_ = B;
  const int p1 = p + 1, nen = p1 * p1 * p1, nd = 3 * nen;
  const int M = B * B * B;
  hG_.assign((size_t)M * 576, 0.0);
  std::vector<double> W((size_t)nen * 8);
  for (int m = 0; m < M; ++m) {
    const int px = m % B, py = (m / B) % B, pz = m / (B * B);
    const int cx = q2 ? 0 : px / n, cy = q2 ? 0 : py / n, cz = q2 ? 0 : pz / n;
    const int sx = q2 ? px : px % n, sy = q2 ? py : py % n, sz = q2 ? pz : pz % n;
    const double* K = &hKsub_[(size_t)(sx + n * (sy + n * sz)) * nd * nd];
    for (int a = 0; a < nen; ++a) {
      const int ax = a % p1, ay = (a / p1) % p1, az = a / (p1 * p1);
      for (int b = 0; b < 8; ++b)
        W[(size_t)a * 8 + b] = q2 ? trilinear_weight(ax, ay, az, b, p)
                                  : trilinear_weight(cx + ax, cy + ay, cz + az, b);
    }
    double* G = &hG_[(size_t)m * 576];
    for (int b = 0; b < 8; ++b)
      for (int i = 0; i < 3; ++i)
        for (int b2 = 0; b2 < 8; ++b2)
          for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int a = 0; a < nen; ++a) {
              const double wa = W[(size_t)a * 8 + b];
              if (wa == 0.0) continue;
              for (int a2 = 0; a2 < nen; ++a2) {
                const double wb = W[(size_t)a2 * 8 + b2];
                if (wb == 0.0) continue;
                s += wa * K[(size_t)(3 * a + i) * nd + 3 * a2 + j] * wb;
              }
            }
            G[(3 * b + i) * 24 + 3 * b2 + j] = s;
          }
  }
  // coarse elements whose fine nodes (lattice rE..rE+r, r = 3 for cubic
  // elements, else 2) carry a support
  const Lat F = lv_[0].L;
  const LevelPlan& c1 = lv_[1];
  const int r = p == 3 ? 3 : 2;
  hmasked_.clear();
  for (int EZ = 0; EZ < c1.ncz; ++EZ)
    for (int EY = 0; EY < c1.ncy; ++EY)
      for (int EX = 0; EX < c1.ncx; ++EX) {
        bool any = false;
        for (int dz = 0; dz <= r && !any; ++dz)
          for (int dy = 0; dy <= r && !any; ++dy)
            for (int dx = 0; dx <= r && !any; ++dx) {
              const long fn = (r * EX + dx) + (long)F.nx * ((r * EY + dy) + (long)F.ny * (r * EZ + dz));
              if (hmask_[fn]) any = true;
            }
        if (any) hmasked_.push_back(EX + c1.ncx * (EY + c1.ncy * EZ));
      }
}

// Blocks per load case of the finest-level apply (the number of per-block
// partial sums its reducing epilogues produce), in FP64 or in the V-cycle
// precision.
int Problem::nblocks_fine(bool fp64) const {
  return apply_blocks(lv_[0].kind, lv_[0].L, fp64);
}

FineOp Problem::fine_op() const {
  FineOp A{};
  A.kind = lv_[0].kind;
  const Lat L = lv_[0].L;
  A.mf = OpMF<double>::make(L, E_, hv64_, B_[0].mask);
  A.st = OpST<double>{L, vbytes_ == 8 ? (const double*)B_[0].coefV : B_[0].coef64};
  A.eq2 = OpEQ2<double>{L, Kq2_, B_[0].mask, Yeq_, d_.family == MGCG_SERENDIPITY, d_.order};
  return A;
}

template <typename T>
VOps<T> Problem::vops(int l) const {
  VOps<T> v{};
  v.kind = lv_[l].kind;
  v.L = lv_[l].L;
  v.mask = B_[l].mask;
  v.invD = (const T*)B_[l].invD;
  if constexpr (sizeof(T) == 8) {
    v.mf = OpMF<T>::make(v.L, E_, hv64_, B_[l].mask);
    v.eq2 = OpEQ2<T>{v.L, Kq2_, B_[l].mask, (T*)Yeq_, d_.family == MGCG_SERENDIPITY, d_.order};
  } else {
    v.mf = OpMF<T>::make(v.L, E32_, hv32_, B_[l].mask);
    v.eq2 = OpEQ2<T>{v.L, Keff32_, B_[l].mask, (T*)Yeq_, d_.family == MGCG_SERENDIPITY, d_.order};
  }
  v.st = OpST<T>{v.L, (const T*)B_[l].coefV};
  return v;
}

void Problem::check_bad(int which) {
  int hb[4] = {0, 0, 0, 0};
  MGCG_HIP(hipMemcpyAsync(hb, bad_, sizeof(hb), hipMemcpyDeviceToHost, stream_));
  sync();
  (void)which;
  if (hb[0] & 1) {
    have_ops_ = false;
    throw Error(MGCG_EINVAL, "density outside [0, 1] or NaN");
  }
  if (hb[0] & 2) {
    have_ops_ = false;
    throw Error(MGCG_EBREAKDOWN, "coarsest-level matrix is not positive definite");
  }
}

void Problem::set_densities(const double* rho, int mem) {
  set_densities_async(rho, mem);
  MGCG_HIP(hipEventSynchronize(ev_s1_));
  float ms = 0.f;
  MGCG_HIP(hipEventElapsedTime(&ms, ev_s0_, ev_s1_));
  setup_ms_ = ms;
  pending_check_ = false;
  check_bad(0);
}

void Problem::set_densities_f32(const float* rho, int mem) {
  allocate();
  MGCG_HIP(hipSetDevice(device_));
  const long n = nrho();
  if (mem == MGCG_MEM_HOST) {
    const std::vector<double> h(rho, rho + n);
    set_densities(h.data(), MGCG_MEM_HOST);
    return;
  }
  convert<float, double>(rho, rho_, n, stream_);
  set_densities(nullptr, MGCG_MEM_DEVICE);  // rho_ holds them already
}

void Problem::set_densities_async(const double* rho, int mem) {
  allocate();
  MGCG_HIP(hipSetDevice(device_));
  const long n = nrho();
  MGCG_HIP(hipEventRecord(ev_s0_, stream_));
  if (rho)
    MGCG_HIP(hipMemcpyAsync(rho_, rho, n * sizeof(double),
                            mem == MGCG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            stream_));
  fill<int>(bad_, 0, 4, stream_);
  if (vbytes_ == 8)
    do_set_densities<double>();
  else
    do_set_densities<float>();
  MGCG_HIP(hipEventRecord(ev_s1_, stream_));
  have_ops_ = true;
  pending_check_ = true;
}

template <typename T>
void Problem::do_set_densities() {
  hipStream_t st = stream_;
  const int L = (int)lv_.size();
  const Lat L0 = lv_[0].L;
  const bool mixed = sizeof(T) == 4;
  setup_simp(rho_, E_, E32_, nrho(), d_.E0, d_.Emin, d_.penal, bad_, st);
  switch (lv_[0].kind) {
    case OP_MF_Q1:
      setup_diag_mf<T>(L0, E_, K0_, B_[0].mask, (T*)B_[0].invD, B_[0].diag64, d_.omega, kTheta, st);
      break;
    case OP_ST27:
      setup_effective(1, d_.nsub, d_.nelx, d_.nely, d_.nelz, E_, Ksub_, B_[0].mask, L0, Keff_, st);
      if (mixed) {
        // FP64 copy for the outer CG, FP32 one for the V-cycle
        setup_stencil<double>(L0, Keff_, B_[0].mask, B_[0].coef64, (double*)tmp64_, B_[0].diag64, d_.omega, kTheta, st);
        setup_stencil<float>(L0, Keff_, B_[0].mask, (float*)B_[0].coefV, (float*)B_[0].invD, nullptr, d_.omega, kTheta, st);
      } else {
        setup_stencil<double>(L0, Keff_, B_[0].mask, (double*)B_[0].coefV, (double*)B_[0].invD,
                              B_[0].diag64, d_.omega, kTheta, st);
      }
      break;
    case OP_EQ3: {
      const long nel0 = (long)d_.nelx * d_.nely * d_.nelz;
      const int ser = d_.family == MGCG_SERENDIPITY;
      setup_effective(3, d_.nsub, d_.nelx, d_.nely, d_.nelz, E_, Ksub_, B_[0].mask, L0, Keff_, st);
      setup_diag_e3<T>(L0, Keff_, B_[0].mask, (T*)B_[0].invD, B_[0].diag64, d_.omega, kTheta, st);
      setup_pack_e3<double>(Keff_, Kq2_, nel0, ser, st);
      if (mixed) setup_pack_e3<float>(Keff_, Keff32_, nel0, ser, st);
      if (Kn_) {
        setup_rows_by_node<T>(3, Keff_, (T*)Kn_, nel0, st);
        setup_gs_diag<T>(3, L0, (const T*)Kn_, (T*)Dn_, st);
      }
      break;
    }
    default:
      setup_effective(2, d_.nsub, d_.nelx, d_.nely, d_.nelz, E_, Ksub_, B_[0].mask, L0, Keff_, st);
      setup_diag_eq2<T>(L0, Keff_, B_[0].mask, (T*)B_[0].invD, B_[0].diag64, d_.omega, kTheta, st);
      {
        const long nel0 = (long)d_.nelx * d_.nely * d_.nelz;
        if (d_.family == MGCG_SERENDIPITY) {
          setup_pack_s2<double>(Keff_, Kq2_, nel0, st);
          if (mixed) setup_pack_s2<float>(Keff_, Keff32_, nel0, st);
        } else {
          setup_pack_q2<double>(Keff_, Kq2_, nel0, st);
          if (mixed) setup_pack_q2<float>(Keff_, Keff32_, nel0, st);
        }
        if (Kn_) {
          setup_rows_by_node<T>(2, Keff_, (T*)Kn_, nel0, st);
          setup_gs_diag<T>(2, L0, (const T*)Kn_, (T*)Dn_, st);
        }
      }
      break;
  }
  for (int l = 1; l < L; ++l) {
    const int src = (l == 1) ? lv_[0].kind : OP_ST27;
    const double* Kc = (l == 1) ? Keff_ : B_[l - 1].KE;
    if (l == 1) {
      setup_galerkin_lin(E_, G_, gB_, d_.nsub, d_.nelx, d_.nely, lv_[1].ncx, lv_[1].ncy, lv_[1].ncz,
                         B_[1].KE, st);
      setup_galerkin(src, lv_[0].L, E_, K0_, Kc, B_[0].mask, lv_[1].ncx, lv_[1].ncy, lv_[1].ncz,
                     B_[1].KE, dmasked_, (int)hmasked_.size(), st);
    } else {
      setup_galerkin(src, lv_[l - 1].L, E_, K0_, Kc, B_[l - 1].mask, lv_[l].ncx, lv_[l].ncy,
                     lv_[l].ncz, B_[l].KE, nullptr, 0, st);
    }
    setup_stencil<T>(lv_[l].L, B_[l].KE, B_[l].mask, (T*)B_[l].coefV, (T*)B_[l].invD, B_[l].diag64,
                     d_.omega, kTheta, st);
  }
  // coarsest: dense operator and its explicit inverse (blocked Gauss-Jordan)
  const int lc = L - 1;
  const int src = (lc == 0) ? lv_[0].kind : OP_ST27;
  const double* KE = (lc == 0) ? Keff_ : B_[lc].KE;
  const int ld = coarse_ld(lv_[lc].L.ndof());
  setup_dense(src, lv_[lc].L, E_, K0_, KE, dfree_, ddofpos_, nc_, ld, Ad_, st);
  Ainv_ = setup_coarse_inverse(Ad_, Ad2_, Dgj_, diag0_, ld, bad_, st);
}

// ------------------------------------------------------------------ V-cycle
template <typename T>
void Problem::vcycle(const double* r_in, int gate, bool fuse_dot, bool x0_ready) {
  hipStream_t st = stream_;
  const CgScalars* cs = gate ? cs_ : nullptr;
  const int L = (int)lv_.size();
  const int R = d_.nrhs;
  const T omega = T(1);  // the Jacobi weights are folded into wD
  const T* b0;
  if constexpr (sizeof(T) == 8) {
    b0 = (const T*)r_in;
  } else {
    b0 = (const T*)B_[0].b;
  }
  // a small coarsest level takes the last (halving) restriction inside its
  // solve
  const bool fuse_cs = L > 1 && lv_[L - 1].L.ndof() <= CS_FUSE_MAX && !(L == 2 && d_.order == 3);
  std::vector<T*> cur(L), oth(L);
  std::vector<const T*> bl(L);
  bl[0] = b0;
  for (int l = 0; l < L; ++l) {
    cur[l] = (T*)B_[l].xa;
    oth[l] = (T*)B_[l].xb;
    if (l > 0) bl[l] = (const T*)B_[l].b;
  }
  // level-0 input and its first sweep from zero (the coarse levels get theirs
  // from the restriction); the Gauss-Seidel smoother sweeps in place from a
  // zeroed level-0 iterate
  const bool gs0 = gs_smoother();
  if (gs0) {
    if constexpr (sizeof(T) == 4)
      convert<double, float>(r_in, (float*)B_[0].b, R * lv_[0].L.ndof(), st);
    fill<T>(cur[0], T(0), R * lv_[0].L.ndof(), st);
  } else if (L > 1 && !x0_ready) {
    v_prepare0<T>(r_in, sizeof(T) == 8 ? nullptr : (T*)B_[0].b, (const T*)B_[0].invD, cur[0],
                  lv_[0].L.ndof(), R, cs, st);
  } else if constexpr (sizeof(T) == 4) {
    // (with x0_ready the residual producers also wrote its FP32 copy)
    if (!x0_ready) convert<double, float>(r_in, (float*)B_[0].b, R * lv_[0].L.ndof(), st);
  }
  for (int l = 0; l < L - 1; ++l) {
    const VOps<T> v = vops<T>(l);
    T* rl = (T*)B_[l].r;
    if (l == 0 && gs0) {
      for (int s = 0; s < d_.pre; ++s)
        v_gauss_seidel<T>(d_.order, lv_[0].L, (const T*)Kn_, (const T*)Dn_, B_[0].mask, bl[0], cur[0],
                          false, R, cs, st);
    } else {
      for (int s = 1; s < d_.pre; ++s) {
        v_jacobi<T>(v, bl[l], cur[l], oth[l], omega, R, cs, st);
        std::swap(cur[l], oth[l]);
      }
    }
    if (l == 0) timed_begin(1);
    v_residual<T>(v, bl[l], cur[l], rl, R, cs, st);
    if (l == 0) timed_end(1);
    const bool coarsest_next = (l + 1 == L - 1);
    // a small coarsest level takes its restriction inside the coarse solve
    if (coarsest_next && fuse_cs) continue;
    v_restrict<T>(lv_[l].L, lv_[l + 1].L, B_[l].mask, B_[l + 1].mask, rl, (T*)B_[l + 1].b,
                  (const T*)B_[l + 1].invD, coarsest_next ? nullptr : cur[l + 1], R, cs, st);
  }
  const int lc = L - 1;
  if (fuse_cs)
    v_coarse_solve_r<T>(Ainv_, coarse_ld(lv_[lc].L.ndof()), lv_[lc - 1].L, lv_[lc].L, B_[lc].mask,
                        (const T*)B_[lc - 1].r, cur[lc], R, cs, st);
  else
    v_coarse_solve<T>(Ainv_, coarse_ld(lv_[lc].L.ndof()), lv_[lc].L.ndof(), bl[lc], cur[lc], R,
                      cs, st);
  for (int l = L - 2; l >= 0; --l) {
    const VOps<T> v = vops<T>(l);
    // small stencil levels take the prolongation inside their first
    // post-smoothing sweep
    const bool fuse_p = d_.post >= 1 && v.kind == OP_ST27 &&
                        lv_[l].L.nn() <= PROLONG_FUSE_MAX_NODES && !(l == 0 && fuse_dot);
    if (!fuse_p)
      v_prolong<T>(lv_[l].L, lv_[l + 1].L, B_[l].mask, B_[l + 1].mask, cur[l + 1], cur[l], R, true,
                   cs, st);
    if (l == 0 && gs0) {
      for (int s = 0; s < d_.post; ++s)
        v_gauss_seidel<T>(d_.order, lv_[0].L, (const T*)Kn_, (const T*)Dn_, B_[0].mask, bl[0], cur[0],
                          true, R, cs, st);
      continue;
    }
    for (int s = 0; s < d_.post; ++s) {
      if (l == 0) timed_begin(2);
      if (s == 0 && fuse_p)
        v_jacobi_prolong<T>(v, vops<T>(l + 1), bl[l], cur[l], oth[l], omega, cur[l + 1], R, cs, st);
      else if (l == 0 && fuse_dot && s == d_.post - 1)
        v_jacobi_dot<T>(v, bl[l], cur[l], oth[l], omega, r_in, q_, R, cs, red_, st);
      else
        v_jacobi<T>(v, bl[l], cur[l], oth[l], omega, R, cs, st);
      if (l == 0) timed_end(2);
      std::swap(cur[l], oth[l]);
    }
  }
  zbuf_ = cur[0];
}

// ------------------------------------------------------------------ PCG
// z = M r, then the new search direction p = z + beta p.  With a post-smoothing
// sweep on a multilevel hierarchy the r.z products come fused out of the last
// finest-level sweep; otherwise a separate dot kernel computes them.
VPrep Problem::vprep() const {
  // the residual producers write the V-cycle's level-0 input (multilevel
  // only; the Gauss-Seidel smoother starts from zero itself)
  if (lv_.size() < 2 || gs_smoother()) return VPrep{nullptr, nullptr, nullptr, 0};
  return VPrep{B_[0].invD, B_[0].xa, vbytes_ == 4 ? B_[0].b : nullptr, vbytes_ == 4 ? 1 : 0};
}

void Problem::precondition_and_direction(bool x0_ready) {
  hipStream_t st = stream_;
  const long nd = lv_[0].L.ndof();
  const int R = d_.nrhs;
  const bool fuse = d_.post >= 1 && lv_.size() > 1 && !gs_smoother();
  const int nbz = fuse ? nblocks_fine(vbytes_ == 8) : cg_beta_blocks(nd);
  if (vbytes_ == 8) {
    vcycle<double>(r_, 1, fuse, x0_ready);
    if (!fuse) cg_beta<double>(r_, q_, (const double*)zbuf_, nd, R, cs_, red_, st);
    cg_update_p<double>((const double*)zbuf_, p_, nd, R, cs_, red_, nbz, st);
  } else {
    vcycle<float>(r_, 1, fuse, x0_ready);
    if (!fuse) cg_beta<float>(r_, q_, (const float*)zbuf_, nd, R, cs_, red_, st);
    cg_update_p<float>((const float*)zbuf_, p_, nd, R, cs_, red_, nbz, st);
  }
}

void Problem::iteration() {
  hipStream_t st = stream_;
  const FineOp A = fine_op();
  const long nd = lv_[0].L.ndof();
  const int R = d_.nrhs;
  timed_begin(0);
  cg_apply_alpha(A, p_, q_, R, cs_, red_, st);
  timed_end(0);
  const VPrep vp = vprep();
  cg_update_xr(p_, q_, x_, r_, nd, R, cs_, red_, nblocks_fine(true), vp, st);
  cg_true_residual(A, f_, x_, r_, R, cs_, red_, vp, st);
  precondition_and_direction(vp.x0 != nullptr);
  ++iter_launched_;
}

void Problem::solve_begin(double rtol, int maxit, int warm) {
  if (!have_ops_) throw Error(MGCG_ESTATE, "set_densities must precede solve");
  if (!(rtol > 0.0) || maxit < 1) throw Error(MGCG_EINVAL, "need rtol > 0 and maxit >= 1");
  MGCG_HIP(hipSetDevice(device_));
  hipStream_t st = stream_;
  const FineOp A = fine_op();
  const long nd = lv_[0].L.ndof();
  const int R = d_.nrhs;
  rtol_ = rtol;
  maxit_ = maxit;
  t0_ = std::chrono::steady_clock::now();
  const bool from_u = warm != MGCG_COLD && have_u_;
  if (!from_u) fill<double>(x_, 0.0, R * nd, st);
  cg_reset(cs_, R, rtol * rtol, maxit, replace_every_, vbytes_ == 4 ? 1 : 0, st);
  cg_init_residual(A, f_, x_, r_, R, cs_, red_, st);
  if (from_u && warm == MGCG_WARM_SCALED) cg_scale_warm(f_, x_, r_, nd, R, cs_, red_, st);
  fill<double>(p_, 0.0, R * nd, st);
  fill<double>(q_, 0.0, R * nd, st);  // read by the first direction's flexible beta
  iter_launched_ = -1;
  timer_used_base_ = timer_.used;
  precondition_and_direction();
  iter_launched_ = 0;
  first_chunk_ = true;
  // read the initial state
  MGCG_HIP(hipMemcpyAsync(hcs_, cs_, 4 * sizeof(CgScalars), hipMemcpyDeviceToHost, st));
  MGCG_HIP(hipEventRecord(ev_chunk_, st));
  chunk_pending_ = true;
  prev_rr_valid_ = false;
}

void Problem::solve_chunk(int iters) {
  hipStream_t st = stream_;
  if (launch_mode_ == MGCG_LAUNCH_GRAPH && !timer_.enabled) {
    if (!iter_exec_) build_iter_graph();
    for (int i = 0; i < iters; ++i) MGCG_HIP(hipGraphLaunch(iter_exec_, st));
    iter_launched_ += iters;
  } else {
    for (int i = 0; i < iters; ++i) iteration();
  }
  MGCG_HIP(hipMemcpyAsync(hcs_, cs_, 4 * sizeof(CgScalars), hipMemcpyDeviceToHost, st));
  MGCG_HIP(hipEventRecord(ev_chunk_, st));
  chunk_pending_ = true;
}

// Every kernel of an iteration takes the same arguments in every iteration
// (buffers of the arena, operator data; the iteration's parity and the
// per-load-case state live on the device), so one captured iteration serves
// every later one until the arena is released.  The capture runs on a
// private stream (the problem's own may be the null stream, which cannot be
// captured); the graph holds kernel nodes only.
void Problem::build_iter_graph() {
  hipStream_t cap = nullptr;
  MGCG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipStream_t saved = stream_;
  const int saved_it = iter_launched_;
  hipGraph_t g = nullptr;
  stream_ = cap;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    try {
      iteration();
    } catch (...) {
      (void)hipStreamEndCapture(cap, &g);
      if (g) (void)hipGraphDestroy(g);
      stream_ = saved;
      iter_launched_ = saved_it;
      (void)hipStreamDestroy(cap);
      throw;
    }
    e = hipStreamEndCapture(cap, &g);
  }
  stream_ = saved;
  iter_launched_ = saved_it;
  if (e == hipSuccess) e = hipGraphInstantiate(&iter_exec_, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    iter_exec_ = nullptr;
    throw Error(MGCG_EDEVICE, std::string("capturing the PCG iteration: ") + hipGetErrorString(e));
  }
}

void Problem::drop_iter_graph() {
  if (iter_exec_) (void)hipGraphExecDestroy(iter_exec_);
  iter_exec_ = nullptr;
}

void Problem::set_launch_mode(int mode) {
  if (mode != MGCG_LAUNCH_EAGER && mode != MGCG_LAUNCH_GRAPH && mode != MGCG_LAUNCH_FUSED)
    throw Error(MGCG_EINVAL,
                "launch mode must be MGCG_LAUNCH_EAGER, MGCG_LAUNCH_GRAPH or MGCG_LAUNCH_FUSED");
  if (mode == MGCG_LAUNCH_FUSED && !fused_ok())
    throw Error(MGCG_EINVAL,
                "the fused solve needs trilinear elements with nsub = 1, FP64, the Jacobi smoother, "
                "2..8 levels, at most 6000 finest-level nodes and 1024 coarsest DOFs");
  launch_mode_ = mode;
}

// ------------------------------------------------------------------ fused solve
bool Problem::fused_ok(const mgcg_desc& d, const std::vector<LevelPlan>& lv) {
  if (d.order != 1 || d.nsub != 1 || d.precision != MGCG_FP64 || d.smoother != MGCG_SMOOTH_JACOBI)
    return false;
  if (lv.size() < 2 || lv.size() > (size_t)FZ_MAXLEV) return false;
  for (size_t l = 1; l + 1 < lv.size(); ++l)
    if (((lv[l].L.nn() + 63) & ~63L) > FZ_MAX_ST_NODES) return false;
  return lv[0].kind == OP_MF_Q1 && lv[0].L.nn() <= FZ_MAX_NODES &&
         lv.back().L.ndof() <= FZ_MAX_COARSE;
}

void Problem::fused_prepare(double rtol, int maxit, int warm, std::vector<FzDesc>& out) {
  if (!have_ops_) throw Error(MGCG_ESTATE, "set_densities must precede solve");
  if (!(rtol > 0.0) || maxit < 1) throw Error(MGCG_EINVAL, "need rtol > 0 and maxit >= 1");
  if (!fz_) throw Error(MGCG_EINVAL, "this problem does not fit the fused solve");
  MGCG_HIP(hipSetDevice(device_));
  const long nd = lv_[0].L.ndof();
  const int R = d_.nrhs, L = (int)lv_.size();
  rtol_ = rtol;
  maxit_ = maxit;
  t0_ = std::chrono::steady_clock::now();
  const bool from_u = warm != MGCG_COLD && have_u_;
  if (!from_u) fill<double>(x_, 0.0, R * nd, stream_);
  timer_used_base_ = timer_.used;
  out.assign(R, FzDesc{});
  for (int r = 0; r < R; ++r) {
    FzDesc& z = out[r];
    z.nlev = L;
    z.pre = d_.pre;
    z.post = d_.post;
    z.maxit = maxit;
    z.scale_warm = from_u && warm == MGCG_WARM_SCALED ? 1 : 0;
    z.tol2 = rtol * rtol;
    z.E = E_;
    z.hv = hv64_;
    z.Ainv = Ainv_;
    z.ld = coarse_ld(lv_.back().L.ndof());
    z.f = f_ + r * nd;
    z.x = x_ + r * nd;
    z.r = r_ + r * nd;
    z.p = p_ + r * nd;
    z.cs = cs_ + r;
    for (int l = 0; l < L; ++l) {
      FzLevel& v = z.lv[l];
      const long ndl = lv_[l].L.ndof();
      v.L = lv_[l].L;
      v.coef = l ? (const double*)B_[l].coefV : nullptr;
      v.wD = (const double*)B_[l].invD;
      v.mask = B_[l].mask;
      v.b = (double*)B_[l].b + r * ndl;
      v.x = (double*)B_[l].xa + r * ndl;
      v.r = (double*)B_[l].r + r * ndl;
    }
  }
}

int Problem::fused_finish(mgcg_info* info) {
  MGCG_HIP(hipMemcpyAsync(hcs_, cs_, 4 * sizeof(CgScalars), hipMemcpyDeviceToHost, stream_));
  sync();
  chunk_pending_ = false;
  active_ = false;
  return solve_finish(info);
}

int Problem::fused_finish(const FzRecord& rec, mgcg_info* info) {
  std::memcpy(hcs_, rec.cs, d_.nrhs * sizeof(CgScalars));
  chunk_pending_ = false;
  active_ = false;
  return solve_finish(info, rec.bad);
}

int Problem::solve_fused(double rtol, int maxit, int warm, mgcg_info* info) {
  std::vector<FzDesc> h;
  fused_prepare(rtol, maxit, warm, h);
  MGCG_HIP(hipMemcpyAsync(fz_, h.data(), h.size() * sizeof(FzDesc), hipMemcpyHostToDevice, stream_));
  fused_solve(fz_, (int)h.size(), stream_);
  return fused_finish(info);
}

bool Problem::solve_poll(bool block) {
  if (chunk_pending_) {
    if (block) {
      MGCG_HIP(hipEventSynchronize(ev_chunk_));
    } else {
      hipError_t e = hipEventQuery(ev_chunk_);
      if (e == hipErrorNotReady) return false;
      if (e != hipSuccess) throw Error(MGCG_EDEVICE, hipGetErrorString(e));
    }
    chunk_pending_ = false;
    // convergence-rate estimate for the next chunk length
    double worst = 0.0;
    int itmax = 0;
    bool any = false;
    for (int r = 0; r < d_.nrhs; ++r) {
      const CgScalars& c = hcs_[r];
      itmax = std::max(itmax, c.iters);
      if (c.state == CG_ACTIVE || c.state == CG_CHECK) {
        any = true;
        const double ratio = (c.tol2 > 0 && c.rr > 0) ? c.rr / c.tol2 : 1.0;
        worst = std::max(worst, ratio);
      }
    }
    if (prev_rr_valid_ && any && itmax > prev_iters_ && worst > 0 && prev_worst_ > 0) {
      const double f = std::log(worst / prev_worst_) / (itmax - prev_iters_);
      if (f < -1e-3) rate_log_ = f;  // log of the per-iteration factor of rr
    }
    prev_worst_ = worst;
    prev_iters_ = itmax;
    prev_rr_valid_ = any;
    active_ = any;
  }
  return !active_;
}

void Problem::solve_abort() {
  MGCG_HIP(hipSetDevice(device_));
  if (stream_) MGCG_HIP(hipStreamSynchronize(stream_));
  chunk_pending_ = false;
  active_ = false;
}

int Problem::suggest_chunk() const {
  int n = 4;
  if (prev_rr_valid_ && rate_log_ < 0 && prev_worst_ > 1.0)
    n = (int)std::ceil(std::log(prev_worst_) / -rate_log_);
  int left = maxit_ - prev_iters_;
  n = std::max(1, std::min(n, 32));
  return std::max(1, std::min(n, std::max(left, 1)));
}

int Problem::solve_finish(mgcg_info* info, const int* bad) {
  const auto t1 = std::chrono::steady_clock::now();
  int status = MGCG_OK;
  if (pending_check_) {
    pending_check_ = false;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev_s0_, ev_s1_) == hipSuccess) setup_ms_ = ms;
    int hb[4] = {0, 0, 0, 0};
    if (bad) {
      std::memcpy(hb, bad, sizeof(hb));
    } else {
      MGCG_HIP(hipMemcpyAsync(hb, bad_, sizeof(hb), hipMemcpyDeviceToHost, stream_));
      sync();
    }
    if (hb[0] & 1) status = MGCG_EINVAL;
    else if (hb[0] & 2) status = MGCG_EBREAKDOWN;
  }
  int itmax = 0;
  for (int r = 0; r < d_.nrhs; ++r) {
    const CgScalars& c = hcs_[r];
    itmax = std::max(itmax, c.iters);
    if (c.state == CG_BREAKDOWN && status >= 0) status = MGCG_EBREAKDOWN;
    else if (c.state == CG_MAXIT && status == MGCG_OK) status = MGCG_ENOTCONV;
  }
  harvest_timing(itmax);
  have_u_ = true;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = status;
    for (int r = 0; r < d_.nrhs && r < 4; ++r) {
      const CgScalars& c = hcs_[r];
      info->iters[r] = c.iters;
      info->rel_res[r] = c.ff > 0 ? std::sqrt(std::max(c.rr, 0.0) / c.ff) : 0.0;
      info->replacements += c.replacements;
    }
    info->t_setup_ms = setup_ms_;
    info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0_).count();
  }
  return status;
}

int Problem::solve(double rtol, int maxit, int warm, mgcg_info* info) {
  if (launch_mode_ == MGCG_LAUNCH_FUSED && !timer_.enabled) return solve_fused(rtol, maxit, warm, info);
  solve_begin(rtol, maxit, warm);
  solve_poll(true);
  while (active_) {
    solve_chunk(suggest_chunk());
    solve_poll(true);
  }
  return solve_finish(info);
}

// ------------------------------------------------------------------ outputs
void Problem::get_u(double* u, int mem) {
  if (!arena_) throw Error(MGCG_ESTATE, "no solution");
  const size_t n = (size_t)d_.nrhs * lv_[0].L.ndof();
  MGCG_HIP(hipMemcpyAsync(u, x_, n * sizeof(double),
                          mem == MGCG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          stream_));
  sync();
}

void Problem::set_u(const double* u, int mem) {
  allocate();
  const long nd = lv_[0].L.ndof();
  const size_t n = (size_t)d_.nrhs * nd;
  MGCG_HIP(hipMemcpyAsync(x_, u, n * sizeof(double),
                          mem == MGCG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          stream_));
  // zero the fixed DOFs: identity rows of the system with zero load there
  std::vector<double> h(n);
  MGCG_HIP(hipMemcpyAsync(h.data(), x_, n * sizeof(double), hipMemcpyDeviceToHost, stream_));
  sync();
  for (int r = 0; r < d_.nrhs; ++r)
    for (long i = 0; i < nd; ++i)
      if ((hmask_[i / 3] >> (i % 3)) & 1) h[(size_t)r * nd + i] = 0.0;
  MGCG_HIP(hipMemcpyAsync(x_, h.data(), n * sizeof(double), hipMemcpyHostToDevice, stream_));
  sync();
  have_u_ = true;
}

void Problem::compliance_sensitivity(double* c, double* dc, int mem) {
  if (!have_u_ || !have_ops_) throw Error(MGCG_ESTATE, "solve first");
  hipStream_t st = stream_;
  const long nd = lv_[0].L.ndof();
  const int R = d_.nrhs;
  comp_dot(f_, x_, nd, R, compout_, red_, st);
  if (dc) {
    double* out = mem == MGCG_MEM_DEVICE ? dc : dcbuf_;
    sens_kernel(d_.order, d_.nsub, d_.nelx, d_.nely, d_.nelz, lv_[0].L, rho_, x_, nd, R,
                lv_[0].kind == OP_MF_Q1 ? K0_ : Ksub_, Kp_, d_.E0 - d_.Emin, d_.penal, out, st);
    if (mem != MGCG_MEM_DEVICE)
      MGCG_HIP(hipMemcpyAsync(dc, dcbuf_, nrho() * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  double h[16];
  MGCG_HIP(hipMemcpyAsync(h, compout_, R * sizeof(double), hipMemcpyDeviceToHost, st));
  sync();
  double s = 0.0;
  for (int r = 0; r < R; ++r) {
    c[r] = h[r];
    s += h[r];
  }
  c[R] = s;
}

// ------------------------------------------------------------------ inspection
void Problem::level_dims(int level, int32_t* dims, int64_t* ndof) const {
  if (level < 0 || level >= (int)lv_.size()) throw Error(MGCG_EINVAL, "level out of range");
  const Lat L = lv_[level].L;
  if (dims) {
    dims[0] = L.nx;
    dims[1] = L.ny;
    dims[2] = L.nz;
  }
  if (ndof) *ndof = L.ndof();
}

namespace {
struct DevTmp {
  std::vector<void*> ptrs;
  ~DevTmp() {
    for (void* p : ptrs) hipFree(p);
  }
  template <class T>
  T* get(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess)
      throw Error(MGCG_ENOMEM, "inspection scratch allocation failed");
    ptrs.push_back(p);
    return (T*)p;
  }
};
}  // namespace

static void to_dev(const double* src, double* dst, size_t n, int mem, hipStream_t st) {
  MGCG_HIP(hipMemcpyAsync(dst, src, n * sizeof(double),
                          mem == MGCG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
}
static void from_dev(const double* src, double* dst, size_t n, int mem, hipStream_t st) {
  MGCG_HIP(hipMemcpyAsync(dst, src, n * sizeof(double),
                          mem == MGCG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
}

template <typename T>
void Problem::do_apply_v(int level, const double* x, double* y) {
  DevTmp tmp;
  const long nd = lv_[level].L.ndof();
  const int R = d_.nrhs;
  const VOps<T> v = vops<T>(level);
  const T* xt;
  T* yt;
  if constexpr (sizeof(T) == 8) {
    xt = x;
    yt = y;
  } else {
    T* a = tmp.get<T>(R * nd);
    T* b = tmp.get<T>(R * nd);
    convert<double, float>(x, a, R * nd, stream_);
    xt = a;
    yt = b;
  }
  switch (v.kind) {
    case OP_MF_Q1: launch_apply_mf<T>(v.mf, xt, yt, R, stream_); break;
    case OP_ST27: launch_apply_st<T>(v.st, xt, yt, R, stream_); break;
    default: launch_apply_eq2<T>(v.eq2, xt, yt, R, stream_); break;
  }
  if constexpr (sizeof(T) == 4) convert<float, double>(yt, y, R * nd, stream_);
  sync();
}

void Problem::apply(int level, int prec, const double* x, double* y, int mem) {
  if (!have_ops_) throw Error(MGCG_ESTATE, "set_densities first");
  if (level < 0 || level >= (int)lv_.size()) throw Error(MGCG_EINVAL, "level out of range");
  DevTmp tmp;
  const long nd = lv_[level].L.ndof();
  const size_t n = (size_t)d_.nrhs * nd;
  double* xraw = tmp.get<double>(n);
  double* xd = tmp.get<double>(n);
  double* yd = tmp.get<double>(n);
  to_dev(x, xraw, n, mem, stream_);
  // A = Z K Z + (I - Z): the kernels take inputs that vanish on fixed DOFs
  mask_copy(xraw, xd, B_[level].mask, lv_[level].L.nn(), d_.nrhs, stream_);
  if (level == 0 && (prec == MGCG_FP64 || vbytes_ == 8)) {
    const FineOp A = fine_op();
    switch (A.kind) {
      case OP_MF_Q1: launch_apply_mf<double>(A.mf, xd, yd, d_.nrhs, stream_); break;
      case OP_ST27: launch_apply_st<double>(A.st, xd, yd, d_.nrhs, stream_); break;
      default: launch_apply_eq2<double>(A.eq2, xd, yd, d_.nrhs, stream_); break;
    }
  } else if (vbytes_ == 8) {
    do_apply_v<double>(level, xd, yd);
  } else {
    do_apply_v<float>(level, xd, yd);
  }
  identity_rows(xraw, yd, B_[level].mask, lv_[level].L.nn(), d_.nrhs, stream_);
  from_dev(yd, y, n, mem, stream_);
  sync();
}

void Problem::diag(int level, double* d, int mem) {
  if (!have_ops_) throw Error(MGCG_ESTATE, "set_densities first");
  if (level < 0 || level >= (int)lv_.size()) throw Error(MGCG_EINVAL, "level out of range");
  from_dev(B_[level].diag64, d, lv_[level].L.ndof(), mem, stream_);
  sync();
}

void Problem::restrict_(int level, const double* f, double* c, int mem) {
  if (!arena_) allocate();
  if (level < 0 || level + 1 >= (int)lv_.size()) throw Error(MGCG_EINVAL, "level out of range");
  DevTmp tmp;
  const long nf = (long)d_.nrhs * lv_[level].L.ndof(), ncd = (long)d_.nrhs * lv_[level + 1].L.ndof();
  double* fraw = tmp.get<double>(nf);
  double* fd = tmp.get<double>(nf);
  double* cd = tmp.get<double>(ncd);
  to_dev(f, fraw, nf, mem, stream_);
  mask_copy(fraw, fd, B_[level].mask, lv_[level].L.nn(), d_.nrhs, stream_);
  v_restrict<double>(lv_[level].L, lv_[level + 1].L, B_[level].mask, B_[level + 1].mask, fd, cd,
                     nullptr, nullptr,
                     d_.nrhs, nullptr, stream_);
  from_dev(cd, c, ncd, mem, stream_);
  sync();
}

void Problem::prolong(int level, const double* c, double* f, int mem) {
  if (!arena_) allocate();
  if (level < 0 || level + 1 >= (int)lv_.size()) throw Error(MGCG_EINVAL, "level out of range");
  DevTmp tmp;
  const long nf = (long)d_.nrhs * lv_[level].L.ndof(), ncd = (long)d_.nrhs * lv_[level + 1].L.ndof();
  double* fd = tmp.get<double>(nf);
  double* craw = tmp.get<double>(ncd);
  double* cd = tmp.get<double>(ncd);
  to_dev(c, craw, ncd, mem, stream_);
  mask_copy(craw, cd, B_[level + 1].mask, lv_[level + 1].L.nn(), d_.nrhs, stream_);
  v_prolong<double>(lv_[level].L, lv_[level + 1].L, B_[level].mask, B_[level + 1].mask, cd, fd,
                    d_.nrhs, false, nullptr, stream_);
  from_dev(fd, f, nf, mem, stream_);
  sync();
}

void Problem::precondition(const double* r, double* z, int mem) {
  if (!have_ops_) throw Error(MGCG_ESTATE, "set_densities first");
  const long n = (long)d_.nrhs * lv_[0].L.ndof();
  to_dev(r, tmp64_, n, mem, stream_);
  if (vbytes_ == 8) {
    vcycle<double>(tmp64_, 0, false);
    from_dev((const double*)zbuf_, z, n, mem, stream_);
  } else {
    vcycle<float>(tmp64_, 0, false);
    DevTmp tmp;
    double* zd = tmp.get<double>(n);
    convert<float, double>((const float*)zbuf_, zd, n, stream_);
    from_dev(zd, z, n, mem, stream_);
    sync();
  }
  sync();
}

void Problem::coarse_solve(const double* b, double* x, int mem) {
  if (!have_ops_) throw Error(MGCG_ESTATE, "set_densities first");
  DevTmp tmp;
  const int lc = (int)lv_.size() - 1;
  const long n = (long)d_.nrhs * lv_[lc].L.ndof();
  double* bd = tmp.get<double>(n);
  double* xd = tmp.get<double>(n);
  to_dev(b, bd, n, mem, stream_);
  fill<double>(xd, 0.0, n, stream_);
  v_coarse_solve<double>(Ainv_, coarse_ld(lv_[lc].L.ndof()), lv_[lc].L.ndof(), bd, xd, d_.nrhs,
                         nullptr, stream_);
  from_dev(xd, x, n, mem, stream_);
  sync();
}

// ------------------------------------------------------------------ timing
void Problem::set_timing(bool on, int kernel) {
  timer_.enabled = on;
  timer_.kernel = kernel;
  timer_.total_ms = 0.0;
  timer_.launches = 0;
  timer_.recs.clear();
}

void Problem::timed_begin(int id) {
  if (!timer_.enabled || id != timer_.kernel) return;
  if (timer_.used >= timer_.pool.size()) {
    hipEvent_t a, b;
    MGCG_HIP(hipEventCreate(&a));
    MGCG_HIP(hipEventCreate(&b));
    timer_.pool.push_back({a, b});
  }
  time_next_apply(timer_.pool[timer_.used].first, timer_.pool[timer_.used].second);
}

void Problem::timed_end(int id) {
  if (!timer_.enabled || id != timer_.kernel) return;
  timer_.recs.push_back(iter_launched_);
  ++timer_.used;
}

void Problem::harvest_timing(int itmax) {
  if (!timer_.enabled) {
    timer_.used = 0;
    return;
  }
  // launches of iterations after every load case converged were no-ops
  for (size_t i = timer_used_base_; i < timer_.used; ++i) {
    const int it = timer_.recs[i];
    // the CG apply of iteration i works iff some load case needs i+1 iterations;
    // the V-cycle of iteration i (i = -1: the initial one) iff one needs i+2
    if (timer_.kernel == 0 && it >= itmax) continue;
    if (timer_.kernel != 0 && it >= itmax - 1) continue;
    float ms = 0.f;
    MGCG_HIP(hipEventElapsedTime(&ms, timer_.pool[i].first, timer_.pool[i].second));
    timer_.total_ms += ms;
    timer_.launches += 1;
  }
  timer_.used = 0;
  timer_.recs.clear();
}

void Problem::get_timing(int kernel, double* ms, long long* launches) {
  (void)kernel;
  if (ms) *ms = timer_.total_ms;
  if (launches) *launches = timer_.launches;
}

void Problem::copy(const void* src, void* dst, size_t bytes) {
  allocate();
  copy_bytes(src, dst, bytes, stream_);
  sync();
}

}  // namespace mgcg
