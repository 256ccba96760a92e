// Device-side operator views and kernel launchers (host-callable).
#pragma once

#include "common.h"
#include "q1table.h"

#include <vector>

namespace mgcg {

// Node lattice of a level.
struct Lat {
  int nx, ny, nz;
  __host__ __device__ long nn() const { return (long)nx * ny * nz; }
  __host__ __device__ long ndof() const { return 3L * nx * ny * nz; }
};

// Matrix-free trilinear operator: elements (nx-1)(ny-1)(nz-1), modulus E per
// element, the shared unit element matrix in its Haar basis as class values
// (kept in scalar registers), supports in mask (bit c of a node's byte =
// component c fixed).  Inputs must vanish on fixed DOFs (every solver vector
// does); fixed rows return 0.
template <typename T>
struct OpMF {
  Lat L;
  const T* E;
  Q1HaarVals<T> hv;
  const uint8_t* mask;
  static OpMF make(Lat L, const T* E, Q1HaarVals<T> hv, const uint8_t* mask) {
    return OpMF{L, E, hv, mask};
  }
};

// Assembled 27-point block stencil, symmetric half storage: coef[(b*9 + 3c + e) * nn + node]
// holds A_{node, node + d_b}(c, e) for the 14 blocks of st_offset; supports are
// baked in (identity rows/columns).
template <typename T>
struct OpST {
  Lat L;
  const T* coef;
};

// Stored triquadratic element matrices (supported rows/columns zeroed), on
// the quadratic node lattice (nx = 2*nelx + 1, ...), by wrapped diagonals:
// Ke[e][s][i] = K_e[i][(i + s) mod 81] for s = 0..40, i = 0..80 (each entry
// of the symmetric matrix once).
constexpr int Q2_PACKED = 41 * 81;
// The 20-node serendipity element's 60 DOFs by wrapped diagonals, s = 0..30
// (the diagonal s = 30 holds each of its values twice).
constexpr int S2_PACKED = 31 * 60;
// Node of the 27-node layout (a = ax + 3 ay + 9 az) of serendipity node k
// (0..19, in increasing a): the vertices and edge midpoints, those with at
// most one local coordinate at the middle.
__host__ __device__ inline int s2_node(int k) {
  int a = 0;
  for (int m = -1;; ++a) {
    const int mid = (a % 3 == 1) + ((a / 3) % 3 == 1) + (a / 9 == 1);
    if (mid <= 1 && ++m == k) return a;
  }
}
// Tricubic elements on the cubic node lattice (nx = 3*nelx + 1, ...): the
// 64-node element's 192 DOFs, or the 32-node serendipity element's 96, by
// wrapped diagonals s = 0..N/2 (N the DOF count; the diagonal s = N/2 holds
// each of its values twice).
constexpr int L3_ND = 192, S3_ND = 96;
constexpr int L3_PACKED = (L3_ND / 2 + 1) * L3_ND;
constexpr int S3_PACKED = (S3_ND / 2 + 1) * S3_ND;
// Node of the 64-node layout (a = ax + 4 ay + 16 az) of serendipity node k
// (0..31, in increasing a): the vertices and the edges' third-points, those
// with at most one local index inside the edge (1 or 2).
__host__ __device__ inline int s3_node(int k) {
  int a = 0;
  for (int m = -1;; ++a) {
    const int ax = a % 4, ay = (a / 4) % 4, az = a / 16;
    const int in = (ax == 1 || ax == 2) + (ay == 1 || ay == 2) + (az == 1 || az == 2);
    if (in <= 1 && ++m == k) return a;
  }
}
// Stored element matrices of degree p = 2 or 3 (OP_EQ2 / OP_EQ3).
template <typename T>
struct OpEQ2 {
  Lat L;
  const T* Ke;
  const uint8_t* mask;
  T* Y;  // element products K_e u_e, [load case][element][3 (p+1)^3] (scratch of the apply)
  int s2;  // serendipity elements: Ke holds S2_PACKED (S3_PACKED) values per element
  int p;   // element degree
};

// Reduction scratch: one partial sum per block and value, in regions that
// stay untouched until their consumer has read them:
//   partials[region * RED_REGION + v * MAX_BLOCKS + block], v < 8.
// Workgroups (and hence reduction partials) of one operator apply on the
// lattice L: kind OpKind, fp64 = the FP64 instantiation.
int apply_blocks(int kind, const Lat& L, bool fp64);

// Attach the events to the next operator launch on this thread (they then
// hold that kernel's own start and end timestamps).
void time_next_apply(hipEvent_t start, hipEvent_t stop);

struct RedBuf {
  double* partials;
};
constexpr int MAX_BLOCKS = 16384;
constexpr long RED_REGION = 8L * MAX_BLOCKS;
enum RedRegion : int { RED_PQ = 0, RED_RR = 1, RED_TR = 2, RED_INIT = 3, RED_RZ = 4, RED_COMP = 5,
                       RED_NREGIONS = 6 };

// ---------------- launchers ----------------
// All launchers enqueue on `st`; nrhs vectors are stored back to back with
// stride ndof of the level.

// Generic apply y = A x (A = Z K Z + I - Z) for parity inspection.
template <typename T> void launch_apply_mf(const OpMF<T>& op, const T* x, T* y, int nrhs, hipStream_t st);
template <typename T> void launch_apply_st(const OpST<T>& op, const T* x, T* y, int nrhs, hipStream_t st);
template <typename T> void launch_apply_eq2(const OpEQ2<T>& op, const T* x, T* y, int nrhs, hipStream_t st);

// Fine-level FP64 CG operator, one of the three kinds.
struct FineOp {
  int kind;
  OpMF<double> mf;
  OpST<double> st;
  OpEQ2<double> eq2;
  Lat lat() const { return kind == OP_MF_Q1 ? mf.L : kind == OP_ST27 ? st.L : eq2.L; }
};

// CG kernels (FP64), state gated.
void cg_reset(CgScalars* cs, int nrhs, double rtol2, int maxit, int replace_every, int flexible,
              hipStream_t st);
void cg_init_residual(const FineOp& A, const double* f, const double* x, double* r, int nrhs,
                      CgScalars* cs, RedBuf red, hipStream_t st);
// After cg_init_residual from a warm start x (r = f - A x): x <- alpha x,
// r <- f - alpha A x = (1 - alpha) f + alpha r with alpha = f.x / x.(f - r)
// per load case (0 unless x^T A x > 0 and alpha is finite); ||r||^2 and the
// state are refreshed.
void cg_scale_warm(const double* f, double* x, double* r, long ndof, int nrhs, CgScalars* cs,
                   RedBuf red, hipStream_t st);
void cg_apply_alpha(const FineOp& A, const double* p, double* q, int nrhs, CgScalars* cs,
                    RedBuf red, hipStream_t st);
// nbq: blocks per load case of the apply that produced the p.q partials.
// The level-0 input of the next V-cycle, written by the kernels that produce
// the residual r: the first smoothing sweep from zero x0 = W D^-1 r (and, for
// an FP32 V-cycle, b0 = r rounded to FP32).  x0 == nullptr: not written.
struct VPrep {
  const void* wD;  // per DOF, V-cycle precision
  void* x0;
  void* b0;        // FP32 V-cycle only
  int f32;
};
void cg_update_xr(const double* p, const double* q, double* x, double* r, long ndof, int nrhs,
                  CgScalars* cs, RedBuf red, int nbq, VPrep vp, hipStream_t st);
void cg_true_residual(const FineOp& A, const double* f, const double* x, double* r, int nrhs,
                      CgScalars* cs, RedBuf red, VPrep vp, hipStream_t st);
template <typename TZ>
void cg_beta(const double* r, const double* q, const TZ* z, long ndof, int nrhs, CgScalars* cs,
             RedBuf red, hipStream_t st);
// nbz: number of r.z partials per load case (cg_beta_blocks, or the blocks of
// the finest-level fused Jacobi sweep).
template <typename TZ>
void cg_update_p(const TZ* z, double* p, long ndof, int nrhs, CgScalars* cs, RedBuf red, int nbz,
                 hipStream_t st);
int cg_beta_blocks(long ndof);

// V-cycle level kernels in precision T (gated by any active CG state; cs may be null).
struct VLevelArgs;  // fwd
template <typename T>
struct VOps {
  int kind;  // operator kind of this level
  OpMF<T> mf;
  OpST<T> st;
  OpEQ2<T> eq2;
  const T* invD;
  const uint8_t* mask;
  Lat L;
};
// Level-0 V-cycle input: b0 = r in precision T (b0 may be null when T is
// FP64 and r serves directly) and x0 = W D^-1 b0 (first sweep from zero).
template <typename T>
void v_prepare0(const double* r, T* b0, const T* wD, T* x0, long ndof, int nrhs,
                const CgScalars* cs, hipStream_t st);
// One multicolour Gauss-Seidel sweep (relaxation 1) in place on a finest
// level of degree order = 2 or 3: (order+1)^3 launches, one per node colour
// (lattice indices mod order + 1), colours and a node's components in
// increasing order, or both reversed (backward).  Kn: element rows by node
// (setup_rows_by_node).
template <typename T>
void v_gauss_seidel(int order, const Lat& L, const T* Kn, const T* Dn, const uint8_t* mask,
                    const T* b, T* x, bool backward, int nrhs, const CgScalars* cs, hipStream_t st);
// Kn[((e * NEN + a) * ND + j) * 3 + c] = Keff[e][3a + c][j] in precision T
// (NEN = (order+1)^3 nodes, ND = 3 NEN DOFs per element).
template <typename T>
void setup_rows_by_node(int order, const double* Keff, T* Kn, long nel, hipStream_t st);
// Dn[node * 9 + 3 c + c'] = the node's 3x3 diagonal block, summed over its elements.
template <typename T>
void setup_gs_diag(int order, const Lat& L, const T* Kn, T* Dn, hipStream_t st);
// xo = x + omega invD (b - A x)
template <typename T>
void v_jacobi(const VOps<T>& v, const T* b, const T* x, T* xo, T omega, int nrhs,
              const CgScalars* cs, hipStream_t st);
// xo = x + wD (b - A x) and the CG partials r.z, r_old.z of xo (= z)
template <typename T>
void v_jacobi_dot(const VOps<T>& v, const T* b, const T* x, T* xo, T omega, const double* r,
                  const double* q, int nrhs, const CgScalars* cs, RedBuf red, hipStream_t st);
// First post-smoothing sweep of a small stencil level fused with the
// prolongation: xo = y + wD (b - A y) with y = x + P~ e (e on the coarser
// level vc); y itself is not stored.
template <typename T>
void v_jacobi_prolong(const VOps<T>& v, const VOps<T>& vc, const T* b, const T* x, T* xo,
                      T omega, const T* e, int nrhs, const CgScalars* cs, hipStream_t st);
// Levels at most this many nodes take the fused sweep above.
constexpr long PROLONG_FUSE_MAX_NODES = 65536;
// r = b - A x
template <typename T>
void v_residual(const VOps<T>& v, const T* b, const T* x, T* r, int nrhs, const CgScalars* cs,
                hipStream_t st);
// coarse = P~^T fine; when xc is given also xc = wDc * coarse (the coarse
// level's first smoothing sweep from zero)
template <typename T>
void v_restrict(Lat fine, Lat coarse, const uint8_t* mask_f, const uint8_t* mask_c, const T* rf,
                T* bc, const T* wDc, T* xc, int nrhs, const CgScalars* cs, hipStream_t st);
// Coarsest solve with the last restriction fused in: x = A_c^{-1} P~^T r_f,
// for coarsest levels of at most CS_FUSE_MAX DOFs.
constexpr int CS_FUSE_MAX = 1024;
template <typename T>
void v_coarse_solve_r(const double* Ainv, int ld, Lat fine, Lat coarse, const uint8_t* mask_c,
                      const T* rf, T* x, int nrhs, const CgScalars* cs, hipStream_t st);
// fine += P~ coarse  (accumulate=false: fine = P~ coarse)
template <typename T>
void v_prolong(Lat fine, Lat coarse, const uint8_t* mask_f, const uint8_t* mask_c, const T* ec,
               T* xf, int nrhs, bool accumulate, const CgScalars* cs, hipStream_t st);
// x = A_c^{-1} b on the coarsest level: Ainv is the dense inverse over all
// of the level's DOFs (identity rows and columns at fixed DOFs), row stride
// ld >= ndof.
template <typename T>
void v_coarse_solve(const double* Ainv, int ld, long ndof, const T* b, T* x, int nrhs,
                    const CgScalars* cs, hipStream_t st);

// Zero the fixed DOFs of x (nrhs vectors): xm = Z x.
void mask_copy(const double* x, double* xm, const uint8_t* mask, long nn, int nrhs, hipStream_t st);
// Identity rows: y_i = x_i on fixed DOFs.
void identity_rows(const double* x, double* y, const uint8_t* mask, long nn, int nrhs,
                   hipStream_t st);

// Type conversions and fills.
template <typename TA, typename TB>
void convert(const TA* a, TB* b, long n, hipStream_t st);
template <typename T>
void fill(T* a, T v, long n, hipStream_t st);

// ---------------- set-up kernels ----------------
// E_i = Emin + rho_i^p (E0 - Emin); writes bad[0] = 1 on NaN or out-of-range.
void setup_simp(const double* rho, double* E, float* E32, long n, double E0, double Emin,
                double penal, int* bad, hipStream_t st);
// Effective element matrices Keff[e] = sum_s E[dens(e,s)] Ksub[s] (nd x nd),
// rows/columns of supported DOFs zeroed.
// Full symmetric 81x81 element matrices K[e] -> wrapped diagonals (OpEQ2).
template <typename T>
void setup_pack_q2(const double* K, T* D, long nel, hipStream_t st);
template <typename T>
void setup_pack_s2(const double* K, T* D, long nel, hipStream_t st);
// Full symmetric 192x192 element matrices K[e] -> wrapped diagonals of the
// 64-node element (serendipity = 0) or of the 32-node one's 96 DOFs.
template <typename T>
void setup_pack_e3(const double* K, T* D, long nel, int serendipity, hipStream_t st);
void setup_effective(int order, int nsub, int nelx, int nely, int nelz, const double* E,
                     const double* Ksub, const uint8_t* mask, Lat L, double* Keff, hipStream_t st);
// Galerkin coarse element matrices (24x24 Q1-type) of a coarse element grid.
//  src kind OP_MF_Q1: children are E_c * K0 (child mask applied here);
//  OP_ST27 (Q1-type elements with stored matrices Kc [nel_f][576], masks baked or applied);
//  OP_EQ2: each coarse element is one quadratic fine element (81x81 -> 24x24);
//  OP_EQ3: each coarse element is one cubic fine element (192x192 -> 24x24).
// elist (optional): ids of the coarse elements to compute (count n_elist);
// null computes all of them.
void setup_galerkin(int src_kind, Lat fine, const double* E, const double* K0, const double* Kc,
                    const uint8_t* mask_f, int ncx, int ncy, int ncz, double* KE,
                    const int* elist, int n_elist, hipStream_t st);
// First coarse level as a linear combination of precomputed matrices:
// KE[e] = sum_m E[dens(e, m)] G[m], m over the B^3 density cells of a coarse
// element (B = 2 nsub for trilinear children, nsub for one quadratic
// element of degree 2 or 3); valid where no child DOF is supported.
void setup_galerkin_lin(const double* E, const double* G, int B, int nsub, int nelx, int nely,
                        int ncx, int ncy, int ncz, double* KE, hipStream_t st);
// Assemble Q1-type element matrices into the half stencil, with the supports
// of mask baked in, plus the Jacobi data wD_i = min(omega, theta A_ii /
// sum_j |A_ij|) / A_ii (0 on fixed DOFs) and the plain diagonal.
template <typename T>
void setup_stencil(Lat L, const double* KE, const uint8_t* mask, T* coef, T* wD, double* diag64,
                   double omega, double theta, hipStream_t st);
// The same Jacobi data for the matrix-free / stored-Q2 fine operators.
template <typename T>
void setup_diag_mf(Lat L, const double* E, const double* K0, const uint8_t* mask, T* wD,
                   double* diag64, double omega, double theta, hipStream_t st);
template <typename T>
void setup_diag_eq2(Lat L, const double* Ke, const uint8_t* mask, T* wD, double* diag64,
                    double omega, double theta, hipStream_t st);
template <typename T>
void setup_diag_e3(Lat L, const double* Ke, const uint8_t* mask, T* wD, double* diag64,
                   double omega, double theta, hipStream_t st);
// Coarsest level: the dense operator over all of the level's DOFs (row
// stride ld, a multiple of GJ_B; identity rows/columns at fixed DOFs and in
// the padding) from its element matrices, and its inverse by blocked
// Gauss-Jordan elimination.  setup_coarse_inverse works on A and B in turn
// and returns the one holding the inverse; D: GJ_B^2 doubles, diag0: ld
// doubles of scratch.
constexpr int GJ_B = 32;
inline int coarse_ld(long ndof) { return (int)((ndof + GJ_B - 1) / GJ_B * GJ_B); }
void setup_dense(int src_kind, Lat L, const double* E, const double* K0, const double* KE,
                 const int* freedof, const int* dofpos, int nfree, int ld, double* A,
                 hipStream_t st);
double* setup_coarse_inverse(double* A, double* B, double* D, double* diag0, int ld, int* bad,
                             hipStream_t st);

// Compliance and sensitivity.
void comp_dot(const double* f, const double* u, long ndof, int nrhs, double* out, RedBuf red,
              hipStream_t st);
// dc/drho (Sec. 3.4); Kp: the packed form of Ksub (sens_pack:
// sens_packed_doubles(order) values) for 4^3 sub-elements, and for cubic
// elements with any nsub; else null.
long sens_packed_doubles(int order);
// Ksub [n^3][nd][nd] (n^3 <= 64) -> the packed sub-element matrices of the
// sensitivity contraction (zero columns past n^3) and their pair table.
void sens_pack(int order, int nsub, const double* Ksub, std::vector<double>& out);
void sens_kernel(int order, int nsub, int nelx, int nely, int nelz, Lat L, const double* rho,
                 const double* u, long ndof, int nrhs, const double* Ksub, const double* Kp,
                 double E0mEmin, double penal, double* dc, hipStream_t st);

// ---------------- fused small solves ----------------
// One workgroup runs a whole PCG solve of one load case: trilinear
// matrix-free finest level (nsub = 1) of at most FZ_MAX_NODES nodes (its
// node sums live in LDS), stencil levels below, a coarsest level of at most
// FZ_MAX_COARSE DOFs, FP64, Jacobi smoothing.  Vectors are the load case's
// slices of the problem's own buffers.
constexpr int FZ_MAXLEV = 8;
constexpr int FZ_MAX_NODES = 6000;
constexpr int FZ_MAX_COARSE = 1024;
// Stencil levels (node count padded to 64): their four pair sums per DOF
// share the finest level's LDS node sums.  Finest lattices within
// FZ_MAX_NODES that coarsen by 2 have at most 1,344 on their second level.
constexpr int FZ_MAX_ST_NODES = FZ_MAX_NODES / 4;
struct FzLevel {
  Lat L;
  const double* coef;  // stencil (levels >= 1)
  const double* wD;    // W D^-1, 0 on fixed DOFs
  const uint8_t* mask;
  double* b;
  double* x;
  double* r;
};
struct FzDesc {
  FzLevel lv[FZ_MAXLEV];
  int nlev, pre, post, maxit;
  int scale_warm;  // 1: start from x scaled by f.x / x.K x
  double tol2;  // rtol^2 (scaled by ||f||^2 on the device)
  const double* E;
  Q1HaarVals<double> hv;
  const double* Ainv;
  int ld;
  const double* f;
  double* x;
  double* r;
  double* p;
  CgScalars* cs;
};
// descs: n device descriptors, one workgroup each.
void fused_solve(const FzDesc* descs, int n, hipStream_t st);

// End-of-solve records of a batch: where one problem's CG scalars (nrhs load
// cases) and set-up flags (4 ints) live, and their packed copy.
struct FzGatherSrc {
  const CgScalars* cs;
  const int* bad;
  int nrhs, pad;
};
struct FzRecord {
  CgScalars cs[4];
  int bad[4];
};
static_assert(sizeof(CgScalars) % sizeof(int) == 0, "CG scalars copy as 32-bit words");
// src, out: n device entries; one workgroup per problem copies its record.
void fused_gather(const FzGatherSrc* src, int n, FzRecord* out, hipStream_t st);

// Timing-free plain copy (for traffic calibration).
void copy_bytes(const void* src, void* dst, size_t bytes, hipStream_t st);

}  // namespace mgcg
