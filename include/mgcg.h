/*
 * mgcg.h — C ABI of the MI355X (gfx950) multigrid-preconditioned conjugate
 * gradient solver for the SIMP linear-elasticity equilibrium K(rho) u = f on
 * structured hexahedral meshes, with compliance and density gradients.
 *
 * The operation (Vitorino & Gomes, "An efficient topology optimization
 * algorithm for large-scale three-dimensional structures"):
 *   - element stiffness with the modified SIMP law, Sec. 2 eq. (1):
 *       K^(e) = (Emin + rho_e^p (E0 - Emin)) * integral of B^T D B;
 *   - multiresolution elements holding n^3 density sub-elements, Sec. 3.3
 *     eq. (7): K^(e) = sum_i (Emin + rho_{e_i}^p (E0 - Emin)) K^(e_i);
 *   - global K by superposition, supported DOFs removed (Sec. 2, 3.3, 6.1);
 *   - the solve by CG preconditioned with geometric multigrid (Sec. 2.3,
 *     Algorithm 1 applied recursively as a V-cycle; coarse element = 2x2x2
 *     fine elements, trilinear prolongation P, restriction R = P^T,
 *     weighted-Jacobi smoothing, Galerkin coarse operators, an exact dense
 *     FP64 solve on the coarsest mesh (the paper factors it by Cholesky;
 *     here its explicit inverse by blocked Gauss-Jordan elimination, applied
 *     as one matvec per cycle); stop on the relative residual, Sec. 7.2.1;
 *     warm start from the previous solution, Sec. 7.2.1);
 *   - compliance c = f^T u (problem (2)) and its gradient with respect to the
 *     densities, Sec. 3.4: dc/drho_i = -p rho_i^{p-1} (E0 - Emin)
 *     u_e^T K^(e_i) u_e (summed over load cases).
 *
 * Conventions
 *   Node lattice of an order-p mesh with nelx x nely x nelz elements:
 *   NX = p*nelx + 1 (same for y, z); node = i + NX*(j + NY*k), x fastest;
 *   DOF = 3*node + c (c = x, y, z).  Vectors of several load cases are
 *   stored one after another: [nrhs][ndof].  Densities: the C-order array
 *   (n*nelz, n*nely, n*nelx), i.e. index ix + (n*nelx)*(iy + (n*nely)*iz).
 *   Elements are unit cubes.
 *
 * Ownership
 *   The caller owns every buffer it passes.  Input buffers are read before the
 *   call returns (device inputs: read in stream order on the problem's
 *   stream); output buffers are written before the call returns (device
 *   outputs: written in stream order, complete once the stream is
 *   synchronised — every call below that returns results on the host
 *   synchronises the stream itself).  The library owns all hierarchy memory
 *   and frees it in mgcg_problem_destroy.  One problem is used by one host
 *   thread at a time.
 *
 * Errors
 *   Every int-returning call returns MGCG_OK (0), MGCG_ENOTCONV (1: result
 *   written but the tolerance was not reached) or a negative code; the
 *   thread-local message of the last failure is returned by mgcg_last_error.
 *   No C++ exception crosses this interface.
 */
#ifndef MGCG_H
#define MGCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGCG_OK 0
#define MGCG_ENOTCONV 1      /* max iterations reached; info and u written */
#define MGCG_EINVAL (-1)     /* invalid argument or density (NaN, outside [0,1]) */
#define MGCG_ENOMEM (-2)     /* device allocation failed */
#define MGCG_EBUDGET (-3)    /* request larger than the server's HBM budget */
#define MGCG_EBREAKDOWN (-4) /* CG breakdown: p^T A p <= 0 or non-finite */
#define MGCG_EDEVICE (-5)    /* HIP runtime error */
#define MGCG_EAGAIN (-6)     /* server: the request has not finished yet */
#define MGCG_ESTATE (-7)     /* call out of order (e.g. solve before densities) */

#define MGCG_FP64 0  /* FP64 everywhere */
#define MGCG_MIXED 1 /* FP32 V-cycle inside an FP64 CG (FP64 coarsest inverse) */

/* Element families (Sec. 2.1).  MGCG_SERENDIPITY needs order 2 or 3: the
 * 20-node quadratic serendipity element (vertices and edge midpoints) or the
 * 32-node cubic one (vertices and the two third-points of every edge).  It
 * runs on the Lagrange lattice of its order; the DOFs of face-interior and
 * body-interior nodes, which no serendipity element uses, are fixed by the
 * library (their loads ignored, their displacements 0). */
#define MGCG_LAGRANGE 0
#define MGCG_SERENDIPITY 1
/* Finest-level smoother (Sec. 7.5 prefers SSOR for quadratic and cubic
 * elements): MGCG_SMOOTH_GAUSS_SEIDEL is a symmetric Gauss-Seidel sweep in
 * multicolour order on the node lattice of order p = 2 or 3 (nodes coloured
 * by their lattice indices mod p + 1, so that nodes of one colour share no
 * element; colours 0 .. (p+1)^3 - 1 and, within a node, components x, y, z),
 * relaxation 1: pre forward sweeps before and post backward sweeps after the
 * coarse correction, so the V-cycle stays symmetric.  Coarser levels keep
 * the Jacobi sweep (omega).  It stores each element's matrix once more, by
 * node, in the V-cycle precision (81^2 or 192^2 values per element). */
#define MGCG_SMOOTH_JACOBI 0
#define MGCG_SMOOTH_GAUSS_SEIDEL 1

#define MGCG_MEM_HOST 0
#define MGCG_MEM_DEVICE 1

typedef struct mgcg_problem mgcg_problem;
typedef struct mgcg_ctx mgcg_ctx;
typedef struct mgcg_server mgcg_server;

/* Problem description.  Elements are unit cubes. */
typedef struct mgcg_desc {
  int32_t nelx, nely, nelz; /* displacement elements per axis (>= 1) */
  int32_t order;            /* 1: 8-node trilinear, 2: 27-node triquadratic,
                               3: 64-node tricubic (orders 2 and 3 coarsen first
                               onto the vertex lattice of the same elements) */
  int32_t nsub;             /* density sub-elements per axis per element (n_mr >= 1) */
  int32_t nlevels;          /* multigrid levels including the finest (>= 1); every
                               coarsening needs even element counts on every axis */
  int32_t nrhs;             /* load cases, 1..4, solved as independent CG recurrences
                               sharing every operator read */
  int32_t precision;        /* MGCG_FP64 or MGCG_MIXED */
  int32_t pre, post;        /* weighted-Jacobi sweeps before / after the coarse correction */
  double E0, Emin, nu, penal; /* solid modulus, void modulus, Poisson ratio, SIMP p */
  double omega;             /* Jacobi weight */
  int32_t family;           /* MGCG_LAGRANGE or MGCG_SERENDIPITY (order 2 or 3) */
  int32_t smoother;         /* finest-level smoother: MGCG_SMOOTH_JACOBI (0, the
                               capped weighted Jacobi of every level) or, for
                               order 2 or 3 with nlevels >= 2,
                               MGCG_SMOOTH_GAUSS_SEIDEL */
} mgcg_desc;

/* Result of one solve. */
typedef struct mgcg_info {
  int32_t status;        /* return code of the solve */
  int32_t iters[4];      /* PCG iterations per load case */
  double rel_res[4];     /* true ||f - K u|| / ||f|| per load case at exit (FP64) */
  int32_t replacements;  /* residual replacements performed */
  int32_t pad;
  double t_setup_ms;     /* last mgcg_set_densities, device time */
  double t_solve_ms;     /* this solve, host wall time */
} mgcg_info;

/* Thread-local message of the last failing call ("" if none). */
const char* mgcg_last_error(void);
int mgcg_version(void);

/* Device bytes a problem allocates when it is first used (exactly what
 * mgcg_problem_create + first use allocates).  0 on invalid desc. */
size_t mgcg_problem_device_bytes(const mgcg_desc* desc);

/* A context: a device and an HBM budget shared by the problems created in it
 * (mgcg_problem_create_in).  A problem's device memory (exactly
 * mgcg_problem_device_bytes of its desc) is charged when it is allocated (at
 * its first mgcg_set_densities / solve / allocate, or by a server's
 * admission) and refunded when it is destroyed; an allocation the budget
 * cannot hold fails with MGCG_EBUDGET and allocates nothing.  hbm_budget_bytes
 * = 0: no limit.  The context owns nothing but the accounting; destroying it
 * while any of its problems lives is MGCG_EINVAL.  Thread-safe. */
int mgcg_ctx_create(mgcg_ctx** out, int device, size_t hbm_budget_bytes);
int mgcg_ctx_destroy(mgcg_ctx* ctx);
/* Bytes charged now, the budget, and the number of live problems (any
 * output may be null). */
int mgcg_ctx_usage(mgcg_ctx* ctx, size_t* in_use, size_t* budget, int32_t* problems);
/* mgcg_problem_create on the context's device, charged to its budget. */
int mgcg_problem_create_in(mgcg_ctx* ctx, const mgcg_desc* desc, const uint8_t* fixed_mask,
                           const double* f, mgcg_problem** out);

/* Validate desc and copy the supports and loads (host arrays):
 *   fixed_mask  uint8[ndof]       nonzero = DOF fixed (Sec. 6.1);
 *   f           double[nrhs*ndof] nodal loads (entries on fixed DOFs ignored).
 * Device memory is allocated lazily on `device` at the first
 * set_densities/solve (or by the server at admission). */
int mgcg_problem_create(const mgcg_desc* desc, const uint8_t* fixed_mask, const double* f,
                        int device, mgcg_problem** out);
int mgcg_problem_destroy(mgcg_problem* p);

/* Run all later work of this problem on `stream` (a hipStream_t, e.g. the
 * current torch stream; NULL = the library's own stream). */
int mgcg_set_stream(mgcg_problem* p, void* stream);
/* The hipStream_t the problem's work runs on (*stream): the one set above,
 * else the library's own stream of this problem (created by this call if
 * needed; no device memory is allocated).  Device inputs are read in order
 * on this stream, so a caller producing them on another stream makes this
 * one wait for it (an event) before passing them. */
int mgcg_get_stream(mgcg_problem* p, void** stream);

/* How the PCG iterations are launched: MGCG_LAUNCH_EAGER (the default)
 * launches the kernels one by one; MGCG_LAUNCH_GRAPH replays one captured
 * iteration, a HIP graph of its kernel launches (no memset or copy nodes),
 * built at the first chunk after allocation.  Same kernels, same arguments,
 * same results (on one MI355X the replay was not faster: the host keeps
 * ahead of the GPU either way).  MGCG_LAUNCH_FUSED runs each mgcg_solve as
 * one launch in which a single workgroup per load case does the whole PCG
 * solve (Sec. 2.3, V-cycle of Algorithm 1 included) between workgroup
 * barriers: for small problems, whose kernels cost their launch and ramp
 * more than their work.  It needs trilinear elements with nsub = 1, FP64,
 * the Jacobi smoother, 2..8 levels, at most 6000 finest-level nodes and at
 * most 1024 coarsest DOFs (MGCG_EINVAL otherwise); the same iteration in
 * another summation order, so results agree with the other modes to
 * rounding.  The serving loop (mgcg_server_*) always launches eagerly, and
 * so does a solve while kernel timing is on.  MGCG_EINVAL for another mode. */
#define MGCG_LAUNCH_EAGER 0
#define MGCG_LAUNCH_GRAPH 1
#define MGCG_LAUNCH_FUSED 2
int mgcg_set_launch_mode(mgcg_problem* p, int mode);

/* Allocate the device hierarchy now (otherwise done on first use). */
int mgcg_problem_allocate(mgcg_problem* p);

/* Densities rho[n_rho] (FP64, host or device): SIMP moduli, fine operator,
 * Galerkin coarse operators, Jacobi diagonals and the coarsest level's
 * explicit FP64 inverse (the multigrid refresh of Sec. 7.2).  MGCG_EINVAL if any density is
 * NaN or outside [0, 1] (detected on the device; the previous operator is
 * then invalid and must be refreshed before the next solve). */
int mgcg_set_densities(mgcg_problem* p, const double* rho, int mem);

/* The same from FP32 densities (host or device, [n_rho]), converted to FP64
 * on their way in (Sec. 2 eq. (1) is then evaluated in FP64 as above).
 * MGCG_EINVAL for null arguments; otherwise as mgcg_set_densities. */
int mgcg_set_densities_f32(mgcg_problem* p, const float* rho, int mem);

/* Solve K u = f for every load case to ||f - K u|| <= rtol ||f|| (true FP64
 * residual), at most maxit PCG iterations.  Initial guess (warm_start):
 *   MGCG_COLD (0)         zero;
 *   MGCG_WARM_SCALED (1)  the current u (the previous solution, Sec. 7.2, or
 *                         mgcg_set_initial_guess) times the factor
 *                         alpha = f^T u / u^T K u that minimises the energy
 *                         1/2 x^T K x - f^T x along u, per load case (alpha
 *                         = 0 when u^T K u <= 0): never worse in energy than
 *                         either zero or u itself, and alpha = 1 when u
 *                         already solves the system;
 *   MGCG_WARM_PLAIN (2)   the current u as it is.
 * info may be NULL.  Blocks until done. */
#define MGCG_COLD 0
#define MGCG_WARM_SCALED 1
#define MGCG_WARM_PLAIN 2
int mgcg_solve(mgcg_problem* p, double rtol, int maxit, int warm_start, mgcg_info* info);

/* Several small problems solved in one launch (batched multi-problem
 * solve): every problem must fit MGCG_LAUNCH_FUSED (see above; its launch
 * mode need not be set) and have its densities set, and all must live on
 * one device; a workgroup per load case of every problem runs its whole
 * PCG solve, so up to one problem per compute unit progresses at once.
 * The launch goes on ps[0]'s stream after the work already enqueued on
 * every problem's stream; the call returns when all are done, their
 * results read back in one transfer.  infos (may be NULL) receives n results, in
 * the order of ps.  Returns MGCG_OK, or the first problem's error status
 * (MGCG_ENOTCONV, MGCG_EBREAKDOWN, ...) in ps order; MGCG_EINVAL for a
 * problem that does not fit, a problem listed twice, n < 1 or mixed
 * devices. */
int mgcg_solve_batch(mgcg_problem* const* ps, int n, double rtol, int maxit, int warm_start,
                     mgcg_info* infos);

/* u[nrhs*ndof] FP64 (zero on fixed DOFs). */
int mgcg_get_displacement(mgcg_problem* p, double* u, int mem);
int mgcg_set_initial_guess(mgcg_problem* p, const double* u, int mem);

/* Compliance and gradient of the current solution:
 *   c   host double[nrhs+1]: f_l^T u_l per load case, then their sum;
 *   dc  double[n_rho] (host or device, may be NULL): d(sum_l c_l)/d rho. */
int mgcg_compliance_sensitivity(mgcg_problem* p, double* c, double* dc, int mem);

/* ---- Inspection of the operators (for parity tests) ----
 * level 0 is the finest.  prec: MGCG_FP64 = the FP64 operator, MGCG_MIXED =
 * the V-cycle's FP32 copy (levels >= 1 exist only in the V-cycle precision).
 * Vectors are FP64 [nrhs][ndof_level] in the given memory. */
int mgcg_level_dims(mgcg_problem* p, int level, int32_t* dims3, int64_t* ndof);
/* y = A_l x with A_l = Z K_l Z + (I - Z) (identity rows on fixed DOFs). */
int mgcg_apply(mgcg_problem* p, int level, int prec, const double* x, double* y, int mem);
/* diag(A_l)[ndof_level] */
int mgcg_level_diag(mgcg_problem* p, int level, double* d, int mem);
/* coarse = P~^T fine, fine = P~ coarse (P~ = trilinear prolongation with rows
 * of fixed fine DOFs and columns of fixed coarse DOFs zeroed); level is the
 * fine side (0 .. nlevels-2). */
int mgcg_restrict(mgcg_problem* p, int level, const double* fine, double* coarse, int mem);
int mgcg_prolong(mgcg_problem* p, int level, const double* coarse, double* fine, int mem);
/* z = M r: one V-cycle in the problem's precision. */
int mgcg_precondition(mgcg_problem* p, const double* r, double* z, int mem);
/* x = A_c^{-1} b on the coarsest level (a matvec with its explicit inverse). */
int mgcg_coarse_solve(mgcg_problem* p, const double* b, double* x, int mem);

/* ---- Kernel timing (HIP events around each launch of one kernel) ----
 * kernel ids: 0 = finest-level operator apply (all variants). */
int mgcg_set_kernel_timing(mgcg_problem* p, int enable);
int mgcg_get_kernel_timing(mgcg_problem* p, int kernel, double* total_ms, int64_t* launches);
/* Plain device copy of `bytes` bytes on the problem's stream (calibration of
 * memory-traffic counters). */
int mgcg_copy_bytes(mgcg_problem* p, const void* src, void* dst, size_t bytes);

/* ---- Serving: continuous batching of solves over one GPU ----
 * A server keeps up to max_slots problems resident (hierarchy + warm-start u
 * on the device) within hbm_budget bytes and advances every admitted solve
 * a few PCG iterations per step on its own stream, so solves of different
 * sizes overlap on the device.  Requests are admitted in submission order
 * when a slot is free and the problem's device bytes fit the remaining
 * budget; a problem submitted again while resident keeps its memory
 * (warm start).  The server does not own problems. */
int mgcg_server_create(int device, size_t hbm_budget, int max_slots, mgcg_server** out);
/* Requests still running are abandoned: the call waits only for the work
 * already enqueued on their problems' streams (no further iterations), and
 * those problems are left idle with the last iterate as u. */
int mgcg_server_destroy(mgcg_server* s);
/* Queue one solve of p with densities rho (FP64 [n_rho] in density-lattice
 * order), copied before the call returns: mem = MGCG_MEM_HOST copies into
 * host memory held by the request; MGCG_MEM_DEVICE copies device to device,
 * in order on p's stream (mgcg_get_stream), into a stream-ordered device
 * buffer of the request, which is freed in order on that stream when the
 * request ends.  MGCG_EBUDGET if p alone exceeds the budget; MGCG_EINVAL for
 * another device's problem or a bad mem. */
int mgcg_server_submit(mgcg_server* s, mgcg_problem* p, const double* rho, int mem, double rtol,
                       int maxit, int warm_start, uint64_t* ticket);
/* Admit what fits, launch the next chunk of every active solve, retire the
 * finished ones.  *active / *queued receive the counts after the step. */
int mgcg_server_step(mgcg_server* s, int* active, int* queued);
/* MGCG_EAGAIN until the ticket's solve has finished; then its info and the
 * wall time from submission to the step that saw it finish in *latency_ms
 * (queueing included). */
int mgcg_server_poll(mgcg_server* s, uint64_t ticket, mgcg_info* info, double* latency_ms);
/* Release a problem's device memory when it is not in use by a solve
 * (end of a session); MGCG_ESTATE while it is queued or running. */
int mgcg_server_release(mgcg_server* s, mgcg_problem* p);
/* Bytes currently held by resident problems. */
size_t mgcg_server_resident_bytes(mgcg_server* s);

/* Pure admission policy (no device): given the budget, the bytes in use, the
 * free slots and the queue's byte sizes in order, writes admit[i] = 1 for the
 * requests admitted now and returns how many.  In queue order while slots
 * are free: a 0-byte request (its problem already resident) is admitted;
 * requests needing memory are first-come-first-served among themselves (the
 * first that does not fit blocks the memory-needing ones behind it); an
 * entry of SIZE_MAX (cannot start now) is skipped. */
int mgcg_admission_plan(size_t budget, size_t in_use, int free_slots, const size_t* queue_bytes,
                        int nqueue, uint8_t* admit);

/* ---- Projection of design variables onto densities, and the density filter ----
 *
 * The operation (Sec. 3.2 eq. (5), with the weights of Sec. 2.2 eq. (4)):
 * design variables x live on a lattice of d x d x d cells per displacement
 * element, densities rho on n x n x n cells per element (the same unit
 * elements, so the density cells have edge 1/n and the design cells 1/d);
 *     rho_i = sum_j (omega_ij / omega_i) x_j,   omega_i = sum_j omega_ij,
 *     omega_ij = exp(-dist(i,j)^2 / (2 (rmin/3)^2)) / (2 pi rmin/3)
 * for dist(i,j) <= rmin (distance between the cells' centres, in element
 * edges), 0 otherwise; the sums run over the design cells of the domain.
 * With d = n the operation is the weighted-average density filter of Sec. 2.2.
 * The transpose gives the chain rule of Sec. 3.4: with g = d f / d rho,
 * (W^T g)_k = sum_i g_i omega_ik / omega_i = d f / d x_k; with g_i = the
 * density cells' volumes, W^T g is the volume constraint's gradient.
 * The test dist <= rmin is exact: along an axis the centres of density cell
 * i and design cell j lie m / (2 n d) apart with the integer
 * m = (2i + 1) d - (2j + 1) n, and a pair is inside when
 * m_x^2 + m_y^2 + m_z^2 <= (2 n d rmin)^2, the right side in FP64.
 *
 * Layout: x is the C-order array (d*nelz, d*nely, d*nelx), rho the array
 * (n*nelz, n*nely, n*nelx), both FP64, x fastest.  A projection object holds
 * 1/omega_i for every density cell on its device (mgcg_proj_device_bytes);
 * host-memory calls stage their vectors through temporary device buffers and
 * return when the result is on the host; device-memory calls are ordered on
 * the object's stream (the null stream unless set, i.e. torch's default
 * stream) and return at once.  Errors: MGCG_EINVAL for a
 * non-positive size, nsub or ndes outside 1..64, rmin not positive and
 * finite or so large that 2 n d rmin exceeds 4096, a lattice above 2^31 - 1
 * cells or 2^20 cells along an axis, or a radius that leaves some density cell without a design cell
 * inside its ball; MGCG_ENOMEM / MGCG_EDEVICE as elsewhere. */
typedef struct mgcg_proj mgcg_proj;
typedef struct mgcg_proj_desc {
  int32_t nelx, nely, nelz; /* displacement elements per axis */
  int32_t nsub;             /* n: density cells per element and axis */
  int32_t ndes;             /* d: design cells per element and axis */
  int32_t pad;
  double rmin;              /* ball radius, in element edges */
} mgcg_proj_desc;

/* Device bytes a projection object holds (0 on an invalid desc). */
size_t mgcg_proj_device_bytes(const mgcg_proj_desc* desc);
/* Validate desc, allocate on `device` and compute 1/omega_i (blocking). */
int mgcg_proj_create(const mgcg_proj_desc* desc, int device, mgcg_proj** out);
int mgcg_proj_destroy(mgcg_proj* pr);
/* Run later calls on `stream` (a hipStream_t; NULL = the null stream, the
 * default).  Waits for the work already queued on the previous stream. */
int mgcg_proj_set_stream(mgcg_proj* pr, void* stream);
/* rho[n_rho] = W x[n_x] (eq. (5)). */
int mgcg_proj_apply(mgcg_proj* pr, const double* x, double* rho, int mem);
/* gx[n_x] = W^T g[n_rho] (the chain rule of Sec. 3.4). */
int mgcg_proj_apply_transpose(mgcg_proj* pr, const double* g, double* gx, int mem);

/* ---- The SLP step (Sec. 4): LP subproblem and step control ----
 *
 * The LP subproblem (Sec. 4.1, problem (Pstar)) for the topology problem's
 * one linear constraint, the volume, whose gradient a is positive:
 *     min g^T s  s.t.  a^T s = b,  l <= s <= u,
 *     l_i = max(-delta, x_l - x_i),  u_i = min(delta, x_u - x_i)
 * (the volume constraint taken as an equality, the form of problem (P)).
 * With one constraint and a box it is a fractional knapsack: from s = l the
 * variables are raised in order of the ratio -g_i / a_i, highest first and
 * equal ratios in index order, each to u, until the budget B = b - a^T l is
 * used; the first variable (with u > l) whose running capacity a (u - l)
 * reaches B is raised partially and its ratio is the constraint's multiplier
 * lambda.  When B < 0 or B exceeds the total capacity the LP has no solution
 * and s is the artificial problem's (Pstar2, the box shrunk to 0.8 delta):
 * its lower end if B < 0, its upper end otherwise; info->feasible is then 0
 * and lambda NaN.
 *
 * An LP object holds device scratch for n variables (mgcg_lp_device_bytes);
 * g, a, x, s are FP64 [n] in host or device memory (mem); device-memory calls
 * run on the object's stream (the null stream unless set) and return when
 * the results are written (one read-back at the end; the feasibility test
 * picks the LP's solution or the artificial problem's on the device).  On
 * bad input the outputs are undefined and the error is returned.  Errors:
 * MGCG_EINVAL for n outside 1..2^31, delta not positive, non-finite b,
 * x_l > x_u, or any a_i <= 0 or non-finite input. */
typedef struct mgcg_lp mgcg_lp;
typedef struct mgcg_lp_info {
  double lambda;   /* multiplier of the constraint (the critical ratio) */
  double gts;      /* g^T s */
  double ats;      /* a^T s */
  double s_inf;    /* max_i |s_i| */
  double budget;   /* B = b - a^T l */
  int32_t feasible;
  int32_t pad;
} mgcg_lp_info;
size_t mgcg_lp_device_bytes(int64_t n);
int mgcg_lp_create(int64_t n, int device, mgcg_lp** out);
int mgcg_lp_destroy(mgcg_lp* lp);
int mgcg_lp_set_stream(mgcg_lp* lp, void* stream);
int mgcg_lp_solve(mgcg_lp* lp, const double* g, const double* a, const double* x, double b,
                  double delta, double x_l, double x_u, double* s, mgcg_lp_info* info, int mem);
/* The same LP with fixed variables (Sec. 6.1: the design variables of fixed
 * void and solid elements, e.g. design_fixed of mgcg_fix_variables): where
 * fixed[i] != 0, l_i = u_i = 0, so s_i = 0 and the variable adds no capacity
 * (also in the artificial problem).  fixed is uint8[n] in the same memory as
 * the vectors; MGCG_EINVAL for a NULL fixed. */
int mgcg_lp_solve_fixed(mgcg_lp* lp, const double* g, const double* a, const double* x,
                        const uint8_t* fixed, double b, double delta, double x_l, double x_u,
                        double* s, mgcg_lp_info* info, int mem);

/* Density thresholding of Sec. 5, on the scratch of an LP object of n values
 * (same mem, stream and synchronisation rules as mgcg_lp_solve; each call
 * returns when its results are written).
 *
 * mgcg_lp_select_top (the strategy based on the density values, Sec. 5.1):
 * out_i = 1 for the k largest v_i, equal values taken in increasing index
 * order, and 0 for the rest (k = floor(v_frac n) for a volume fraction
 * v_frac).  MGCG_EINVAL for k outside 0..n or a non-finite v_i.
 *
 * mgcg_threshold_round (Sec. 5, before either strategy): out_i = 1 where
 * rho_i >= hi, 0 where rho_i <= lo, rho_i otherwise (0.95 and 0.05 in the
 * paper).  out may equal rho.
 *
 * mgcg_angle_cos (the angle condition of Sec. 5.2): *cosine =
 * -gL^T d / (|gL| |d|), NaN when either vector is zero; the condition holds
 * when it exceeds cos(theta_max), theta_max = 89.9 degrees.
 *
 * mgcg_heaviside (Sec. 5.4): out_i = h(rho_i, beta, eta) =
 * (tanh(beta eta) + tanh(beta (rho_i - eta))) / (tanh(beta eta) +
 * tanh(beta (1 - eta))) with eta the zero of f(eta) = sum h - sum rho (cells of
 * equal volume), found by Newton's method from eta = 1/2 that keeps the
 * bracket of f's sign change and bisects when a step leaves it; stops at
 * |delta eta| <= 1e-14 or |f| <= 1e-13 sum rho, at most 100 iterations (each
 * one reduction pass and one read-back).  *eta and *iters (may be NULL) get
 * the threshold and the iteration count.  MGCG_EINVAL for beta not positive
 * and finite. */
/* mgcg_threshold_lagrangian (the strategy based on the gradient of the
 * Lagrangian, Sec. 5.2), on densities rho already rounded near 0 and 1 and
 * gL = grad L with respect to them: alpha_i is the step at which
 * rho_i - alpha gL_i reaches 0 (gL_i > 0) or 1 (gL_i < 0), infinite for
 * gL_i = 0.  *alpha gets alpha~, the largest alpha_i > 0 such that no density
 * with alpha_j <= alpha_i breaks a safeguard (reaching 1 needs rho_j >= v_u,
 * reaching 0 needs rho_j <= v_l; 0.3 and 0.7 in the paper) and the angle
 * condition holds for d = rho~ - rho at theta_max_deg (89.9); 0 when there is
 * none.  out_i = 0 or 1 (its bound) where alpha_i <= alpha~, else
 * rho_i - alpha~ gL_i, within [0, 1]; out = rho when alpha~ = 0.  The cosine
 * is nonincreasing in alpha; the admissible interval is searched over the
 * bits of alpha in 16 device passes.  MGCG_EINVAL for non-finite inputs. */
int mgcg_threshold_lagrangian(mgcg_lp* lp, const double* rho, const double* gL, double v_u,
                              double v_l, double theta_max_deg, double* out, double* alpha,
                              int mem);
int mgcg_lp_select_top(mgcg_lp* lp, const double* v, int64_t k, double* out, int mem);
int mgcg_threshold_round(mgcg_lp* lp, const double* rho, double lo, double hi, double* out,
                         int mem);
int mgcg_angle_cos(mgcg_lp* lp, const double* gL, const double* d, double* cosine, int mem);
int mgcg_heaviside(mgcg_lp* lp, const double* rho, double beta, double* out, double* eta,
                   int32_t* iters, int mem);

/* Step control of Algorithm 2 (host only).  After a trial step s of the LP:
 * f0 = f(x), f1 = f(x + s), c0 = c(x), c1 = c(x + s) (the constraint's value),
 * gts = g^T s, ats = a^T s, s_inf = |s|_inf.  Computes theta_k =
 * min(theta_large, theta_sup, theta_max) (eqs. (theta1), (theta2), with
 * P_fsb = M(x, 0) - M(x, s), M = (a^T s + c)^2 / 2, and P_opt = -g^T s, the
 * predicted reduction of f), the
 * actual and predicted reductions of psi = theta f + (1 - theta) |c|^2 / 2,
 * and rejects (A_red < 0.1 P_red: delta = min(0.25 s_inf, 0.1 delta),
 * theta_max = theta_k) or accepts (delta doubled up to box_inf when A_red >=
 * 0.5 P_red, then at least delta_min; theta_max = 1; k + 1; the history
 * minimum takes theta_k).  Returns 1 if accepted, 0 if rejected, MGCG_EINVAL
 * for a NULL ctrl.  Start from delta = delta_0, theta_max = theta_min_hist =
 * 1, k = 0. */
typedef struct mgcg_slp_ctrl {
  double delta, delta_min, box_inf; /* radius, its floor, |x_u - x_l|_inf */
  double theta_max, theta_min_hist; /* theta_max and min(theta_0 .. theta_{k-1}) */
  double N;                         /* the constant of eq. (theta1), 1e6 in the paper */
  int32_t k;                        /* outer iteration */
  int32_t pad;
} mgcg_slp_ctrl;
int mgcg_slp_decide(mgcg_slp_ctrl* ctrl, double f0, double f1, double c0, double c1, double gts,
                    double ats, double s_inf, double* theta, double* a_red, double* p_red);

/* ---- Variables fixed before the degree of the elements is raised (Sec. 6.1)
 *
 * An element is void when all its n^3 densities are <= rho_l and all its d^3
 * design-gradient components are >= -eps_grad, solid when all densities are
 * >= rho_u and all gradient components <= eps_grad (the paper: 1e-6, 0.9,
 * 1e-6).  It is fixed when every element sharing a node with it (inside the
 * domain) is of its kind.  Outputs:
 *   elem_kind     uint8[nelx*nely*nelz]  0 free, 1 fixed void, 2 fixed solid;
 *   design_fixed  uint8[d^3 * nel]       1 for the design variables of fixed
 *                                        elements (the design lattice, x fastest);
 *   dof_mask      uint8[3 * nn]          in/out: the DOFs of every node of the
 *                 lattice of degree `order` whose elements are all fixed void
 *                 are set to 1, the rest are left as passed (pass the supports;
 *                 the result is the fixed-DOF mask of the problem of that degree).
 * rho is the density lattice (n cells per element and axis), grad_x the
 * design gradient df/dx (d per element and axis), both FP64, x fastest.
 * mem selects host or device memory for all arrays; the call runs on the
 * null stream, allocates its own scratch and returns when done.  counts may
 * be NULL.  MGCG_EINVAL for a bad geometry (mesh >= 1, n and d in 1..64, order
 * 1..3), non-finite thresholds or NULL arrays. */
typedef struct mgcg_fix_desc {
  int32_t nelx, nely, nelz;
  int32_t nsub;   /* n: density cells per element and axis */
  int32_t ndes;   /* d: design cells per element and axis */
  int32_t order;  /* degree of the displacement lattice whose nodes are suppressed */
  double rho_l, rho_u, eps_grad;
} mgcg_fix_desc;
typedef struct mgcg_fix_counts {
  int64_t void_elems, solid_elems; /* fixed elements of each kind */
  int64_t fixed_design;            /* fixed design variables */
  int64_t suppressed_nodes;        /* nodes whose DOFs were set in dof_mask */
} mgcg_fix_counts;
int mgcg_fix_variables(const mgcg_fix_desc* desc, const double* rho, const double* grad_x,
                       uint8_t* elem_kind, uint8_t* design_fixed, uint8_t* dof_mask,
                       mgcg_fix_counts* counts, int mem);

/* The same choice for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): every
 * array, counts_dev included, is device memory of the current device, and
 * the call only enqueues kernels and one device-to-device copy on `stream`
 * (NULL: the null stream), without allocating, freeing or synchronising.
 * Outputs as for mgcg_fix_variables; counts_dev receives int64[4] = void
 * elements, solid elements, fixed design variables, suppressed nodes (in
 * stream order).  Its scratch (raw element kinds, block partials, counts) is
 * a static array of MGCG_FIX_SCRATCH_BYTES per GPU, held until the process
 * ends and shared by every call on that GPU: calls that overlap on one GPU
 * race (serialise them on one stream).  MGCG_EINVAL as for
 * mgcg_fix_variables, and when the mesh needs more scratch than the limit:
 * nel + 8 (2 ceil(nel/256) + ceil(d^3 nel/256) + ceil(nn/256)) bytes, each
 * part rounded up to 256, plus 256. */
#define MGCG_FIX_SCRATCH_BYTES (16 << 20)
int mgcg_fix_variables_noalloc(const mgcg_fix_desc* desc, const double* rho, const double* grad_x,
                               uint8_t* elem_kind, uint8_t* design_fixed, uint8_t* dof_mask,
                               int64_t* counts_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MGCG_H */
