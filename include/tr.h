/*
 * tr.h -- C ABI of the MI355X angular-multigrid DG transport library.
 *
 * Method: Lathouwers & Perko, "An Angular Multigrid Preconditioner for the
 * Radiation Transport Equation with Forward-Peaked Scatter" (arXiv
 * 2010.04559).  The library solves the steady mono-energetic linear
 * Boltzmann equation (eq. LBE) with a truncated-Legendre scatter kernel,
 * discretised by discontinuous Galerkin in space (nodal Q1 on a Cartesian
 * mesh) and in angle (the Lin basis on hierarchical octahedral patches,
 * Sections 2.1-2.3), with restarted GMRES preconditioned by the angular
 * multigrid V-cycle of Fig. lmg (Section 4) whose coarsest level is solved
 * by the block Gauss-Seidel sweep of Section 5.2 and whose levels may use a
 * lowered scatter order (Section 5.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Vectors ("canonical layout") are flat arrays with index
 *     a * S + j * ns + i
 * a = 3 * patch + m the angular dof (patches octant-major, octant id
 * [s_x<0] + 2[s_y<0] + 4[s_z<0], then depth-first in split order), j = ix +
 * nx (iy + ny iz) the cell, i = bx + 2 by (+ 4 bz) the spatial node,
 * ns = 2^dim, S = cells * ns.  Flux vectors hold the expansion coefficients
 * of eq. Expansion; right-hand sides and residuals are weak-form vectors
 * (one entry per test function, eq. complete).
 *
 * Pointers documented as "device" must be device memory of the current HIP
 * device (for instance torch tensors' data_ptr()); the caller owns them and
 * the library never frees or retains them; they must be 16-byte aligned
 * (vectors are accessed 16 bytes at a time; hipMalloc and torch
 * allocations are), else the call fails with TR_ERR_ARG.  Every call is ordered on the
 * given stream (tr_stream is a hipStream_t; 0 = the null stream).  Calls
 * that return scalars (solves) synchronise that stream.
 *
 * Every function returns TR_OK or an error code; no exception crosses the
 * ABI.  tr_last_error() returns a thread-local message for the last failure
 * on the calling thread.  A handle may be used by one thread at a time.
 */
#ifndef TR_H
#define TR_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tr_handle tr_handle;
typedef void *tr_stream;

enum {
  TR_OK = 0,
  TR_ERR_ARG = 1,          /* bad argument or inconsistent sizes            */
  TR_ERR_UNSUPPORTED = 2,  /* valid request the library does not provide   */
  TR_ERR_ALLOC = 3,        /* device or host allocation failed              */
  TR_ERR_HIP = 4,          /* a HIP runtime call failed                     */
  TR_ERR_NOCONV = 5        /* solver hit its iteration limit (x is written) */
};

/* buffer precision; TR_F32_SPLIT: FP32 buffers whose scatter product uses
 * split-BF16 operands (tr_scatter and the scatter timer only) */
enum { TR_F64 = 0, TR_F32 = 1, TR_F32_SPLIT = 2 };
enum { TR_PREC_F64 = 0, TR_PREC_MIXED = 1, TR_PREC_SG = 2, TR_PREC_MIXED_BF16 = 3 };
enum { TR_INFLOW_NONE = 0, TR_INFLOW_ISO = 1, TR_INFLOW_BEAM = 2 };
enum { TR_RESTRICT = 0, TR_PROLONG = 1 };
/* storage of the preconditioned vectors z_j = M^{-1} v_j in GMRES:
 * TR_Z_AUTO: FP32 preconditioners (non-linear) always keep them, in FP32
 *   (flexible GMRES, x += sum_j y_j z_j); the FP64 preconditioners (linear,
 *   so both forms give the same iterates in exact arithmetic) keep them in
 *   FP64 when they fit in half of the free device memory, else recompute
 *   x += M^{-1}(V y) with one extra preconditioner application per restart;
 * TR_Z_KEEP: always keep them (TR_ERR_ALLOC when they do not fit);
 * TR_Z_RECOMPUTE: never keep them (for an FP32 preconditioner this is the
 *   non-flexible update, kept as a comparison point). */
enum { TR_Z_AUTO = 0, TR_Z_KEEP = 1, TR_Z_RECOMPUTE = 2 };

/* Problem definition (eq. LBE, Sections 2.1, 4.1, 5.2, 5.3, 5.5).
 * All pointers are host memory, read during tr_setup only. */
typedef struct {
  int dim;                      /* 2 or 3                                         */
  int n[3];                     /* cells per axis (n[2] ignored when dim == 2)    */
  double len[3];                /* domain [0,len[0]] x [0,len[1]] (x [0,len[2]])  */
  int ang_base_level;           /* uniform octahedron refinements (Section 2.1)  */
  double cone_axis[3];          /* local refinement around this direction ...    */
  double cone_half_angle_deg;   /* ... for vertices strictly inside this cone     */
  int cone_extra_levels;        /* extra levels inside the cone (0 = none)        */
  int irregularity_closure;     /* 1: refine until neighbours differ <= 2 levels  */
  int band_lmax;                /* > 0: the z-band rule of Section 5.5 instead of */
                                /* uniform refinement (levels lmax .. lmax-4 by   */
                                /* the largest vertex Omega_z: 0.97/0.9/0.8/0.6)  */
  const double *sigma_t;        /* [cells] total cross section (> 0)              */
  const double *sigma_s;        /* [cells] scatter cross section sigma_{s,0}      */
  int order;                    /* Legendre order L of the problem operator       */
  const double *moments;        /* [max order + 1] f_n, sigma_{s,n} = sigma_s f_n */
  int n_levels;                 /* number of angular levels T_0..T_Lmax           */
  const int *mg_order;          /* [n_levels] scatter order per level, coarsest 1st */
  int nu_pre, nu_post;          /* V(nu_pre, nu_post) smoothing (Fig. lmg), >= 1, >= 0 */
  int nu_coarse;                /* Gauss-Seidel sweeps on T_0 (Section 5.2)      */
  int octant_order[8];          /* Gauss-Seidel octant order (a permutation)     */
  int angular_basis;            /* TR_BASIS_LIN or TR_BASIS_CONST (Section 2.2)  */
  int nu_post_coarse;           /* post-smoothing sweeps on the levels below the  */
                                /* finest (>= 0; 0: nu_post on every level)       */
} tr_problem;

/* Angular basis (Section 2.2).  LIN: the three nodal functions of a patch.
 * CONST: one constant per patch, carried by the Lin data layout and kernels
 * as three coincident ordinates (the patch's mean direction int_q Omega /
 * |q|, a third of its area each) that hold equal values: a Const function
 * c_q is the vector with all three coefficients of patch q equal to c_q,
 * and a Const weak-form vector (right-hand side, residual, detector
 * weights) has a third of the Const entry in each of the three.  Every
 * operator maps such vectors to such vectors, and restricted to them is
 * exactly the Const discretisation (transport terms and X integrals
 * integrated to round-off, daughters taking their parent's value).  The
 * layout triples the work of a one-dof-per-patch path. */
enum { TR_BASIS_LIN = 0, TR_BASIS_CONST = 1 };

/* how a level's scatter product G_l u is formed (multiply-adds per spatial
 * dof): DENSE 2 A^2; FACTORED through the K = (order+1)^2 harmonics, 4 A K;
 * OCTANT through the Walsh-Hadamard blocks of the octant reflection group
 * of R axes (meshes mapped onto themselves by those reflections), 2 A^2/2^R */
enum { TR_SCATTER_DENSE = 0, TR_SCATTER_FACTORED = 1, TR_SCATTER_OCTANT = 2 };

typedef struct {
  int dim, cells, spatial_dofs, n_levels;
  int patches[16];              /* patches on each level T_l                       */
  int order_outer;
  size_t device_bytes;          /* device memory held by the handle                */
  int scatter_form[16];         /* TR_SCATTER_* of each level's scatter (level 0:  */
                                /* dense, used by the Gauss-Seidel solve)          */
  int scatter_axes[16];         /* R of the OCTANT form, else 0                    */
  int scatter_k[16];            /* K of the FACTORED form, else 0                  */
  int outer_axes;               /* R of the problem operator's scatter, 0 = dense  */
  int sweep_lds[2];             /* 1: the FP64 / FP32 forward sweeps keep the      */
                                /* previous diagonal plane in LDS (planes fit)     */
  int sweep_pair[2];            /* 1: the FP64 / FP32 forward sweeps run over      */
                                /* bricks of two x-adjacent cells (3-D grids with  */
                                /* an even cell count along x, planes fit in LDS)  */
} tr_info_t;

typedef struct {
  int kind;                     /* TR_INFLOW_ISO or TR_INFLOW_BEAM                 */
  int axis, side;               /* boundary face: axis 0..dim-1, side 0 low / 1 high */
  int lo[3], hi[3];             /* cell-index box on the face (face axis ignored)  */
  double value;                 /* ISO: angular flux; BEAM: current per area       */
  double direction[3];          /* BEAM: unit direction (entering the domain)      */
} tr_inflow;

typedef struct {
  double tol;                   /* stop when ||b - A x|| / ||b|| < tol             */
  int restart;                  /* GMRES(m)                                        */
  int max_restarts;
  int prec_mode;                /* TR_PREC_F64, _MIXED, _SG or _MIXED_BF16         */
  int timing;                   /* 1: time components with HIP events              */
  int z_store;                  /* TR_Z_AUTO, TR_Z_KEEP or TR_Z_RECOMPUTE          */
} tr_solve_opts;

typedef struct {
  int iters, restarts, converged;
  double rel_res;               /* final explicit relative residual               */
  double ms_total, ms_sweep, ms_scatter, ms_transfer, ms_coarse, ms_apply, ms_orth, ms_other;
  int n_sweep, n_scatter, n_coarse; /* launches timed in each component           */
  double ms_sweep_finest;       /* time in finest-level transport sweeps          */
  int n_sweep_finest;
  int n_precond;                /* preconditioner applications                    */
  double sweep_dof_updates;     /* sum over transport sweeps of (ordinates x spatial dofs) */
  int coarse_steps;             /* dependent steps of one coarse Gauss-Seidel solve */
  int flexible;                 /* preconditioned vectors kept: 64 / 32 (bits), 0 recomputed */
  double ms_scatter_outer;      /* time in the problem operator's scatter products */
  int n_scatter_outer;          /* (included in ms_scatter / n_scatter)            */
  double ms_scatter_finest;     /* time in the finest multigrid level's scatter    */
  int n_scatter_finest;         /* products (included in ms_scatter / n_scatter)   */
} tr_solve_stats;

/* Build the angular mesh, quadrature, level operators, prolongations and
 * sweep schedules for a problem (Sections 2.1-2.3, 4.1, 5.2) and allocate
 * the solver workspace on the current device.  *out receives the handle.
 * Errors: TR_ERR_ARG (bad sizes, sigma_t <= 0 or not finite, n_levels not
 * equal to the mesh's level count, orders out of range), TR_ERR_ALLOC. */
int tr_setup(const tr_problem *prob, tr_handle **out);
/* Device memory (bytes) a handle for prob holds after tr_setup, plus, when
 * opts is not NULL, what a solve with those options adds (FP32 level
 * buffers, the GMRES(opts->restart) workspace with the preconditioned
 * vectors counted as kept, split-BF16 level matrices, the coarse solve's
 * schedule and counters); the adjoint solve adds one more vector when its
 * lambda argument is NULL.  Runs the host part of the setup only: no device
 * is needed and nothing is allocated.  Errors: as tr_setup; TR_ERR_ARG for
 * bad options. */
int tr_workspace_bytes(const tr_problem *prob, const tr_solve_opts *opts, size_t *bytes);
/* Release a handle and its device memory (NULL is ignored). */
void tr_destroy(tr_handle *h);
/* Thread-local text of the last error on this thread. */
const char *tr_last_error(void);
/* Sizes of a handle's discretisation. */
int tr_info(const tr_handle *h, tr_info_t *out);

/* Replace the per-cell cross sections (device pointers, [cells] FP64).
 * Nothing else of the setup depends on them.  They are checked as in
 * tr_setup (TR_ERR_ARG, the handle's values unchanged); synchronises st. */
int tr_set_sigma(tr_handle *h, const double *sigma_t, const double *sigma_s, tr_stream st);

/* Weak-form right-hand side b (device, FP64, canonical, finest level): the
 * isotropic volume source q_cell (device [cells] per steradian, or NULL)
 * plus the boundary term of eq. complete for the inflow data (NULL = none;
 * a BEAM is a Dirac in angle shared equally by the patches whose closure
 * holds the direction, Section 5.5).  b is overwritten. */
int tr_rhs(tr_handle *h, const double *q_cell, const tr_inflow *inflow, double *b, tr_stream st);

/* Detector weights w (device, FP64, canonical): R = w . phi is the scalar
 * flux integrated over the cell box lo..hi. */
int tr_detector(tr_handle *h, const int lo[3], const int hi[3], double *w, tr_stream st);

/* Detector response R = w . phi (host *R), the integrated quantity whose
 * gradient tr_adjoint_grad returns; w, phi device FP64 canonical finest
 * level.  Synchronises st. */
int tr_response(tr_handle *h, const double *w, const double *phi, double *R, tr_stream st);

/* Transport sweep phi = L_l^{-1} g on angular level l (Section 3; exact on
 * the Cartesian mesh since every patch is inflow or outflow per face).
 * g, phi: device, canonical layout of level l, precision prec. */
int tr_sweep(tr_handle *h, int level, int prec, const void *g, void *phi, tr_stream st);
/* Adjoint sweep lambda = L_l^{-T} g (transposed blocks, downwind first). */
int tr_sweep_adjoint(tr_handle *h, int level, int prec, const void *g, void *lam, tr_stream st);

/* Scatter source s = S phi = sigma_s N (x) S~ phi on level l (Section 5.2,
 * discrete source Q with the X integrals of eq. X).  outer = 1 selects the
 * problem operator (finest level, order L); outer = 0 the multigrid level
 * operator (order mg_order[l]).  Device buffers of precision prec
 * (TR_F32_SPLIT: FP32 buffers, the product S~ phi formed from split-BF16
 * operands, x = bf16(x) + bf16(x - bf16(x)), as three BF16 matrix-core
 * products with FP32 accumulation; relative error about 2^-16 per term). */
int tr_scatter(tr_handle *h, int level, int outer, int prec, const void *phi, void *s, tr_stream st);

/* y = A x = (L - S) x, the problem operator on the finest level (FP64). */
int tr_apply(tr_handle *h, const double *x, double *y, tr_stream st);

/* Inter-level transfer between T_{l-1} and T_l (Section 4.1): PROLONG
 * writes out = P in (in: level l-1, out: level l); RESTRICT writes
 * out = P^T in (in: level l, out: level l-1).  Device buffers, precision prec. */
int tr_transfer(tr_handle *h, int level, int dir, int prec, const void *in, void *out, tr_stream st);

/* nu Gauss-Seidel sweeps on T_0 from zero (Section 5.2), FP64, canonical
 * level-0 layout; adjoint = 1 uses A_0^T with each octant visited downwind
 * first. */
int tr_coarse_gs(tr_handle *h, int nu, int adjoint, const double *f, double *phi, tr_stream st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): tr_coarse_gs
 * without any allocation.  Its update counters and error word live in a
 * library-owned static device array of 4 MiB + 256 B per device (up to
 * 2^20 counters: one per 2 x 2 x 2 brick of an even 3-D grid, else one per
 * cell), which every call on that device shares: calls that overlap on one
 * device race.  Only the dataflow forms (nu <= 15) run here; the schedule
 * for nu must exist (nu_coarse of the problem is prepared by tr_setup,
 * other counts by one earlier tr_coarse_gs call).  Errors: TR_ERR_ARG (no
 * schedule, too many counters), TR_ERR_UNSUPPORTED (nu > 15), TR_ERR_HIP
 * (a wait timed out).  Synchronises st. */
int tr_coarse_gs_noalloc(tr_handle *h, int nu, int adjoint, const double *f, double *phi, tr_stream st);

/* Preconditioner z = M^{-1} r: the V-cycle of Fig. lmg (TR_PREC_F64: all
 * levels FP64; TR_PREC_MIXED: levels >= 1 in FP32, T_0 in FP64;
 * TR_PREC_MIXED_BF16: as TR_PREC_MIXED with the FP32 scatter products
 * formed from split-BF16 operands, see tr_scatter), or one transport sweep
 * (TR_PREC_SG).  adjoint = 1 builds the cycle from the
 * transposed level operators.  r, z: device FP64 canonical finest level. */
int tr_mg_vcycle(tr_handle *h, int prec_mode, int adjoint, const double *r, double *z, tr_stream st);

/* Solve A x = b with restarted right-preconditioned GMRES(m) from x = 0
 * (modified Gram-Schmidt, explicit residual test at each restart; FP64
 * throughout except the preconditioner per prec_mode).  Returns
 * TR_ERR_NOCONV (x and stats still written) at max_restarts. */
int tr_gmres_solve(tr_handle *h, const double *b, double *x, const tr_solve_opts *opts,
                   tr_solve_stats *stats, tr_stream st);

/* Solve A x = b with right-preconditioned BiCGStab from x = 0, the Krylov
 * method of the paper (Section 3): per iteration two preconditioner and two
 * operator applications; the recurrence residual is confirmed by the
 * explicit residual ||b - A x|| / ||b|| < tol (a failed confirmation
 * restarts the recurrences from it).  Iteration limit restart x
 * (max_restarts + 1); opts->z_store is ignored.  FP64 throughout except the
 * preconditioner per prec_mode (an FP32 preconditioner makes the method
 * inexact; it receives unit-norm inputs).  stats->iters counts BiCGStab
 * iterations.  TR_ERR_NOCONV at the limit (x and stats still written). */
int tr_bicgstab_solve(tr_handle *h, const double *b, double *x, const tr_solve_opts *opts, tr_solve_stats *stats,
                      tr_stream st);

/* Detector-response gradient by the adjoint method: solves A^T lambda = w
 * with GMRES and the adjoint V-cycle, then per cell j
 *   grad_t[j] = -sum_q lambda_jq^T (N (x) M_q) phi_jq,
 *   grad_s[j] = +lambda_j^T (N (x) S~) phi_j.
 * phi: forward solution (device FP64).  lambda (device, may be NULL)
 * receives the adjoint solution.  grad_t, grad_s: device [cells] FP64. */
int tr_adjoint_grad(tr_handle *h, const double *w, const double *phi, double *lambda,
                    double *grad_t, double *grad_s, const tr_solve_opts *opts,
                    tr_solve_stats *stats, tr_stream st);

/* Average duration (ms) of the finest-level FP64/FP32 transport-sweep
 * kernel over `reps` back-to-back launches on the stream, timed with HIP
 * events on that stream (a measurement helper; g and phi as in tr_sweep,
 * but in the library's internal ordinate layout, see tr_sweep). */
int tr_time_sweep_kernel(tr_handle *h, int level, int prec, int reps, double *ms_per_launch, tr_stream st);
/* Same for the scatter GEMM of level l (outer as in tr_scatter). */
int tr_time_scatter_kernel(tr_handle *h, int level, int outer, int prec, int reps,
                           double *ms_per_launch, tr_stream st);

#ifdef __cplusplus
}
#endif
#endif /* TR_H */
