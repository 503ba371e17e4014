/*
 * infoesrf.h -- C ABI of the InFo-ESRF update library for AMD Instinct MI355X (gfx950).
 *
 * The library implements the perturbation update of the Integral-Form Ensemble
 * Square-Root Filter (Armstrong & Grooms): the matrix square root of the
 * localized ensemble Kalman update is replaced by a quadrature sum over
 * shifted symmetric positive definite systems (Sec. 3.2, eq. 3.5), one per
 * (quadrature node q, ensemble member i), each solved by preconditioned
 * conjugate gradients (Appendix E, eq. E.1) against the localized forecast
 * covariance P = L o (Z Z^T) (Sec. 2.3, eq. 2.11), which is only ever applied
 * as an operator (eq. 2.12).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer in infoesrf_problem, infoesrf_stats, the workspace
 *    and the outputs is HIP *device* memory owned by the caller.  Host
 *    pointers are marked "host".  The library never allocates or frees device
 *    memory: all scratch lives in the caller's workspace, sized by
 *    infoesrf_workspace_bytes().
 *  - Matrices are column-major FP64 unless stated otherwise.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Work is ordered on that stream.  With opts->host_sync == 0 a
 *    call performs no host synchronization and no host read-back, so it can
 *    be captured in a HIP graph; status is then left in stats->counters.
 *  - Calls are reentrant given distinct workspaces.
 *  - Return codes: INFOESRF_OK (0), INFOESRF_WARN_NOT_CONVERGED (+1: outputs
 *    are written, per-system flags tell which systems missed the
 *    tolerance), or a negative error.  A message for the last error of the
 *    calling thread is available from infoesrf_last_error().
 *
 * Notation (paper -> ABI): ensemble size m -> N, observation dimension d -> m,
 * normalized perturbations Z (n x N) and W = H Z (m x N) (eq. 2.9), the
 * normalized observation covariance S = R^{-1/2} H P H^T R^{-1/2} (called C in
 * Theorem 3), shifted matrices C_q = (1 + s_q) I + S (eq. E.1).
 */
#ifndef INFOESRF_H
#define INFOESRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define INFOESRF_OK 0
#define INFOESRF_WARN_NOT_CONVERGED 1
#define INFOESRF_ERR_INVALID_ARG (-1) /* bad dims, NULL, CSR out of range, N < 2, Q < 1, r <= 0 */
#define INFOESRF_ERR_NOT_SPD (-2)     /* PCG curvature p^T C p <= 0 (localization not PSD) */
#define INFOESRF_ERR_NUMERIC (-3)     /* NaN or Inf met in inputs or iterates */
#define INFOESRF_ERR_WORKSPACE (-4)   /* workspace NULL or smaller than required */
#define INFOESRF_ERR_HIP (-5)         /* a HIP runtime call failed */

/* ---- form of the covariance apply (Sec. 2.3) ------------------------------
 * OPERATOR: sum_i z_i o L (z_i o v) (eq. 2.12), 2 N nnz(L) flops per vector,
 *           no storage beyond Z; the only form for BF16 and dense L.
 * BAND:     P = L o (Z Z^T) built once per call as an explicit band with the
 *           stencil's sparsity ((2bz+1)(2bx+1) entries per row, FP64, plus an
 *           FP32 copy for MIXED_FP32), then applied as a banded product,
 *           2 nnz(L) flops per vector.  Same result up to rounding.
 * AUTO:     BAND for a stencil localization in FP64 or MIXED_FP32 when the
 *           band needs at most 2 GiB, else OPERATOR. */
#define INFOESRF_COV_AUTO 0
#define INFOESRF_COV_OPERATOR 1
#define INFOESRF_COV_BAND 2

/* ---- form of the normalized observation covariance S ---------------------
 * S = R^{-1/2} H P H^T R^{-1/2} (the matrix of Theorem 3; every shifted system
 * of Appendix E is (1 + s_q) I + S).
 * OPERATOR: every PCG apply goes through P (in the form above), in the
 *           state domain or on the observed lattice.
 * DENSE:    S is assembled once per call as a dense m x m FP64 matrix (m
 *           applies of P, symmetrized; plus an FP32 copy for MIXED_FP32) and
 *           every PCG apply is an m x m product, 2 m^2 flops per vector.
 *           m <= 16384; not with MIXED_BF16.  Same result up to rounding.
 * AUTO:     DENSE in FP64 or MIXED_FP32 when m <= 4096, an m x m product costs
 *           at most half of an apply of P in the working domain, and
 *           m <= 8 (systems + sketch columns + 16) (forming S takes m applies
 *           of P); else OPERATOR. */
#define INFOESRF_S_AUTO 0
#define INFOESRF_S_OPERATOR 1
#define INFOESRF_S_DENSE 2

/* ---- localization kinds ------------------------------------------------- */
#define INFOESRF_LOC_STENCIL 1 /* stationary stencil on an nz x nx grid */
#define INFOESRF_LOC_DENSE 0   /* explicit n x n matrix (small n, tests) */

/* ---- precision of the covariance applies inside PCG --------------------- */
#define INFOESRF_FP64 0        /* every apply in FP64 */
#define INFOESRF_MIXED_FP32 1  /* FP32 MFMA applies + FP64 residual correction */
#define INFOESRF_MIXED_BF16 2  /* BF16 MFMA applies, FP32 accumulation + FP64 correction */

/* ---- solver scheduling -------------------------------------------------- */
#define INFOESRF_SOLVER_PLAIN 0      /* one launch per iteration over all systems, converged ones masked */
#define INFOESRF_SOLVER_COMPACT 1    /* converged systems retired from the launched set each iteration */
#define INFOESRF_SOLVER_PERSISTENT 2 /* one persistent launch; work queue of systems (batched instances) */
/* MULTISHIFT (perturbation update; the first alternative of Sec. 3.2): one CG process per
 * member on the smallest node's system serves every node as a shift of it (shared Krylov
 * spaces, collinear residuals), one apply of S per member per iteration instead of Q.  It has no
 * preconditioner (n_ritz is used by the mean update only); FP64 and the zero start only.  FP64
 * residual sweeps then check every (q, i) system and correct any above rtol with PCG. */
#define INFOESRF_SOLVER_MULTISHIFT 3
/* BLOCK (perturbation update; the second alternative of Sec. 3.2): for each node one block PCG
 * (O'Leary) over the N members' systems, with the node's limited-memory preconditioner: every
 * member's iterate is optimal over the sum of all members' Krylov spaces, so the block needs
 * fewer iterations than its slowest member alone, at the cost of N x N products per iteration.
 * FP64, zero start, N <= 64; FP64 residual sweeps then check and correct as for MULTISHIFT. */
#define INFOESRF_SOLVER_BLOCK 4

/* ---- where the normalized covariance S is applied ----------------------- */
#define INFOESRF_DOMAIN_STATE 0       /* general H: scatter to state space, apply P, gather */
#define INFOESRF_DOMAIN_OBS_LATTICE 1 /* point observations on a regular sub-lattice, see below */

/* ---- warm start --------------------------------------------------------- */
#define INFOESRF_START_ZERO 0
#define INFOESRF_START_LEARNED 1

/* ---- counters written to infoesrf_stats.counters ------------------------ */
#define INFOESRF_CNT_APPLIES 0       /* covariance applies, counted per vector, all precisions */
#define INFOESRF_CNT_APPLIES_FP64 1  /* of which in FP64 */
#define INFOESRF_CNT_ITERATIONS 2    /* PCG iterations summed over systems (inner + outer) */
#define INFOESRF_CNT_SWEEPS 3        /* FP64 residual-correction sweeps (mixed precision) */
#define INFOESRF_CNT_FALLBACKS 4     /* learned starts replaced by the zero start */
#define INFOESRF_CNT_NOT_CONVERGED 5 /* systems that missed rtol */
#define INFOESRF_CNT_MAX_ITERS 6     /* largest per-system iteration count */
#define INFOESRF_CNT_STATUS 7        /* status code of the call (see return codes) */
#define INFOESRF_NUM_COUNTERS 8

/*
 * Localization L (Sec. 2.3, eq. 2.11): symmetric, entries in [0,1], positive
 * semidefinite.  STENCIL: the state is an nz x nx grid, state index
 * z*nx + x, and L[(z1,x1),(z2,x2)] = table[(dz+bz)*(2bx+1) + (dx+bx)] for
 * dz = z2-z1, dx = x2-x1 (wrapped to the nearest image on a periodic axis)
 * with |dz| <= bz and |dx| <= bx, and 0 otherwise.  The table (device,
 * (2bz+1)*(2bx+1) doubles, row-major) must be point-symmetric:
 * table[dz][dx] == table[-dz][-dx].  A periodic axis needs nx >= 2bx+1
 * (nz >= 2bz+1).  DENSE: `dense` is the n x n matrix (column-major).
 */
typedef struct infoesrf_loc {
  int32_t kind;
  int32_t nz, nx;
  int32_t periodic_z, periodic_x;
  int32_t bz, bx;
  int32_t reserved;
  const double* table;
  const double* dense;
} infoesrf_loc;

/*
 * One filter instance (Sec. 2.2 and Sec. 2.3).
 *   X      n x N forecast members (column i = member x^(i)), ld = n.
 *   H      linear observation operator, m rows in CSR: row k has entries
 *          h_w[e] at state index h_idx[e] for e in [h_ptr[k], h_ptr[k+1]).
 *          Column indices within a row must be strictly increasing; at most
 *          max(64 m, 16 n) entries in total; m <= 4096.
 *   r_var  m diagonal entries of R (all > 0).
 *   loc    localization L.
 * N >= 2 (eq. 2.9 divides by N-1), m >= 1, n = loc.nz * loc.nx.
 */
typedef struct infoesrf_problem {
  int64_t n, N, m;
  const double* X;
  const int32_t* h_ptr;
  const int32_t* h_idx;
  const double* h_w;
  const double* r_var;
  infoesrf_loc loc;
} infoesrf_problem;

/*
 * Observation sub-lattice for INFOESRF_DOMAIN_OBS_LATTICE: the caller asserts
 * that H row k = a*nxo + b (a < nzo, b < nxo) observes exactly one state
 * point, (z0 + a*sz, x0 + b*sx), with any nonzero weight.  Then
 * H P H^T = L_JJ o (W W^T) exactly, and S is applied on the m observed points
 * with the sub-sampled stencil, which is the same operator restricted to the
 * rows H reads.  Periodic sub-axes need nx % sx == 0 (nz % sz == 0).
 */
typedef struct infoesrf_lattice {
  int32_t z0, sz, nzo;
  int32_t x0, sx, nxo;
} infoesrf_lattice;

typedef struct infoesrf_opts {
  double rtol;          /* target of the true FP64 relative residual ||b - C u|| / ||b|| per system (default 1e-8) */
  double inner_rtol;    /* mixed precision: inner PCG tolerance (0 = 1e-2 for BF16, 1e-7 for FP32) */
  int32_t max_iter;     /* cap on PCG iterations per system (inner iterations summed in mixed mode) */
  int32_t n_ritz;       /* p: Ritz pairs in the limited-memory preconditioner (Appendix E), one of
                           0 (none), 4, 8, 10, 12, 16, 20; n_ritz + oversample <= min(48, m) */
  int32_t oversample;   /* extra sketch columns for the randomized eigendecomposition */
  int32_t precision;    /* INFOESRF_FP64 | INFOESRF_MIXED_FP32 | INFOESRF_MIXED_BF16 */
  int32_t solver;       /* INFOESRF_SOLVER_* */
  int32_t warm_start;   /* INFOESRF_START_ZERO | INFOESRF_START_LEARNED */
  int32_t host_sync;    /* 1: read back and return status; 0: no host sync (graph-capture safe) */
  int32_t apply_domain; /* INFOESRF_DOMAIN_STATE | INFOESRF_DOMAIN_OBS_LATTICE */
  infoesrf_lattice lattice;
  uint64_t seed;        /* seed of the library's own sketch generator when sketch == NULL */
  const double* sketch; /* device m x (n_ritz+oversample) Gaussian test matrix, or NULL */
  const void* net;      /* warm-start network from infoesrf_net_load (LEARNED only) */
  int32_t tile_rows;    /* operator-form tile variant: 0 = default; 16, 32, 64, 128 select blocks of
                           16x32, 32x32, 64x16, 64x32 (rows x systems) */
  int32_t cov_form;     /* INFOESRF_COV_AUTO | INFOESRF_COV_OPERATOR | INFOESRF_COV_BAND */
  int32_t fixed_iters;  /* > 0: every system runs exactly this many PCG iterations (FP64 only; the
                           experiments of Sec. 4 and Sec. 5 run 2 and 10) and stops earlier only on
                           an exactly zero residual; reaching the count is not a warning, and
                           stats->converged still reports relres <= rtol.  0: iterate to rtol. */
  int32_t s_form;       /* INFOESRF_S_AUTO | INFOESRF_S_OPERATOR | INFOESRF_S_DENSE */
  int32_t tail_systems; /* FP64 or MIXED_FP32 PCG on the observed lattice with the band form, or
                           with the dense S, when that band or S takes at most 1 MiB in the
                           iterations' precision (m <= 4096): once at most this many systems are
                           left, one persistent launch finishes them (each workgroup iterates a
                           system to convergence, its direction in LDS, applying the band or S in
                           place, the smallest shifts first; from a zero start it also takes the
                           first step and every FP64 residual sweep).  0 = every system from its
                           zero start in one launch (the default; 64 in infoesrf_update_batched
                           when it does not take its one-launch path), -1 = never. */
  int32_t warm_fp32;    /* learned start: 0 = BF16 inference on MFMA with FP32 accumulation
                           (default), 1 = FP32 inference */
  int32_t reserved[2];
} infoesrf_opts;

/* Per-system results (device arrays, each may be NULL).  Systems of the
 * perturbation update are ordered s = q*N + i (node-major); the mean update
 * has one system. */
typedef struct infoesrf_stats {
  int32_t* iters;     /* PCG iterations (inner + outer) */
  double* relres;     /* final true relative residual in FP64 */
  uint8_t* converged; /* 1 when relres <= rtol */
  int64_t* counters;  /* INFOESRF_NUM_COUNTERS totals of the call */
} infoesrf_stats;

/* Fills *opts with defaults: rtol 1e-8, max_iter 1000, n_ritz 10, oversample 10,
 * FP64, COMPACT solver, zero start, host_sync 1, state domain. */
void infoesrf_default_opts(infoesrf_opts* opts);

/* Bytes of device workspace needed by a call with this problem, Q nodes
 * (Q = 0 for infoesrf_mean_update, B vectors for infoesrf_cov_apply via
 * infoesrf_cov_apply_workspace_bytes) and options.  Returns 0 on invalid
 * arguments (see infoesrf_last_error). */
size_t infoesrf_workspace_bytes(const infoesrf_problem* prob, int32_t Q, const infoesrf_opts* opts);
size_t infoesrf_cov_apply_workspace_bytes(const infoesrf_problem* prob, int64_t B, const infoesrf_opts* opts);

/*
 * PV = P V with P = L o (Z Z^T) (eq. 2.11), evaluated in the operator form
 * sum_i z_i o L (z_i o v) (eq. 2.12); Z is formed from prob->X.
 *   V   n x B state-space vectors, column b at V + b*ldv (ldv >= n).
 *   PV  n x B output, column b at PV + b*ldpv (ldpv >= n).  May not alias V.
 * opts->precision selects FP64, FP32 or BF16 (FP32 accumulation) arithmetic.
 */
int infoesrf_cov_apply(const infoesrf_problem* prob, const double* V, int64_t ldv, int64_t B, double* PV,
                       int64_t ldpv, const infoesrf_opts* opts, void* ws, size_t ws_bytes, void* stream);

/*
 * infoesrf_cov_apply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and result, with no workspace argument.
 * Its scratch is a fixed array of INFOESRF_NOALLOC_SCRATCH_BYTES (64 MiB) per
 * device, part of the library's device code, held from the library's load
 * until the process ends; the call allocates nothing (no hipMalloc/hipFree).
 *   Limit: a call whose infoesrf_cov_apply_workspace_bytes(prob, B, opts)
 *   exceeds INFOESRF_NOALLOC_SCRATCH_BYTES returns INFOESRF_ERR_WORKSPACE
 *   (n = 4096, N = 40: up to 1667 columns per call with the band form,
 *   1986 with the operator form; n = 256, N = 16: about 32000).
 *   Sharing: every call on a device uses that device's array and leaves its
 *   contents behind; nothing in it needs to start at zero.  Calls that
 *   overlap on one device (other host threads, other streams) race: order
 *   them on one stream or serialize them.  The device is the current one, on
 *   which `stream` must live.
 * Arguments, layouts, ownership and the other errors as infoesrf_cov_apply.
 */
#define INFOESRF_NOALLOC_SCRATCH_BYTES (64ull << 20)
int infoesrf_cov_apply_noalloc(const infoesrf_problem* prob, const double* V, int64_t ldv, int64_t B, double* PV,
                               int64_t ldpv, const infoesrf_opts* opts, void* stream);

/*
 * Mean update (Sec. 3.2, eq. 3.4): mean_a = mu + P H^T R^{-1/2} u0 where
 * (I + S) u0 = R^{-1/2} (y - H mu) is solved by PCG with the limited-memory
 * preconditioner.  y: m observations.  mean_a: n outputs.
 */
int infoesrf_mean_update(const infoesrf_problem* prob, const double* y, double* mean_a, const infoesrf_opts* opts,
                         infoesrf_stats* stats, void* ws, size_t ws_bytes, void* stream);

/*
 * Perturbation update (Sec. 3.2, eq. 3.5 in the normalized form of eq. E.1):
 * for every node q and member i solve C_q u_{q,i} = R^{-1/2} w_i by PCG,
 * u_bar_i = sum_q p_q u_{q,i}, z_a^(i) = z^(i) - P H^T R^{-1/2} u_bar_i, and
 * write Xa_pert = sqrt(N-1) Z_a (n x N, ld = n): the analysis deviations, so
 * the analysis ensemble is mean_a 1^T + Xa_pert.
 *   s_nodes, p_weights  host arrays of Q quadrature nodes (>= 0) and
 *                       weights (>= 0), e.g. from infoesrf_quadrature_elliptic.
 *   y                   m observations; not used by the perturbation update
 *                       (kept for callers that pass them), may be NULL.
 * Q must be in [1, 64].
 */
int infoesrf_perturbation_update(const infoesrf_problem* prob, int32_t Q, const double* s_nodes,
                                 const double* p_weights, const double* y, double* Xa_pert,
                                 const infoesrf_opts* opts, infoesrf_stats* stats, void* ws, size_t ws_bytes,
                                 void* stream);

/*
 * Many independent filter instances of uneven n, N, m, Q in one call (the
 * uneven batch of Section 3.2's remark that the solves parallelize across
 * members and nodes, extended across instances).  Instance j is probs[j]
 * with Q[j] nodes s_nodes[j], p_weights[j] (host arrays), observations y[j]
 * (device, may be NULL unless its mean is wanted), mean_a[j] (device, n_j; the
 * mean update of eq. 3.4 is skipped when mean_a or mean_a[j] is NULL) and
 * Xa_pert[j] (device, n_j x N_j, as in infoesrf_perturbation_update).
 *   lattices  host array of count observed lattices, read only when
 *             opts->apply_domain is INFOESRF_DOMAIN_OBS_LATTICE (instance j
 *             then uses lattices[j] in place of opts->lattice); else NULL.
 *   stats     per-system arrays hold sum_j (Q_j N_j + 1) entries in instance
 *             order (node-major systems, then the mean system); counters are
 *             the totals over all instances, the status the most severe one.
 *   ws        one workspace of infoesrf_batched_workspace_bytes() bytes,
 *             split into one slice per instance.
 * One launch (infoesrf_batched_one_launch returns 1): when every instance's
 * inner PCG can run in the persistent kernel (compacted solver, zero start,
 * tail_systems >= 0, FP64 or MIXED_FP32, the band on the observed lattice or
 * the dense S, m <= 4096, one n_ritz for all), the instances' set-ups are
 * forked onto library-owned streams (default priority) that wait on and join
 * back into `stream` through events (its mean system, at shift 0, joins an
 * instance's perturbation systems); then one persistent launch per kernel
 * shape (instances with m <= 1024, and larger ones) runs every sweep of every
 * instance's systems from a queue (largest instance first, smallest shifts
 * first within it): a workgroup restarts a system from its true FP64 residual
 * while that is above rtol, up to the sweep budget (2 for FP64 and 4 for
 * MIXED_FP32 inner applies with host_sync 0, 40 with host_sync 1); then each
 * instance's quadrature sum and final update.  The call makes no host read
 * before the final status when host_sync is 1 and none at all when it is 0
 * (capturable in a HIP graph).
 * Otherwise instances run largest first on a pool of library-owned streams
 * (default priority) that fork from and join back into `stream`, each as the
 * single-instance calls.  With host_sync 1 the return code is the most severe
 * instance code and the message names the first failing instance (an
 * instance that fails does not stop the others); with host_sync 0 the status
 * is left in stats->counters.  Validation of every instance precedes any
 * device work.
 */
size_t infoesrf_batched_workspace_bytes(const infoesrf_problem* probs, int32_t count, const int32_t* Q,
                                        const infoesrf_opts* opts, const infoesrf_lattice* lattices);
/* 1 when infoesrf_update_batched takes the one-launch path for these arguments, else 0 (also
 * for invalid arguments).  Host only. */
int infoesrf_batched_one_launch(const infoesrf_problem* probs, int32_t count, const int32_t* Q,
                                const infoesrf_opts* opts, const infoesrf_lattice* lattices);
int infoesrf_update_batched(const infoesrf_problem* probs, int32_t count, const int32_t* Q,
                            const double* const* s_nodes, const double* const* p_weights,
                            const double* const* y, double* const* mean_a, double* const* Xa_pert,
                            const infoesrf_opts* opts, const infoesrf_lattice* lattices, infoesrf_stats* stats,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * Elliptic quadrature rule (Appendix D, eq. D.1; host): with k^2 = ell/(1+ell)
 * and K = K(k^2), u_q = (q - 1/2) K / Q, s_q = sc^2(u_q|k^2),
 * p_q = (2K/(pi Q)) dn(u_q|k^2)/cn^2(u_q|k^2) / (1 + s_q).  ell should exceed
 * the largest eigenvalue of S.  Writes Q nodes and weights (host arrays).
 */
int infoesrf_quadrature_elliptic(int32_t Q, double ell, double* s_nodes, double* p_weights);

/* Trigonometric rule with Gauss-Legendre nodes (Appendix D, eq. D.2; host). */
int infoesrf_quadrature_gauss_legendre(int32_t Q, double* s_nodes, double* p_weights);

/* Static description of a return code, and the message of the calling
 * thread's last error ("" if none). */
const char* infoesrf_error_string(int code);
const char* infoesrf_last_error(void);

/*
 * Learned warm start (an extension of the method; the paper starts every
 * system from zero).  A 1-D convolutional network over the m observation rows
 * runs once per member: the trunk (1 -> H -> H -> H -> D channels, D = 4, odd
 * kernel width K <= 15, "same" zero padding, GELU after the first three
 * layers, FP32 parameters) maps bh_i = sqrt(m) b_i / ||b_i|| to Y_i (D x m).
 * The shift enters last: system (q, i), c_q = 1 / (1 + s_q), starts from
 *     u0 = (||b_i|| / sqrt(m)) sum_d c_q^(d+1) Y_i[d]
 * (the Neumann series of C_q^{-1} b = sum_d c^(d+1) (-S)^d b has this form,
 * eq. E.1), so the convolutions cost N, not Q N, passes per update.  A created
 * network's output layer is zero (it predicts the zero start until trained).
 * With warm_start = INFOESRF_START_LEARNED and opts->net set, the perturbation
 * update starts every system from u0; a system whose u0 is not finite starts
 * from zero and counters[FALLBACKS] counts it.  The mean system always starts
 * from zero.
 *
 * Handles own device memory (parameters, Adam moments, a gradient buffer),
 * allocated by create/load and released by free; never on the update path.
 * File: little-endian "IENET002", 5 int32 (4, 1, H, K, D), then the FP32
 * parameters W1 (H x 1 x K) b1 (H) W2 (H x H x K) b2 W3 b3 W4 (D x H x K) b4 (D).
 *
 * Batches (FP32, row-contiguous device arrays): X is B x m (the members' bh),
 * Y is B x D x m (the trunk output); training adds cq, the Q values
 * c_q = 1 / (1 + s_q) shared by the batch, and targets T, B x Q x m
 * (T[b, q] = sqrt(m) u*_{q,b} / ||b_b|| for exact solutions u*).  Workspaces
 * from infoesrf_net_workspace_bytes (training != 0 keeps every activation for
 * the backward pass; Q is read only then).  The loss is the mean over the B Q
 * systems of ||y - T|| / ||T|| with y the head's output, written to the device
 * float *loss; gradients have the parameter layout; a training step is one
 * Adam update (beta1 0.9, beta2 0.999, eps 1e-8).
 */
int infoesrf_net_create(int32_t hidden, int32_t kernel, uint64_t seed, void** net);
int infoesrf_net_load(const char* path, void** net);
int infoesrf_net_save(const void* net, const char* path);
void infoesrf_net_free(void* net);
int64_t infoesrf_net_param_count(const void* net);
int infoesrf_net_get_params(const void* net, float* host);        /* host array of param_count */
int infoesrf_net_set_params(void* net, const float* host);        /* also resets the Adam state */
size_t infoesrf_net_workspace_bytes(const void* net, int64_t B, int64_t Q, int64_t m, int32_t training);
int infoesrf_net_forward(const void* net, const float* X, int64_t B, int64_t m, float* Y, void* ws,
                         size_t ws_bytes, void* stream);
/* The same trunk output with BF16 weights and activations on MFMA (v_mfma_f32_16x16x32_bf16) and
 * FP32 accumulation, as the learned start runs it by default; needs H <= 64, H % 8 == 0.  Same
 * workspace (training = 0).  The output differs from infoesrf_net_forward by the BF16 rounding of
 * weights and activations (a relative error of order 1e-2). */
int infoesrf_net_forward_bf16(const void* net, const float* X, int64_t B, int64_t m, float* Y, void* ws,
                              size_t ws_bytes, void* stream);
int infoesrf_net_gradients(const void* net, const float* X, const float* cq, const float* T, int64_t B, int64_t Q,
                           int64_t m, float* grads, float* loss, void* ws, size_t ws_bytes, void* stream);
int infoesrf_net_train_step(void* net, const float* X, const float* cq, const float* T, int64_t B, int64_t Q,
                            int64_t m, float lr, float* loss, void* ws, size_t ws_bytes, void* stream);

/*
 * Training pairs for the warm start: solves the Q N systems of the
 * perturbation update exactly as infoesrf_perturbation_update does (same
 * options; warm_start must be ZERO) and writes the network's batch of the N
 * members: X (N x m) their bh, cq (Q) the shift factors c_q = 1 / (1 + s_q),
 * and T (N x Q x m) with T[i, q] = sqrt(m) u*_{q,i} / ||b_i||, the converged
 * solutions scaled like the head's output (FP32, device).  y may be NULL (the
 * systems do not depend on it).  Workspace: infoesrf_workspace_bytes(prob, Q, opts).
 */
int infoesrf_warmstart_pairs(const infoesrf_problem* prob, int32_t Q, const double* s_nodes,
                             const double* p_weights, const double* y, float* X, float* cq, float* T,
                             const infoesrf_opts* opts, infoesrf_stats* stats, void* ws, size_t ws_bytes,
                             void* stream);

/*
 * Autotuner of the covariance apply's block shape (process-wide).  For the
 * apply the solve of (prob, Q, opts) would run -- its form, domain and inner
 * precision, plus the FP64 apply of the residual sweeps -- times every block
 * shape (band form: 8/16/32/64 systems per block; operator form: tiles 16, 32,
 * 64, 128) with HIP events at three batch sizes (the Q N systems, a quarter
 * and a sixteenth of them), and records the fastest per batch-size bucket
 * (>= 256, 64..255, < 64 systems) for grids of this shape.  Later applies on
 * such grids use the recorded choice unless opts->tile_rows forces one.  The
 * band form's results do not depend on the choice (each output keeps its
 * summation order); the operator form's do by rounding only.  Synchronizes
 * the stream.  Workspace: infoesrf_workspace_bytes(prob, Q, opts).
 *   report  host int32[24] or NULL: per measured (precision, batch) the
 *           precision, the batch size, the chosen shape and the microseconds
 *           per launch.
 * infoesrf_autotune_reset forgets every recorded choice.
 */
int infoesrf_autotune(const infoesrf_problem* prob, int32_t Q, const infoesrf_opts* opts, void* ws, size_t ws_bytes,
                      void* stream, int32_t* report);
void infoesrf_autotune_reset(void);

/*
 * Cycled assimilation around the update (the experiment of Sec. 5).
 *
 * infoesrf_l96_forecast: advances the k columns of X (n = nz nx rows each,
 * column c at X + c ld, state index layer * nx + site, device FP64) by `steps`
 * classical RK4 steps of length dt of the coupled multi-layer Lorenz-96 model
 * (Sec. 5.1, eq. 5.1): periodic sites, forcing[j] per layer (device, nz
 * values), coupling gamma between adjacent layers, no exchange through the
 * top and bottom layers.  n <= 8192 (a column is integrated on chip).
 *
 * infoesrf_observe: y = H x + noise for one state x (device n), noise (device
 * m, may be NULL), H the problem's CSR rows.
 *
 * infoesrf_rtps_assemble: analysis members Xout[:, i] = mean_a + f o Xa'[:, i]
 * with the relaxation-to-prior-spread factor f_k = 1 + alpha (s_f - s_a)/s_a
 * per state variable (Whitaker & Hamill; Sec. 5.3 uses alpha = 0.01), s_f the
 * standard deviation of the forecast members Xf (n x N, ldf), s_a that of the
 * analysis deviations Xa' (n x N, lda, e.g. the output of
 * infoesrf_perturbation_update); f_k = 1 where s_a = 0.  Xout may alias Xf.
 */
int infoesrf_l96_forecast(double* X, int64_t ld, int64_t k, int32_t nz, int32_t nx, const double* forcing,
                          double gamma, double dt, int32_t steps, void* stream);
int infoesrf_observe(const infoesrf_problem* prob, const double* x, const double* noise, double* y, void* stream);
int infoesrf_rtps_assemble(const double* Xf, int64_t ldf, const double* mean_a, const double* Xa_pert, int64_t lda,
                           int64_t n, int64_t N, double alpha, double* Xout, int64_t ldo, void* stream);

/*
 * Measurement hooks (results are unaffected).  While enabled, every launch of
 * a covariance-apply kernel is bracketed by HIP events recorded on the stream
 * it runs on, and the kernel adds the number of vectors it applies and their
 * algorithmic FLOPs to device counters: 2 N nnz(L) + 3 n N per vector in
 * operator form, 2 nnz(L) in band form (nnz(L) = nonzeros of the localization
 * on the grid the launch uses, n its rows).  Algorithmic bytes are counted as
 * well: per vector one read of its input column and one write of its output
 * column; per launch one read of the band (band form) or of Z (operator form).
 * infoesrf_profile_read synchronizes the device and returns, per slot
 * (INFOESRF_PROF_*), the summed kernel time in ms, the launches, the vectors
 * applied, the FLOPs and the bytes.  Enabling resets the totals.  The hook
 * allocates its event pool and counters when enabled; it is meant for
 * benchmarks, not for the update path.  Launches from several threads are
 * serialized by a lock while it is on.
 */
#define INFOESRF_PROF_OP_FP64 0
#define INFOESRF_PROF_OP_FP32 1
#define INFOESRF_PROF_OP_BF16 2
#define INFOESRF_PROF_BAND_FP64 3
#define INFOESRF_PROF_BAND_FP32 4
#define INFOESRF_PROF_PCG 5 /* the fused PCG step: vectors = live systems, bytes per system 6-8 m-vector passes */
#define INFOESRF_PROF_TAIL 6 /* the persistent PCG kernel: vectors = system-iterations, FLOPs per
                                system-iteration = the apply (2 nnz(L) on the observed lattice, or
                                2 m^2 with the dense S) + the PCG step (12 + 8 p) m; bytes per
                                system = a read of its residual and a read and write of its solution
                                (a solve it starts) or a read and write of x, r, p (one it takes over
                                from the batched loop), plus the band (or S) and the FP32 Ritz bases
                                once per launch */
#define INFOESRF_PROF_SLOTS 7
int infoesrf_profile_enable(int on);
/* Restricts the hook to the slots whose bit (1 << slot) is set in mask (all slots after enabling);
 * launches of other slots then run without events.  Fewer event pairs perturb the timeline less. */
int infoesrf_profile_select(uint32_t mask);
int infoesrf_profile_read(double ms[7], int64_t launches[7], int64_t vectors[7], double flops[7], double bytes[7]);

#ifdef __cplusplus
}
#endif

#endif /* INFOESRF_H */
