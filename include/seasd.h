/*
 * seasd.h - C ABI of the MI355X (gfx950) Spectral Ewald far-field mobility
 * library: the periodic grand-mobility product of Spectral Ewald accelerated
 * Stokesian Dynamics and the GMRES far-field solve that calls it.
 *
 * Reference: M. Wang and J. F. Brady, "Spectral Ewald Acceleration of
 * Stokesian Dynamics for polydisperse suspensions" (arXiv:1506.08481).
 *
 * Operator. For N spheres with centres r_i and radii a_i in a periodic cell,
 * y = M x with 12 components per sphere:
 *   x_i = (F_i[3], T_i[3], S_i[5], s_i)  force, torque, traceless stresslet
 *         and pressure-moment coordinate, all exerted by sphere i on the fluid;
 *   y_i = (U_i[3], W_i[3], E_i[5], e_i)  velocity, spin, (minus the ambient)
 *         rate of strain and its trace coordinate.
 * The five traceless coordinates use the orthonormal basis
 *   Y0 = (xx - yy)/sqrt2, Y1 = (2zz - xx - yy)/sqrt6,
 *   Y2 = (xy + yx)/sqrt2, Y3 = (xz + zx)/sqrt2, Y4 = (yz + zy)/sqrt2,
 * and the trace coordinate is trace/sqrt3, so that S:E is a plain dot product.
 * M is the Rotne-Prager-level grand mobility built from the Faxen laws and
 * multipole expansion (Sec. 2.1, eqs. faxen-f, faxen-t, faxen-s,
 * mul-expand), the periodic Oseen tensor (Sec. 2.2, eq. oseen-peridoic) and
 * the compressible-solvent pressure-moment couplings (Sec. 2.3, eqs.
 * pres-vel-disturb, faxen-p, pres-multi-expans, wave-dist-S). The 11x11
 * incompressible block is symmetric positive definite; the trace row is the
 * one-way pressure coupling of Sec. 2.3, so M as a whole is not symmetric.
 *
 * Evaluation (Sec. 3): Hasimoto's Ewald split (Sec. 2.2, eqs.
 * oseen-ewald-rs, oseen-ewald-ws, source-split) into
 *   - a real-space pair sum over neighbour bins within
 *     r_c = rc_factor (a_i + a_j) (Sec. 3.3), recomputed on every call;
 *   - a Spectral Ewald wave-space part (Sec. 3.1-3.2, eqs. rp-wave-tq,
 *     shape, grid-space, wave-result, parseval-sum): Gaussian spreading of
 *     the force moments to an M^3 grid with the Faxen operators applied to the
 *     window (the real-space size approach of Sec. 3.2), forward 3-D FFT,
 *     k-space Green's-function multiply with deconvolution, inverse FFT and
 *     Gaussian gather by the trapezoid rule;
 *   - the single-sphere self terms minus the wave-space self terms
 *     (eq. uf-self and its analogues).
 *
 * Conventions for every entry point:
 *   - Device arrays are caller-owned (for example torch tensor data pointers)
 *     and must stay valid until the work queued on `stream` has finished.
 *     The library never frees them. It owns only its workspace, which it
 *     allocates on first use for a given size and keeps with the handle.
 *   - Layouts are row-major: pos [n][3], radius [n], x/y/b [n][12], all FP64
 *     whatever the internal precision.
 *   - box is a HOST array of 9 doubles holding the lattice vectors a1, a2, a3
 *     as consecutive triples (the columns of the paper's matrix A, Sec. 2.2).
 *     Accepted cells: a1 = (a1x, 0, 0), a2 = (a2x, a2y, 0), a3 = (0, 0, a3z)
 *     with a1x, a2y, a3z > 0 and |a2x| <= a1x: cubes, rectangular boxes and
 *     boxes sheared in the x-y plane, such as the simple-shear cell
 *     a2 = (gamma L, L, 0) of Sec. 3.2 (eq. non-ortho-shape). Other shapes
 *     return SEASD_E_UNSUPPORTED. The Spectral Ewald grid lives in the
 *     fractional coordinates t = A^-1 r (Sec. 3.1), with M points along each
 *     lattice direction.
 *   - Work is queued on `stream` (a hipStream_t; NULL = default stream).
 *     seasd_mobility_apply returns without synchronising unless the
 *     configuration asks for input checks; seasd_solve_farfield synchronises.
 *   - Return value: 0 on success, negative on error, positive for warnings.
 *   - A handle is not thread safe; use one handle per host thread / stream.
 *     Calls made through different handles may overlap on one GPU.
 */
#ifndef SEASD_H
#define SEASD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes --------------------------------------------------------- */
#define SEASD_OK                0
#define SEASD_E_INVALID_ARG    -1   /* bad pointer, size or parameter           */
#define SEASD_E_NONFINITE      -2   /* NaN or Inf in positions, radii or x      */
#define SEASD_E_OVERLAP        -3   /* two spheres closer than a_i + a_j        */
#define SEASD_E_CUTOFF         -4   /* cut-off or window does not fit the cell  */
#define SEASD_E_SINGULAR       -5   /* a preconditioner block is singular       */
#define SEASD_E_HIP            -6   /* a HIP runtime call failed                */
#define SEASD_E_NOMEM          -7   /* workspace allocation failed              */
#define SEASD_E_UNSUPPORTED    -8   /* valid request this build does not handle */
#define SEASD_E_FORMAT         -9   /* weights file missing, wrong or corrupt   */
#define SEASD_E_SCRATCH       -10   /* input too large for the static workspace */
                                    /* of seasd_mobility_apply_static           */
#define SEASD_W_NOT_CONVERGED   1   /* solve stopped at max_iter above tol      */
#define SEASD_W_PRECOND_FALLBACK 2  /* learned preconditioner rejected; the     */
                                    /* block-diagonal one was used instead      */

/* ---- configuration --------------------------------------------------------- */
#define SEASD_FP64 0
#define SEASD_FP32 1
#define SEASD_MIXED 2  /* FP64 products, except inside the GMRES Arnoldi steps  */
                       /* of seasd_solve_farfield, seasd_solve_mixed and        */
                       /* seasd_brownian_farfield, which take the FP32 product: */
                       /* each restart's true residual stays FP64, so the       */
                       /* restart cycles are steps of iterative refinement      */

#define SEASD_PARTS_REAL 1  /* real-space pair sum (Sec. 3.3)                 */
#define SEASD_PARTS_WAVE 2  /* Spectral Ewald wave-space sum (Sec. 3.1)       */
#define SEASD_PARTS_SELF 4  /* single-sphere terms minus wave-space self      */
#define SEASD_PARTS_ALL  7

#define SEASD_PRECOND_NONE      0
#define SEASD_PRECOND_BLOCKDIAG 1   /* per-sphere inverse of the self block (Sec. 4.2) */
/* 2 is not accepted: per-sphere rescalings S B S of the blocks by the        */
/* network were measured to slow GMRES down (more iterations than the blocks) */
#define SEASD_PRECOND_LEARNED_GUESS 3 /* block-diagonal blocks, the network's guess   */

#define SEASD_SIZE_REAL   0 /* Faxen operators applied to the window on both  */
                            /* sides (the real-space approach of Sec. 3.2)   */
#define SEASD_SIZE_HYBRID 1 /* Faxen operators on the window when spreading;  */
                            /* when reading, the second derivatives are taken */
                            /* in k space (eq. parseval-sum-2 with the grid-  */
                            /* space H of eq. grid-space: the hybrid approach */
                            /* of Sec. 3.2; 4 forward, 7 inverse transforms)  */
#define SEASD_SIZE_WAVE   2 /* every Faxen operator in k space (eqs. wave-   */
                            /* only-*): SEASD_E_UNSUPPORTED in this build     */

typedef struct seasd_config {
    int32_t grid[3];        /* M, grid points along each lattice direction: equal,    */
                            /* a power of two, 8..256 (unequal: SEASD_E_UNSUPPORTED)  */
    int32_t P;              /* window support in grid points per dimension, 4..min(M,32), */
                            /* odd or even (eq. fgg-exp; centred either way)           */
    int32_t size_approach;  /* SEASD_SIZE_REAL or SEASD_SIZE_HYBRID (Sec. 3.2); the      */
                            /* wave-space approach returns SEASD_E_UNSUPPORTED          */
    double  m;              /* window shape parameter (eq. theta-param); <= 0: sqrt(pi P)   */
    double  xi;             /* Ewald splitting parameter, Beenakker convention (Sec. 2.2)   */
    double  rc_factor;      /* real-space cut-off r_c = rc_factor (a_i + a_j), > 1           */
    double  eta;            /* solvent viscosity, > 0                                        */
    int32_t precision;      /* SEASD_FP64, SEASD_FP32 or SEASD_MIXED: spreading, FFTs and    */
                            /* gather (SEASD_MIXED: FP32 only in solve Arnoldi steps); the */
                            /* real-space pair sum and the solver always run in FP64        */
    int32_t parts;          /* SEASD_PARTS_* bit mask; SEASD_PARTS_ALL for the operator      */
    int32_t compressible;   /* 1: include the pressure-moment row and column; 0: zero them  */
    int32_t checks;         /* 1: check inputs (finite, no overlap) and synchronise          */
    /* far-field solve (seasd_solve_farfield) */
    double  tol;            /* stop when ||b - M x||_2 / ||b||_2 <= tol                      */
    int32_t max_iter;       /* total GMRES iterations (matrix-vector products) allowed       */
    int32_t restart;        /* Krylov subspace size before restart, 1..200                   */
    int32_t precond;        /* SEASD_PRECOND_*                                               */
} seasd_config;

typedef struct seasd_solve_stats {
    int32_t iterations;      /* Arnoldi steps taken (one M x each)                  */
    int32_t restarts;        /* completed restart cycles                            */
    int32_t matvecs;         /* all products with M, true-residual checks included  */
    int32_t converged;       /* 1 if the true residual met tol                      */
    double  true_residual;   /* ||b - M x|| / ||b|| from a fresh product at exit     */
    double  setup_ms;        /* block-diagonal preconditioner construction           */
    double  solve_ms;        /* total wall time of the call                          */
    int32_t precond_used;    /* SEASD_PRECOND_* actually applied                     */
    int32_t guess_used;      /* 1 if the learned initial guess was kept              */
    double  initial_residual;/* ||b' - A x0|| / ||b'|| of the starting iterate       */
    double  guess_scale;     /* alpha applied to the learned guess (0: dropped)      */
    double  learned_ms;      /* learned guess: graph, network, scaling product       */
    int32_t inner_iterations;/* mixed solve: near-field GMRES iterations, all solves */
} seasd_solve_stats;

/* Near-field force-velocity resistance for seasd_solve_mixed: a symmetric
 * positive semi-definite block-sparse matrix of 6x6 blocks (force and torque
 * against velocity and spin) in compressed block-row form, on the device. */
typedef struct seasd_bsr6 {
    int64_t        nnzb;     /* stored blocks                                        */
    const int32_t* rowptr;   /* [n + 1] device: blocks of block row i are            */
                             /*   rowptr[i] .. rowptr[i + 1] - 1                     */
    const int32_t* col;      /* [nnzb] device: block column of each stored block     */
    const double*  val;      /* [nnzb][6][6] device, row-major                       */
} seasd_bsr6;

typedef struct seasd_handle_s* seasd_handle;

/* Create a handle bound to HIP device `device` (the caller's device ordinal).
 * Allocates nothing on the device yet. Returns SEASD_E_HIP if the device
 * cannot be selected or is not a gfx950 part. */
int seasd_create(seasd_handle* handle, int32_t device);

/* Release the handle and all workspace it owns. Safe on NULL. */
int seasd_destroy(seasd_handle handle);

/* Fill *cfg with defaults: M=64 (all directions), P=16, m=sqrt(pi P), xi=0.5, rc_factor=4
 * (the paper's r_c = 4(a_i+a_j), Sec. 5.1.2 and 5.3), eta=1, FP64, all parts,
 * compressible, checks on, tol 1e-6, max_iter 1000, restart 50, block-diagonal
 * preconditioner. */
int seasd_default_config(seasd_config* cfg);

/* Validate and store the configuration (parameters of Sec. 5.1: M, P, m, xi,
 * r_c). Workspace is sized lazily on the next call that needs it. Returns
 * SEASD_E_INVALID_ARG for out-of-range values. */
int seasd_set_config(seasd_handle handle, const seasd_config* cfg);

/* y = M x: the grand mobility applied to the force moments (Sec. 3).
 *   n      number of spheres, >= 1
 *   pos    device [n][3] centres (any real coordinates; wrapped into the cell)
 *   radius device [n] radii, > 0
 *   box    host [9] lattice vectors (see the accepted cells above)
 *   x      device [n][12] force moments
 *   y      device [n][12] output, overwritten (may not alias x)
 * Errors: SEASD_E_INVALID_ARG, SEASD_E_UNSUPPORTED (cell shape),
 * SEASD_E_CUTOFF (window wider than the grid), SEASD_E_NOMEM, SEASD_E_HIP; with
 * checks on also SEASD_E_NONFINITE and SEASD_E_OVERLAP (y is then undefined). */
int seasd_mobility_apply(seasd_handle handle, int64_t n,
                         const double* pos, const double* radius, const double* box,
                         const double* x, double* y, void* stream);

/* Allocation-free variant of seasd_mobility_apply, for callers that cannot
 * allocate device memory: code recorded under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc. Same arguments, result and
 * kernels as seasd_mobility_apply with the handle's configuration, but every
 * workspace buffer (binned copies, neighbour list, window records, grids,
 * spectra, twiddles, counters) is carved from one static device array of
 * SEASD_STATIC_SCRATCH_BYTES per GPU, held until the process ends; the call
 * makes no hipMalloc, hipFree or other allocating call. The neighbour list
 * takes whatever the fixed buffers leave (at most 4096 slots per sphere).
 * The call synchronises `stream` once, after queuing the pair sum and the
 * spreading/FFT work, to check that every neighbour list fitted.
 * Limits: about 1.2 kB per sphere (FP64, P = 32) plus the list, and
 * 32 M^3 bytes of grids in FP64 (64 M^3 with the hybrid size approach):
 * e.g. n = 16384 spheres on a 64^3 grid fit with room for 700-entry lists.
 * Returns SEASD_E_SCRATCH, before queuing any work, when the fixed buffers do
 * not fit, and after the product's first half when a neighbour list would
 * overflow the remaining room (y is then not written); otherwise the codes of
 * seasd_mobility_apply. Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (each call clears what must start at zero):
 * calls that overlap in time on one GPU, through any handles, race. */
#define SEASD_STATIC_SCRATCH_BYTES (128u << 20)
int seasd_mobility_apply_static(seasd_handle handle, int64_t n,
                                const double* pos, const double* radius, const double* box,
                                const double* x, double* y, void* stream);

/* Far-field solve (Sec. 4.1, eq. HI-ff with no near-field resistance) by
 * right-preconditioned restarted GMRES in FP64 on the device, with the
 * block-diagonal far-field preconditioner of Sec. 4.2 (each sphere's 11x11
 * incompressible block with its own periodic images, inverted in FP64).
 * The pressure moments follow the paper's one-way coupling (Sec. 2.3): only
 * the part of each pressure moment fixed by its own trace equation,
 * s_self = b_trace / m_self, drives source flows while F, T, S are solved;
 * the interaction part comes afterwards from the pressure Faxen law:
 *   A f = b_f - C s_self,   s = (b_trace - D f) / m_self,
 * with A the 11x11 incompressible block of M, C its source-flow column and D
 * its pressure row. With compressible = 0 the trace is dropped (s = 0).
 *   b      device [n][12] right-hand side (U, W, E, e)
 *   x      device [n][12] in: initial guess for F, T, S (trace ignored),
 *          out: solution
 *   stats  host, may be NULL; true_residual is ||b' - A f|| / ||b'|| of the
 *          incompressible system (b' = b_f - C s_self) from a fresh product
 * With precision SEASD_MIXED the Arnoldi steps use the FP32 product and
 * every restart's true residual the FP64 one: each cycle solves for the
 * correction of the current iterate with the FP32 operator (iterative
 * refinement), is also ended once its residual estimate falls by 1e-5, and
 * tol is met on the FP64 residual.
 * Synchronises `stream`. Returns SEASD_W_NOT_CONVERGED if max_iter was reached
 * with the true residual above tol (x then holds the last iterate), and the
 * errors of seasd_mobility_apply or SEASD_E_SINGULAR. */
int seasd_solve_farfield(seasd_handle handle, int64_t n,
                         const double* pos, const double* radius, const double* box,
                         const double* b, double* x, seasd_solve_stats* stats, void* stream);

/* The near-field / far-field hydrodynamic solve of Sec. 4.1 for a
 * caller-supplied near-field resistance R (eqs. HI-nf, HI-ff):
 *   0 = -R U + F + Fp,   [U; -E] = -M [F; S],
 * with M the force-torque-stresslet block of the grand mobility (the
 * product of seasd_mobility_apply on components 0..10). Following eqs.
 * HI-solve and fM-comp, with Rt = R + lambda I and D = diag(Rt^-1, 0), GMRES
 * solves Mt y = (lambda M - I) D [Fp; 0] + [0; E], Mt = (I - lambda M) D + M,
 * for y = [F + lambda U; S]; every application of Mt costs one product with M
 * and one near-field solve with Rt. The near-field solves use GMRES with the
 * inverses of the diagonal blocks of Rt as preconditioner (the paper's IC0
 * after reverse Cuthill-McKee ordering is a sequential triangular solve);
 * the outer preconditioner is the block-diagonal approximation of Sec. 4.2
 * (eq. rfu-approx: per sphere (I - lambda M_ii) diag(Rt_ii^-1, 0) + M_ii,
 * M_ii with its own periodic images, inverted in FP64). Pressure moments are
 * not part of this solve.
 *   rnf     near-field resistance (device arrays); every block row that has
 *           no stored diagonal block needs lambda > 0
 *   lambda  shift, > 0 (the paper suggests 6 pi eta a with a reference radius);
 *           the solution does not depend on it
 *   fp      device [n][6] interparticle plus near-field strain forces and torques
 *   einf    device [n][5] imposed strain, traceless orthonormal basis
 *   f, s, u device outputs: [n][6] far-field hydrodynamic force and torque,
 *           [n][5] far-field stresslet, [n][6] velocity and spin
 * Uses the handle's tol (outer GMRES on the true residual of the shifted
 * system; the near-field solves use tol/10), restart and max_iter. Synchronises
 * `stream`. Returns SEASD_W_NOT_CONVERGED when the outer solve stopped above
 * tol, SEASD_E_SINGULAR for a singular diagonal block of Rt, and the errors
 * of seasd_mobility_apply. */
int seasd_solve_mixed(seasd_handle handle, int64_t n, const double* pos, const double* radius, const double* box,
                      const seasd_bsr6* rnf, double lambda, const double* fp, const double* einf,
                      double* f, double* s, double* u, seasd_solve_stats* stats, void* stream);

/* Far-field Brownian force moments (Sec. 4.3, eq. br-f-ff): x = M^(-1/2) psi
 * on the 11 incompressible components (force, torque, stresslet), computed
 * with the initial value problem of eq. ivp-1,
 *   dx/dtau = -(1/2) [tau I + (1 - tau) A]^-1 (A - I) x,  x(0) = psi,
 * whose value at tau = 1 is A^(-1/2) psi, marched in K = round(1/dtau) steps
 * of a forward Euler half step (eq. ivp-forward) and a backward Euler half
 * step (eq. ivp-backward); every linear system (alpha I + beta A) is solved
 * by the GMRES of seasd_solve_farfield (tolerance tol, restart, max_iter
 * per solve) with the shifted block-diagonal preconditioner (alpha I +
 * beta A_ii)^-1. A = s M is the mobility made dimensionless with the Stokes
 * drag of the smallest sphere, s = 6 pi eta a_min, and x = sqrt(s) A^(-1/2) psi.
 * The caller multiplies by sqrt(2 kT / dt) for the force moments of a
 * time step.
 *   psi    device [n][12] unit Gaussian noise (trace column ignored)
 *   x      device [n][12] output (trace column 0); may not alias psi
 *   dtau   IVP step, 0 < dtau <= 1 (the paper uses 0.1)
 *   stats  host, may be NULL
 * Synchronises. Returns SEASD_W_NOT_CONVERGED if a linear solve stopped at
 * max_iter, and the errors of seasd_solve_farfield. */
typedef struct seasd_brownian_stats {
    int32_t steps;           /* IVP steps K                                      */
    int32_t solves;          /* shifted linear solves (2 K)                      */
    int32_t iterations;      /* GMRES iterations over all solves                 */
    int32_t matvecs;         /* products with M                                  */
    int32_t converged;       /* 1 if every solve met tol                         */
    double  max_residual;    /* largest final true residual of the solves        */
    double  scale;           /* s = 6 pi eta a_min                               */
    double  solve_ms;        /* wall time of the call                            */
} seasd_brownian_stats;

int seasd_brownian_farfield(seasd_handle handle, int64_t n, const double* pos, const double* radius,
                            const double* box, const double* psi, double* x, double dtau,
                            seasd_brownian_stats* stats, void* stream);

/* Per-phase timing of mobility products, recorded with HIP events on each
 * call's stream while enabled (off by default; one event per phase, no
 * synchronisation). Phases, in order: bin, pair, window, spread, fft_x_fwd,
 * fft_y_fwd, fft_z_scale, fft_y_inv, fft_x_inv, gather (window: the
 * per-sphere window records; spread: the spreading kernel alone).
 * seasd_profile_enable(h, 1) starts a new recording (also discarding any
 * unread one); seasd_profile_read synchronises the stream of the last
 * product, writes the average duration in ms of each phase over the products
 * recorded since then into ms[0..9], the number of those products into ms[10]
 * (when count > 10), starts a new recording and returns the number of phases
 * (10), or a negative error. */
int seasd_profile_enable(seasd_handle handle, int32_t enable);
int seasd_profile_read(seasd_handle handle, double* ms, int32_t count);

/* ---- many independent suspensions -------------------------------------------
 * Autotuner: parameters for one suspension of n spheres (radii a_min..a_max)
 * in the cell `box` (host [9], accepted shapes as above), aiming at a global
 * relative error of `target` (1e-6 or looser) in the given precision. It
 * picks the grid M (a power of two, 32..256: for targets of 1e-6 or looser
 * the finest with spacing h >= 0.21 a_max across the thinnest direction of
 * the cell, below which the window's Faxen terms lose accuracy; for tighter
 * targets the spacing nearest 0.4 a_max), xi from the grid spacing so that
 * the k-space tail exp(-k_max^2/(4 xi^2)) stays fixed, the real-space
 * cut-off factor so that xi r_c is fixed for a pair of spheres of radius
 * a_min (the batch planner passes the 10th-percentile radius, and the
 * 99th-percentile radius as a_max), and the window (P, m) from accuracy
 * scans of the method against the oracle (Sec. 5.1). SEASD_MIXED takes the
 * FP64 choices (its products outside solve steps are FP64).
 * Other fields take the defaults. */
int seasd_autotune(int64_t n, const double* box, double a_min, double a_max, double target, int32_t precision,
                   seasd_config* cfg);

typedef struct seasd_batch_s* seasd_batch;

/* Plan for nsys independent suspensions, all sphere arrays
 * concatenated: suspension k owns spheres offsets[k] .. offsets[k+1]-1.
 *   offsets  host [nsys+1], offsets[0] = 0, increasing
 *   pos      device [N][3], radius device [N] (N = offsets[nsys]); read during
 *            this call only (the plan keeps binned copies)
 *   boxes    host [nsys][9] lattice vectors (accepted shapes as above)
 *   per_sys  host [nsys] configurations, or NULL to autotune each suspension
 *            for `target` with the handle's precision
 * Builds every suspension's geometry (binning, neighbour lists) and captures
 * the product phases of all of them into one hipGraph (suspensions spread
 * over 8 streams that fork from and join `stream`). Synchronises `stream`.
 * The plan holds its own workspace; destroy it with seasd_batch_destroy. */
int seasd_batch_create(seasd_handle handle, int32_t nsys, const int64_t* offsets, const double* pos,
                       const double* radius, const double* boxes, const seasd_config* per_sys, double target,
                       seasd_batch* plan, void* stream);

/* y = M x for every suspension of the plan with one graph launch on `stream`:
 * x, y device [N][12] (concatenated like the positions). Asynchronous. */
int seasd_batch_apply(seasd_batch plan, const double* x, double* y, void* stream);

/* Per-suspension configuration chosen for the plan (host out[nsys]). */
int seasd_batch_configs(seasd_batch plan, seasd_config* out);

int seasd_batch_destroy(seasd_batch plan);

/* One-shot batched product: create a plan, apply it once, destroy it. */
int seasd_mobility_apply_batched(seasd_handle handle, int32_t nsys, const int64_t* offsets,
                                 const double* pos, const double* radius, const double* boxes,
                                 const seasd_config* per_sys, const double* x, double* y, void* stream);

/* ---- learned preconditioner (not in the paper) ------------------------------
 * A two-layer message-passing network on the neighbour graph (edges between
 * spheres closer than 2 (a_i + a_j)) that works on top of the block-diagonal
 * preconditioner of Sec. 4.2. For every sphere it predicts three
 * log-scalings o_i (force, torque, stresslet groups) that turn the inverse
 * block B_i into S_i B_i S_i, S_i = diag(exp(o_i / 2)); for every edge it
 * predicts 15 coefficients of the rotation-covariant 11x11 maps that a pair
 * direction allows, giving the initial guess
 *   x0_i = S_i B_i S_i b_i + sum_j sigma_i * Q(c_ij, u_ij) (sigma_j * b_j),
 * sigma = sqrt(diag B). Node features: degree, neighbour crowding, size
 * ratios; edge features: r/(a_i+a_j), its inverse powers, log(a_j/a_i),
 * a_j/(a_i+a_j). Hidden width 64. Dense layers run on the matrix cores with
 * BF16 operands and FP32 accumulation; the initial guess and the rescaled
 * blocks are FP64. Training minimises the relative residual of the guess,
 * ||b' - A x0||^2 / ||b'||^2, over far-field problems (configuration and
 * right-hand side), with the method's own product supplying A.
 * A network object lives on one device; it holds FP32 master weights, their
 * BF16 copies, the Adam moments and the activations of the last
 * configuration it saw. Not thread safe. */
typedef struct seasd_net_s* seasd_net;

/* Create a network on `device` with random weights from `seed` (uniform
 * He-style ranges, zero biases, output layers scaled by 0.01 so that a fresh
 * network reproduces the block-diagonal preconditioner closely). */
int seasd_net_create(seasd_net* net, int32_t device, uint64_t seed);
int seasd_net_destroy(seasd_net net);

/* Number of FP32 parameters (the flat layout: W_in[16][64], b_in[64], then
 * per layer W_uv[64][128], W_e[16][64], b_a[64], W_m[64][64], b_m[64],
 * W_h[128][64], b_h[64], then W_o[64][16], b_o[16], W_c[64][16], b_c[16];
 * weights row-major as [fan_in][fan_out]). */
int64_t seasd_net_param_count(void);

/* Copy the FP32 master weights to / from a host array of exactly
 * seasd_net_param_count() floats (set also refreshes the BF16 copies). */
int seasd_net_get_params(seasd_net net, float* host, int64_t count);
int seasd_net_set_params(seasd_net net, const float* host, int64_t count);

/* Weights file: magic "SEASDNET", version 1, parameter count, Adam step, FP32
 * weights and both Adam moments, FNV-1a 64-bit checksum of all preceding
 * bytes. load returns SEASD_E_FORMAT for a missing, truncated, mismatched or
 * corrupt file and leaves the network unchanged. */
int seasd_net_save(seasd_net net, const char* path);
int seasd_net_load(seasd_net net, const char* path);

/* One configuration and 1 <= nrhs <= 4096 right-hand sides:
 *   b      device [nrhs][n][12] right-hand sides (trace component ignored)
 *   x0     device [nrhs][n][12] initial guesses out (trace 0), or NULL
 *   loss   host, or NULL: the training loss, the mean over right-hand sides
 *          of ||b' - A x0||^2 / ||b'||^2, with b' the incompressible
 *          components of b and A the 11x11 incompressible block of M
 *          applied by this library's own product (the handle's
 *          configuration); the relative residual is what GMRES reduces
 *   grad   host [seasd_net_param_count()] gradient of the loss, or NULL
 * The gradient with respect to x0 is -2 A (b' - A x0) / (nrhs ||b'||^2), so
 * each right-hand side costs two products when loss or grad is asked for.
 * The block-diagonal blocks are built as in seasd_solve_farfield.
 * Synchronises. Errors as seasd_solve_farfield, and SEASD_E_CUTOFF when
 * 8 a_max >= L (edge cut-off beyond half the cell). */
int seasd_net_loss_grad(seasd_handle handle, seasd_net net, int64_t n, const double* pos, const double* radius,
                        const double* box, int32_t nrhs, const double* b, double* x0, double* loss, float* grad,
                        void* stream);

/* Loss and gradient as above followed by one Adam step (beta 0.9 / 0.999,
 * eps 1e-8, learning rate lr) on the device. */
int seasd_net_train_step(seasd_handle handle, seasd_net net, int64_t n, const double* pos, const double* radius,
                         const double* box, int32_t nrhs, const double* b, float lr, double* loss, void* stream);

/* Attach a network for solves with precond = SEASD_PRECOND_LEARNED_GUESS
 * (NULL detaches; the handle does not own it). Such a solve builds the
 * graph, runs the network once and starts GMRES from the network's x0
 * (overwriting the caller's guess), preconditioned by the block-diagonal
 * blocks. It falls
 * back to the block-diagonal blocks and a zero guess, and returns
 * SEASD_W_PRECOND_FALLBACK if the solve otherwise converged, when an output
 * is non-finite or a scaling is beyond e^8. The true residual judges the
 * guess: GMRES starts from alpha x0 with alpha = argmin ||b' - alpha A x0||
 * (one product), so the starting residual never exceeds ||b'||; alpha <= 0
 * drops the guess (guess_used = 0). */
int seasd_precond_attach(seasd_handle handle, seasd_net net);

/* Load a weights file into a network owned by the handle and attach it. */
int seasd_precond_load(seasd_handle handle, const char* path);

/* Short description of a return code (static storage). */
const char* seasd_error_string(int32_t code);

#ifdef __cplusplus
}
#endif

#endif /* SEASD_H */
