/*
 * pfnks.h -- C ABI of the MI355X Newton-Krylov-Schwarz solver for one time step of the
 * discrete-variational-derivative (DVD) scheme of Huang & Yang, "Parallel energy stable
 * phase field simulations of Ni-based alloys system".
 *
 * The library advances the composition c, the three long-range order parameters eta_1..3
 * and the displacement u_1..u_d on a periodic d-dimensional grid (d = 2 or 3) by one step
 * of scheme (NSOA-1) (Section 3): the semi-implicit DVD update of (c, eta) together with the
 * discrete mechanical equilibrium (mechanicalequilibrium-dis), solved by inexact Newton with
 * right-preconditioned restarted GMRES and a restricted additive Schwarz (RAS) preconditioner
 * (Section 4).  Free energy: Appendix A (sublattice chemical energy with the logarithmic
 * terms, cubic elastic energy); discrete gradient: Section 3 eqs. (D2-1), (dvds-1) and
 * Appendix B, generalised to three order parameters.
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status (PFNKS_OK = 0 or a negative PFNKS_E* code);
 *     none throws, none keeps global mutable state.  pfnks_strerror() gives the text.
 *   - Arrays handed in by pointer are HOST arrays unless the name starts with d_.  Fields are
 *     structure-of-arrays planes of n[0]*n[1]*n[2] doubles each, x fastest (index
 *     i + n0*(j + n1*k)), in the order c, eta_1, eta_2, eta_3, u_1 .. u_d.
 *   - Device memory: the library never allocates device memory.  The caller allocates the
 *     workspace (pfnks_workspace_bytes) and keeps it alive until pfnks_destroy; the library
 *     allocates only a small pinned host buffer per problem.
 *   - Work is ordered on the HIP stream given at creation (NULL = the null stream).  Every
 *     call that returns host values synchronises that stream.
 *   - Distinct problems may be used from distinct host threads; one problem must not be used
 *     by two threads at once.
 */
#ifndef PFNKS_H
#define PFNKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PFNKS_OK = 0,
  PFNKS_EINVAL = -1,   /* bad argument: null pointer, size, parameter outside its range  */
  PFNKS_EDOMAIN = -2,  /* a state outside the log domain: need 0 < c < 1, 0 < c eta_i < 1  */
  PFNKS_ENOSPACE = -3, /* workspace smaller than pfnks_workspace_bytes                      */
  PFNKS_ENOCONV = -4,  /* Newton did not converge; the state is left at t_n                */
  PFNKS_EDEVICE = -5   /* a HIP runtime error; pfnks_last_error() has its text              */
};

typedef enum { PFNKS_FP64 = 0, PFNKS_MIXED = 1 } pfnks_precision;

/* Preconditioner.  PFNKS_PC_RAS: one-level restricted additive Schwarz over all fields
 * (Section 4, left-RAS z = sum_t R_t^0' A_t^{-1} R_t^delta r), tile solve in LDS.
 * PFNKS_PC_RAS_SPECTRAL: the same RAS over (c, eta) composed block-lower-triangularly with an
 * exact Fourier solve of the constant-coefficient periodic displacement block.
 * PFNKS_PC_NONE: identity (unpreconditioned GMRES; for testing and comparison).
 * PFNKS_PC_SPECTRAL: identity on (c, eta) composed with the same exact displacement solve
 * (isolates the Fourier block for testing).
 * PFNKS_PC_AS: classical additive Schwarz over all fields, z = sum_t R_t^delta' A_t^{-1}
 * R_t^delta r (the extended solutions are summed where tiles overlap; Section 4, the paper's
 * classical-AS runs).  PFNKS_PC_RRAS: right-RAS, z = sum_t R_t^delta' A_t^{-1} R_t^0 r (r
 * restricted to the owned nodes).  Both need overlap <= tile side. */
typedef enum {
  PFNKS_PC_RAS = 0,
  PFNKS_PC_RAS_SPECTRAL = 1,
  PFNKS_PC_NONE = 2,
  PFNKS_PC_SPECTRAL = 3,
  PFNKS_PC_AS = 4,
  PFNKS_PC_RRAS = 5
} pfnks_pc;

typedef struct {
  int dim;      /* 2 or 3                                                     */
  int n[3];     /* nodes per direction (n[2] = 1 when dim == 2): even, >= 4, and
                   products of 2, 3, 5, 7, 11 and 13 (the radices of the Fourier solve) */
  double h;     /* grid spacing; periodic box of side n[k]*h                  */
} pfnks_grid;

/* Dimensionless model parameters (Appendix A; values divided by V_m*DeltaE). */
typedef struct {
  double theta;      /* RT / (V_m DeltaE)                                              */
  double w_c;        /* weight of theta*Psi(c): 1 = the form of Section 2 and (D2-1)    */
  double e0;         /* (E0_Al - E0_Ni)                                                */
  double L[4];       /* Redlich-Kister L0..L3 of the disordered excess energy          */
  double U1, U4;     /* ordering parameters of E^ord                                   */
  double gamma_c;    /* gradient coefficient of c                                      */
  double gamma_eta;  /* gradient coefficient of each eta_p                             */
  double kappa;      /* mobility prefactor, M = kappa c (1 - c)                        */
  double L_eta;      /* relaxation coefficient of eta (1 as written)                   */
  double eps0;       /* lattice misfit per unit composition                            */
  double C11, C12, C44; /* cubic elastic constants                                     */
  double Lscale;     /* multiplier of the Hooke tensor (Section 5.1); 0 = no elasticity */
  int S;             /* order of the Taylor-stabilised quotient Psi_S (Section 3), 1..30 */
} pfnks_model;

typedef struct {
  double newton_rtol;     /* eps_r of the relative residual test ||F|| <= eps_r ||F(X0)||     */
  double newton_atol_rms; /* eps_a per unknown: eps_a = newton_atol_rms * sqrt(#unknowns)     */
  int newton_maxit;       /* Newton iterations before PFNKS_ENOCONV                         */
  double gmres_rtol;      /* xi_r: ||J S + F|| <= max(xi_r ||F||, xi_a)                     */
  double gmres_atol_rms;  /* xi_a per unknown                                               */
  int gmres_restart;      /* Krylov basis size m (1..64)                                    */
  int gmres_maxit;        /* total GMRES iterations per Newton step                         */
  int tile[3];            /* owned tile of the Schwarz preconditioner (tile[2] = 1 in 2D)   */
  int overlap;            /* delta: extra layers of each subdomain on every side (0..4)     */
  int sweeps;             /* symmetric multicolour block Gauss-Seidel sweeps per tile solve */
  double sor_omega;       /* over-relaxation of those sweeps (SSOR), 0 < omega < 2; 1 = GS */
  pfnks_pc pc;            /* preconditioner                                                 */
  pfnks_precision precision; /* PFNKS_FP64, or PFNKS_MIXED (float Krylov basis and preconditioner) */
  double ls_alpha;        /* Armijo constant of the backtracking line search                */
  int ls_max_halvings;    /* halvings of lambda before the step is declared failed          */
  double newton_stol;     /* update test of the Newton stop: besides the residual test, the
                             error left by the last accepted correction, estimated from the
                             contraction theta of consecutive corrections as
                             theta / (1 - theta) max|lambda S_f|, must be <= newton_stol *
                             max|X_f| in every field f (0 = residual test only) */
  int pc_refresh;         /* 0: the preconditioner is built once per time step, at X^n, and
                             reused over the Newton iterations (the reuse of Section 5.4);
                             1: rebuilt at every Newton iteration                         */
} pfnks_solver;

typedef struct {
  int newton_its, gmres_its, ls_backtracks, status;
  double res0;            /* ||F(X^n)||                                 */
  double res_final;       /* ||F(X^{n+1})||                             */
  double dx_rms;          /* RMS of X^{n+1} - X^n over c and eta        */
  double energy;          /* discrete energy E~^{n+1}                   */
  double energy_parts[3]; /* chemical, elastic, interfacial             */
  double mass;            /* <c^{n+1}> = h^d sum c                      */
  double update_rel;      /* the update test's error estimate of the last iteration, relative
                             to max|X_f|, largest over the fields (0 when no iteration ran;
                             infinite after a single iteration, which has no estimate)   */
} pfnks_step_stats;

typedef struct pfnks_problem pfnks_problem;

/* Bytes of device workspace a problem of this shape needs (device memory the caller owns).
 * Errors: PFNKS_EINVAL for a null pointer, dim not 2 or 3, a size that is odd, below 4 or has
 * a prime factor above 13, a tile that does not divide the grid, overlap or restart out of
 * range. */
int pfnks_workspace_bytes(const pfnks_grid* grid, const pfnks_model* model,
                          const pfnks_solver* solver, size_t* bytes);

/* Create a problem from the initial data c^0 and eta^0 (Section 2: initial conditions;
 * periodic boundary conditions).  c0: one host plane; eta0: three host planes, both copied.
 * Computes cbar^0 = mean(c^0) (the reference composition of the eigenstrain, Section 3) and the
 * initial displacement u^0 from the discrete equilibrium (mechanicalequilibrium-dis) at c^0,
 * with zero mean on every parity class (the gauge of the central difference).
 * d_workspace: device buffer of ws_bytes >= pfnks_workspace_bytes(), 256-byte aligned,
 * owned by the caller.  hip_stream: a hipStream_t or NULL.
 * Errors: PFNKS_EINVAL, PFNKS_ENOSPACE, PFNKS_EDOMAIN (some 0 < c, c*eta_i < 1 violated,
 * eta_4 = 4 - eta_1 - eta_2 - eta_3), PFNKS_EDEVICE. */
int pfnks_create_problem(const pfnks_grid* grid, const pfnks_model* model,
                         const pfnks_solver* solver, const double* c0, const double* eta0,
                         void* d_workspace, size_t ws_bytes, void* hip_stream,
                         pfnks_problem** out);

/* One step of scheme (NSOA-1) with step size dt (Section 3), solved by the Newton-Krylov-
 * Schwarz method of Section 4 from X_0 = X^n.  The c-part of every Newton update is
 * projected so that the total mass is exactly that of X^n (Theorem 3.2, item 1).  Newton
 * stops when ||F|| <= eps_a, or when ||F|| <= eps_r ||F(X_0)|| (the relative test of Section
 * 4) and the last accepted correction passes the update test of solver.newton_stol (the
 * residual test alone bounds the distance to the root only through ||J^{-1}||).  On
 * success the state becomes X^{n+1}, t += dt, and stats (may be NULL) is filled.
 * On PFNKS_ENOCONV the state is unchanged (the adaptive driver of Section 4 retries
 * with a smaller dt).  Errors: PFNKS_EINVAL (dt <= 0), PFNKS_ENOCONV, PFNKS_EDEVICE. */
int pfnks_step(pfnks_problem* p, double dt, pfnks_step_stats* stats);

/* One step of each of k independent problems (an ensemble), dts[i] for problem i, run
 * concurrently: host threads (at most `threads`, 0 = min(k, 16)) take problems from a shared
 * counter and call pfnks_step on them, so each problem's kernels go to the stream it was
 * created with; problems on distinct streams overlap on the GPU.  Every problem must appear
 * once (a handle is not used by two threads).  stats (may be NULL) and status (may be NULL)
 * receive k records.  Each problem's result is bitwise the result of pfnks_step on it alone.
 * Returns PFNKS_OK when every step succeeded, else the status of the first failing index
 * (PFNKS_ENOCONV steps leave their problem unchanged, the others advance); when that status is
 * PFNKS_EDEVICE, pfnks_last_error() on the calling thread gives the failing problem's text.
 * Errors: PFNKS_EINVAL (null arrays, k < 0, a handle given twice). */
int pfnks_batch_step(pfnks_problem* const* problems, int k, const double* dts, int threads,
                     pfnks_step_stats* stats, int* status);

/* ---- lockstep problem groups (ensembles of one grid shape) ----------------------------
 * `count` (1 .. 32) problems with one grid, model and solver, stepped together.  Every phase
 * of the step of Section 4 (residual, linearisation, the preconditioner set-up, each Arnoldi
 * step of GMRES with its Schwarz tile solve, Fourier block and J v, the line-search trials,
 * the step close) is one launch per kernel for all instances still working in that phase;
 * the Hessenberg columns, Givens rotations and the triangular solve of each GMRES cycle run
 * on the device, and the host synchronises once per Arnoldi step, residual evaluation and
 * cycle end for all instances together.  Each instance follows the iteration pfnks_step
 * would take on it alone (its own dt, Newton and GMRES counts, line search and stop rule);
 * the results agree with pfnks_step's to rounding (the rotations are computed on the device
 * instead of the host).  An instance's arithmetic does not depend on the other members: its
 * result is bitwise its result in a group of one.
 * The workspace (device, 256-byte aligned, caller-owned, kept alive until
 * pfnks_group_destroy) holds count copies of the single-problem layout, instance i at
 * i * pfnks_workspace_bytes bytes.  c0: count * N doubles, eta0: count * 3 N doubles
 * (instance-major, each as for pfnks_create_problem).  Errors: PFNKS_EINVAL (count outside
 * 1 .. 32, bad configuration, misaligned workspace), PFNKS_ENOSPACE, PFNKS_EDOMAIN,
 * PFNKS_EDEVICE. */
typedef struct pfnks_group pfnks_group;
int pfnks_group_workspace_bytes(const pfnks_grid* grid, const pfnks_model* model,
                                const pfnks_solver* solver, int count, size_t* bytes);
int pfnks_group_create(const pfnks_grid* grid, const pfnks_model* model, const pfnks_solver* solver,
                       int count, const double* c0, const double* eta0, void* d_workspace,
                       size_t ws_bytes, void* hip_stream, pfnks_group** out);
/* One step of every instance, dts[i] for instance i (host array of count); an instance with
 * dts[i] = 0 sits the step out (state unchanged, status PFNKS_OK, zero stats), so that an
 * adaptive driver can retry only the instances that failed.  stats and status (may be NULL)
 * receive count records.  An instance whose step succeeds advances (X^{n+1}, t += dts[i]);
 * one that does not converge keeps its state (status PFNKS_ENOCONV).  Returns PFNKS_OK when
 * every instance succeeded, else the first failing instance's status.
 * Errors: PFNKS_EINVAL (null group or dts, dts[i] < 0 or not finite), PFNKS_EDEVICE. */
int pfnks_group_step(pfnks_group* g, const double* dts, pfnks_step_stats* stats, int* status);
/* Give instance i a new initial state (c0: N doubles, eta0: 3 N, as pfnks_create_problem):
 * its displacement from the elastic equilibrium, its mean composition and t = 0; the other
 * instances are untouched.  A serving loop reuses a freed slot this way.  Synchronises the
 * group's stream.  Errors: PFNKS_EINVAL, PFNKS_EDOMAIN, PFNKS_EDEVICE. */
int pfnks_group_set_instance(pfnks_group* g, int i, const double* c0, const double* eta0);
/* State of instance i to host (4 + dim planes, as pfnks_get_state); t may be NULL. */
int pfnks_group_get_state(pfnks_group* g, int i, double* X, double* t);
/* Kernel launches and host synchronisations of the last pfnks_group_step. */
int pfnks_group_counters(pfnks_group* g, long long* launches, long long* syncs);
/* Release the handle (host memory only; the caller frees the workspace afterwards). */
int pfnks_group_destroy(pfnks_group* g);

/* Discrete free energy E~ of eqs. (relations)/(freeenergy) at the current state; parts
 * (may be NULL) receives (chemical E1+E2, elastic E3, interfacial E4). */
int pfnks_energy(pfnks_problem* p, double* total, double parts[3]);

/* Discrete mass <c> = h^d sum_i c_i (Theorem 3.2). */
int pfnks_mass(pfnks_problem* p, double* mass);

/* Copy the state to host: X receives 4 + dim planes (c, eta_1..3, u_1..u_d); t may be NULL. */
int pfnks_get_state(pfnks_problem* p, double* X, double* t);

/* Replace the state (4 + dim host planes) and time, e.g. to resume from a checkpoint taken
 * with pfnks_get_state.  The displacement is used as given.  Errors: PFNKS_EDOMAIN. */
int pfnks_set_state(pfnks_problem* p, const double* X, double t);

/* Release the handle (host memory only; the caller frees the workspace afterwards). */
int pfnks_destroy(pfnks_problem* p);

const char* pfnks_strerror(int status);
/* Text of the last PFNKS_EDEVICE on this thread. */
const char* pfnks_last_error(void);

/* ---- building blocks of the step, exposed for parity tests (host arrays) ------------ */

/* F(X; X^n, dt), the residual of (NSOA-1) with the current state as X^n.
 * X, F: 4 + dim host planes. */
int pfnks_debug_residual(pfnks_problem* p, const double* X, double dt, double* F);

/* w = J(X) v, the Jacobian of the residual at X (current state as X^n) applied to v.
 * X, v, w: 4 + dim host planes. */
int pfnks_debug_jv(pfnks_problem* p, const double* X, double dt, const double* v, double* w);

/* z = M^{-1} r, the preconditioner built at X (current state as X^n).  r, z: host planes. */
int pfnks_debug_pc(pfnks_problem* p, const double* X, double dt, const double* r, double* z);

/* ---- allocation-free residual ------------------------------------------------------ */

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the residual F(X; X^n, dt) of pfnks_debug_residual,
 * on device arrays and without a problem handle.  Its scratch (the four G planes between the
 * two stencil passes and the reductions' partial sums) is a file-scope device array of the
 * library, 64 MiB + 17 KiB per GPU, held from first use until the process ends; the call
 * allocates nothing (no hipMalloc, no pinned memory, no library allocation).
 * grid, model: as for pfnks_create_problem, at most 2^21 nodes (PFNKS_ENOSPACE beyond).
 * cbar0: the eigenstrain's reference composition (mean of c^0 at creation).
 * d_X, d_Xn: 4 + dim device planes (X, and X^n); d_F: 4 + dim device planes, written.
 * norm, bad (host, may be NULL): ||F||_2 and the count of nodes of X outside the log domain;
 * when either is given the call synchronises the stream, otherwise it only enqueues work on
 * hip_stream (the device of the current context).  Every call on one GPU shares that GPU's
 * scratch: calls that overlap on one GPU (distinct streams or threads) race.
 * Errors: PFNKS_EINVAL, PFNKS_ENOSPACE, PFNKS_EDEVICE. */
int pfnks_residual_static(const pfnks_grid* grid, const pfnks_model* model, double cbar0, double dt,
                          const double* d_X, const double* d_Xn, double* d_F, double* norm, double* bad,
                          void* hip_stream);

/* Counters of the last pfnks_step: kernel launches and host synchronisations. */
int pfnks_debug_counters(pfnks_problem* p, long long* launches, long long* syncs);

/* Live kernel timing.  pfnks_debug_profile(p, mask) clears the totals and brackets every
 * launch of the kernel kinds whose bit (1 << kind) is set in mask with HIP events recorded on
 * the problem's stream (mask 0 switches it off; each bracket costs two event records).  pfnks_debug_kernel_time returns, for one kind, the number of timed launches, their
 * summed GPU duration in milliseconds and their summed algorithmic bytes (the bytes the
 * operation must move: reads of its inputs plus writes of its outputs, once each). */
enum {
  PFNKS_K_RESIDUAL = 0,  /* residual F (two kernels)                    */
  PFNKS_K_LINEARISE = 1, /* local 4 x 4 chemical blocks (and, once per
                            step, the tile solve's node blocks)         */
  PFNKS_K_JV = 2,        /* matrix-free Jacobian apply                  */
  PFNKS_K_RAS = 3,       /* Schwarz tile solve                          */
  PFNKS_K_SPECTRAL = 4,  /* Fourier solve of the displacement block     */
  PFNKS_K_MULTIDOT = 5,  /* GMRES classical Gram-Schmidt dot products   */
  PFNKS_K_UPDATE = 6,    /* GMRES orthogonal update and normalisation   */
  PFNKS_KERNEL_KINDS = 7
};
int pfnks_debug_profile(pfnks_problem* p, int mask);
int pfnks_debug_kernel_time(pfnks_problem* p, int kind, long long* launches, double* ms_total,
                            double* bytes_total);

#ifdef __cplusplus
}
#endif

#endif /* PFNKS_H */
