/* pisoc.h -- C ABI of the MI355X (gfx950) PISO step library.
 *
 * One time step of the fast-Eulerian model of Cerminara et al. (arXiv
 * 1404.0959, Results section): a compressible gas with the barotropic closure
 * p = C rho^gamma (second footnote), advanced by a collocated finite-volume PISO
 * pressure-based scheme with fourth-order central face interpolation and an
 * adaptive time step, carrying K dust classes in the Equilibrium-Eulerian model
 * (particle velocity u_p = u - tau_p Du/Dt, first order in the Stokes number;
 * tau_p = 0 is Marble's dusty gas, third footnote), on the periodic cube
 * [0, 2 pi)^3 with n cells per side (the paper's decaying homogeneous isotropic
 * turbulence setting, Introduction and Fig. 1).
 *
 * Conventions for every entry point:
 *  - Cell arrays hold n^3 doubles at offset i + n*(j + n*k) (x fastest).
 *    Vector fields are structure-of-arrays: component d at offset d*n^3.
 *    Face array d holds, at the offset of cell P, the value on the face
 *    between P and P + e_d.
 *  - Pointers named d_* are device pointers (hipMalloc'd or torch CUDA
 *    tensors); h_* are host pointers.  The caller owns every buffer.  The
 *    library never allocates device memory: all of its scratch lives in the
 *    caller's workspace (see pisoc_workspace_bytes).  It allocates only the
 *    small host context and a few bytes of pinned host memory for status.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as void*,
 *    NULL = default stream).  Calls that return host-visible results
 *    synchronise that stream before returning.
 *  - Errors are status codes; no exception crosses the ABI.  Warnings
 *    (status > 0) still advance the state; errors (status < 0) leave the state
 *    at the last completed step.  pisoc_last_error gives a message.
 */
#ifndef PISOC_H
#define PISOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PISOC_MAX_CLASSES 8
#define PISOC_MAX_CORR 4
#define PISOC_MIN_N 8
#define PISOC_MAX_N 1024

typedef struct pisoc_ctx pisoc_ctx;

typedef enum {
    PISOC_OK = 0,
    PISOC_WARN_NOT_CONVERGED = 1, /* a pressure solve hit p_maxit (state advanced) */
    PISOC_WARN_GUESS_FALLBACK = 2, /* learned guess rejected, zero guess used */
    PISOC_WARN_DUST = 3,           /* PISOC_FLAG_DUST_NEG, _DUST_DIAG or _DUST_COURANT raised
                                      (state advanced) */
    PISOC_ERR_INVALID = -1,        /* bad argument, or dt undefined/non-positive */
    PISOC_ERR_HIP = -2,            /* a HIP runtime call failed */
    PISOC_ERR_DIVERGED = -3,       /* non-finite or non-positive gas density, non-finite
                                      field or dust density; step rejected */
    PISOC_ERR_WORKSPACE = -4       /* workspace missing, too small or misaligned */
} pisoc_status;

/* arithmetic of the step */
enum {
    PISOC_FP64 = 0,         /* every field and operation in FP64 */
    PISOC_FP32_REFINED = 1  /* FP32 fields, stencils and inner CG; FP64 residual
                               refinement of the pressure solve, FP64 reductions */
};

/* initial value of each pressure solve */
enum {
    PISOC_GUESS_ZERO = 0,   /* p' = 0 */
    PISOC_GUESS_LEARNED = 1, /* 3D conv net prediction; 0 where it does not lower ||r|| */
    PISOC_GUESS_PREVIOUS = 2 /* a non-learned rival: the same corrector's solution of the
                                previous step (the first step starts from 0); the same
                                rescaling by alpha = g.b / g.(M g) and the same fallback */
};

/* step-info flag bits */
enum {
    PISOC_FLAG_PCG_MAXIT = 1,
    PISOC_FLAG_NONFINITE = 2,
    PISOC_FLAG_RHO_NONPOS = 4,
    PISOC_FLAG_GUESS_FALLBACK = 8,
    PISOC_FLAG_BAD_DT = 16,
    PISOC_FLAG_GUESS_SKIPPED = 32,
    /* Dust transport of the Equilibrium-Eulerian model (Results section), any
     * class.  The central fourth-order fluxes are not monotone, so a bulk
     * density can undershoot below zero near sharp concentration fronts: */
    PISOC_FLAG_DUST_NEG = 64,       /* some rho_j < 0 after the step (PISOC_WARN_DUST) */
    PISOC_FLAG_DUST_NONFINITE = 128,/* a non-finite rho_j (PISOC_ERR_DIVERGED) */
    /* the diagonal rho^{n+1}/dt + (9/16) div G of the implicit mass-ratio
     * equation is <= 0 in some cell: the drift compresses the dust faster than
     * the equation's Jacobi sweeps can follow (PISOC_WARN_DUST) */
    PISOC_FLAG_DUST_DIAG = 256,
    /* the dust's Courant number (pisoc_step_info.courant_dust) is >= 0.638: for a
     * uniform drift the dust update (its 4 Jacobi sweeps and the conservative
     * finish, the polynomial sum_{l<=5} (-z)^l of the I4 transport symbol z)
     * amplifies some Fourier mode beyond it.  The time step follows the gas's
     * Courant number only; the drift tau_j (g - Du/Dt) raises the dust's
     * (PISOC_WARN_DUST) */
    PISOC_FLAG_DUST_COURANT = 512,
    /* the momentum predictor's BiCGStab (mom_tol > 0) reached mom_maxit first
     * (PISOC_WARN_NOT_CONVERGED) */
    PISOC_FLAG_MOM_MAXIT = 1024
};

typedef struct {
    int32_t n;                 /* cells per side, PISOC_MIN_N..PISOC_MAX_N */
    int32_t n_classes;         /* dust classes, 0..PISOC_MAX_CLASSES */
    double gamma, C, mu;       /* p = C rho^gamma; dynamic viscosity */
    double tau_p[PISOC_MAX_CLASSES]; /* particle response times (>= 0) */
    double cfl;                /* target convective Courant number */
    double dt_growth;          /* dt <= dt_growth * previous dt */
    double dt_fixed;           /* > 0: use this dt every step, else adaptive */
    double dt_max;             /* > 0: upper bound of the adaptive dt */
    int32_t n_corr;            /* PISO correctors, 1..PISOC_MAX_CORR */
    int32_t n_mom_sweeps;      /* Jacobi sweeps of the momentum predictor (>= 1) */
    int32_t n_dust_sweeps;     /* Jacobi sweeps of each dust class (>= 1) */
    double p_tol;              /* stop each pressure solve at ||r||_2 <= p_tol ||b||_2 */
    int32_t p_maxit;           /* CG iteration cap per solve */
    int32_t precision;         /* PISOC_FP64 or PISOC_FP32_REFINED */
    int32_t guess;             /* PISOC_GUESS_ZERO or PISOC_GUESS_LEARNED */
    const void* d_guess_weights; /* learned guess: device pointer to PISOC_NET_NWEIGHTS FP32
                                    weights (layout at pisoc_net_forward); read at init */
    double inner_tol;          /* FP32_REFINED: relative tolerance of each inner FP32 solve */
    int32_t max_refine;        /* FP32_REFINED: cap on FP64 refinement rounds per solve */
    int32_t capture;           /* != 0: keep corrector-1 pressure system of the last step
                                  (b, p', p0, diag, w, and with the learned guess g and
                                  x0) and the predictor's u* for pisoc_fields */
    int32_t guess_audit;       /* learned guess, pisoc_step: 0 = apply it to every solve;
                                  k > 0 = apply it to a corrector's solve only while the CG
                                  iterations it saves (running means of solves with and
                                  without it) exceed its own cost in CG-iteration
                                  equivalents (timed with events), trying the other choice
                                  once after k steps and then at intervals that double, up
                                  to 16 k, while each trial confirms the verdict (back to k
                                  when one overturns it; PISOC_FLAG_GUESS_SKIPPED marks steps
                                  that went without it).  A rejected guess whose cost is at
                                  least the mean iterations of the zero-start solve is not
                                  tried: saving every iteration would not pay for it.  Eager ensemble steps audit the
                                  same way; a captured ensemble step keeps the verdict
                                  its graph was built with (without the periodic trial) */
    int32_t two_way;           /* != 0: two-way coupling.  The momentum equation is the
                                  mixture's: density rho_m = rho + sum_j rho_j, convected by
                                  the gas plus dust mass fluxes (the dust's of the last
                                  step), with the buoyancy (rho_m - <rho_m>) gravity; the
                                  pressure stays the gas's C rho^gamma (Introduction:
                                  buoyancy of the gas-particle mixture; Results: Marble's
                                  dusty gas, third footnote) */
    double gravity[3];         /* g: the dust settles with u_j = u + tau_j (g - Du/Dt); with
                                  two_way the mixture also feels its buoyancy */
    int32_t closure;           /* PISOC_BAROTROPIC (p = C rho^gamma, the step above) or
                                  PISOC_FOURIER (Results, first footnote): the ideal gas
                                  p = rho R_gas T with an energy equation whose heat flux
                                  is q = -kappa grad T.  After the momentum predictor, the
                                  internal energy c_v T is predicted like the momentum
                                  (backward Euler, I4 convection with phi^n, compact
                                  Laplacian for q, n_mom_sweeps Jacobi sweeps from T^n),
                                  with the compression work -p^n div u^n; the correctors
                                  take p0 = rho_k R T* and psi = 1/(R T*), and T* is
                                  T^{n+1}.  FOURIER needs FP64, one grid (no ensemble)
                                  and two_way = 0; C and gamma are then unused */
    double R_gas, cv, kappa;   /* FOURIER: gas constant, c_v, heat conductivity (> 0,
                                  > 0, >= 0) */
    double T0;                 /* FOURIER: initial uniform temperature (> 0); see
                                  pisoc_set_temperature */
    int32_t time_scheme;       /* PISOC_BDF1: backward Euler throughout (the step above);
                                  PISOC_BDF2: variable-step BDF2, d/dt y ~ (c0 y^{n+1} -
                                  c1 y^n + c2 y^{n-1})/dt with w = dt/dt_prev, c0 =
                                  (1+2w)/(1+w), c1 = 1+w, c2 = w^2/(1+w) (backward Euler
                                  on the first step), in the density predictor, the
                                  momentum coefficients and source, the corrector's
                                  defect, compressibility (c0 psi/dt) and density update,
                                  and the dust's acceleration and transport.  BDF2 needs
                                  FP64, the barotropic closure, two_way = 0 and one grid */
    double mom_tol;            /* 0: the momentum predictor is n_mom_sweeps Jacobi sweeps (the
                                  step above).  > 0 (FP64, one grid): the predictor's system
                                  a_P u + N(u) = s - grad p^n, the three components stacked,
                                  is solved from u^n to ||r|| <= mom_tol ||s - grad p^n|| by
                                  BiCGStab (van der Vorst) preconditioned with diag(a_P);
                                  reaching mom_maxit first raises PISOC_FLAG_MOM_MAXIT */
    int32_t mom_maxit;
} pisoc_params;

enum { PISOC_BAROTROPIC = 0, PISOC_FOURIER = 1 };
enum { PISOC_BDF1 = 0, PISOC_BDF2 = 1 };

typedef struct {
    double t, dt, courant;           /* time after the step, dt, sigma*dt */
    int32_t pcg_iters[PISOC_MAX_CORR]; /* CG iterations per corrector (all rounds) */
    double pcg_relres[PISOC_MAX_CORR]; /* final ||r||/||b|| per corrector */
    int32_t refinements[PISOC_MAX_CORR]; /* FP64 refinement rounds (FP32_REFINED) */
    int32_t flags;                   /* PISOC_FLAG_* */
    double mass_gas;                 /* sum rho V after the step */
    double mass_p[PISOC_MAX_CLASSES];/* sum rho_j V after the step */
    double courant_dust;             /* max over the classes of sigma_j dt, sigma_j =
                                        max_P sum_f |G_f| / (2 rho^{n+1} V) with G the
                                        class's mass flux per unit mass ratio */
    int32_t mom_iters;               /* BiCGStab iterations of the momentum predictor
                                        (mom_tol > 0; else 0) */
    double mom_relres;               /* its final ||r|| / ||s - grad p^n|| */
} pisoc_step_info;

typedef struct {
    double ke;        /* <rho |u|^2 / 2> */
    double enstrophy; /* <|curl u|^2 / 2>, Gauss-I4 derivatives */
    double rho_rms;   /* sqrt(<(rho - <rho>)^2>) / <rho> */
    double mach_rms;  /* sqrt(<|u|^2>) / c0, c0^2 = gamma C <rho>^(gamma-1) */
    double mass_gas;  /* sum rho V */
    double conc_var[PISOC_MAX_CLASSES]; /* <(rho_j / <rho_j> - 1)^2> */
    double mass_p[PISOC_MAX_CLASSES];   /* sum rho_j V */
} pisoc_stats;

/* field selectors for pisoc_fields (bit mask) */
enum {
    PISOC_FIELD_RHO = 1u << 0,      /* n^3 */
    PISOC_FIELD_U = 1u << 1,        /* 3 n^3 */
    PISOC_FIELD_PHI = 1u << 2,      /* 3 n^3 face mass fluxes */
    PISOC_FIELD_RHO_P = 1u << 3,    /* n_classes n^3 */
    PISOC_FIELD_P = 1u << 4,        /* n^3, C rho^gamma (PISOC_FOURIER: rho R_gas T) */
    PISOC_FIELD_PSOLVE_B = 1u << 5, /* captured: right-hand side b (needs capture) */
    PISOC_FIELD_PSOLVE_X = 1u << 6, /* captured: solution p' */
    PISOC_FIELD_P_PREV = 1u << 7,   /* captured: p(rho) at the corrector's start */
    PISOC_FIELD_PSOLVE_DIAG = 1u << 8, /* captured: diagonal of the pressure operator */
    PISOC_FIELD_USTAR = 1u << 9,    /* captured: 3 n^3, the momentum predictor's output u* */
    PISOC_FIELD_GUESS = 1u << 10,   /* captured, learned guess: the network's guess g of
                                       corrector 1's solve (s1 times its output) */
    PISOC_FIELD_GUESS_X0 = 1u << 11,/* captured, learned guess: that solve's start x0 =
                                       alpha g, alpha = g.b / g.(M g), or 0 on a fallback */
    PISOC_FIELD_PSOLVE_W = 1u << 12,/* captured: w = rho/a_P, whose I4 face values are the
                                       operator's K_f (with diag, M is then known:
                                       psi/dt = diag - (1/h^2) sum_f K_f) */
    PISOC_FIELD_PSOLVE_PSIDT = 1u << 13,/* captured: that psi/dt, formed from the captured
                                           diag and w (for pisoc_helm_solve) */
    PISOC_FIELD_T = 1u << 14        /* n^3, temperature (PISOC_FOURIER only) */
};

/* Bytes of device workspace pisoc_init needs for these parameters (0 if the
 * parameters are invalid).  The workspace must be 256-byte aligned. */
size_t pisoc_workspace_bytes(const pisoc_params* prm);

/* Set up one simulation of the paper's problem statement (Introduction: freely
 * decaying homogeneous isotropic turbulence in the subsonic regime; Results:
 * barotropic closure p = C rho^gamma of the second footnote, dust classes of
 * the Equilibrium-Eulerian model with response times tau_p from the Stokes
 * law): validate prm, lay out the workspace, convert the initial state and
 * compute the initial face mass fluxes phi = I4(rho) I4(u_d) A with the
 * fourth-order central interpolation I4 of the Results section.
 * d_rho: n^3 FP64, d_u: 3 n^3 FP64 (SoA), d_rho_p: n_classes n^3 FP64 dust bulk
 * densities (may be NULL when n_classes = 0).  The inputs are copied; the
 * caller may free them afterwards.  On success *out receives a context that
 * stays bound to d_workspace and hip_stream until pisoc_destroy. */
pisoc_status pisoc_init(const pisoc_params* prm, void* d_workspace, size_t ws_bytes,
                        const double* d_rho, const double* d_u, const double* d_rho_p,
                        void* hip_stream, pisoc_ctx** out);

/* Advance n_steps time steps of the Results section's scheme: the PISO
 * pressure-based step (adaptive time step, density predictor, momentum
 * predictor, n_corr pressure correctors with fourth-order central
 * interpolation), then each dust class transported with the Equilibrium-
 * Eulerian particle velocity u_p = u - tau_p Du/Dt (first order in the Stokes
 * number; tau_p = 0 is the dusty gas of the third footnote).  h_info (host, may
 * be NULL) receives one record per completed step.  Synchronises the stream before returning.  On an error
 * the state stays at the last completed step and the number of completed steps
 * is available from pisoc_steps_done. */
pisoc_status pisoc_step(pisoc_ctx* ctx, int32_t n_steps, pisoc_step_info* h_info);

/* Copy selected fields of the current state out as FP64: the gas density,
 * velocity and face mass fluxes, the dust bulk densities and the barotropic
 * pressure C rho^gamma (second footnote of the Results section), and, with
 * params.capture, corrector 1's pressure system of the last step.  One
 * destination per set bit of `which`, in increasing bit order (d_dst[0] for
 * the lowest set bit), each sized as its selector states.  Asynchronous. */
pisoc_status pisoc_fields(pisoc_ctx* ctx, uint32_t which, double* const* d_dst);

/* PISOC_FOURIER: replace the temperature field of the current state (n^3 FP64
 * device array, > 0) -- e.g. a non-uniform initial temperature before the
 * first step.  PISOC_ERR_INVALID for the barotropic closure.  Synchronises. */
pisoc_status pisoc_set_temperature(pisoc_ctx* ctx, const double* d_T);

/* Volume statistics of the current state (FP64 reductions; synchronises). */
pisoc_status pisoc_get_stats(pisoc_ctx* ctx, pisoc_stats* h_out);

/* Simulated time and completed steps since init. */
double pisoc_time(const pisoc_ctx* ctx);
int64_t pisoc_steps_done(const pisoc_ctx* ctx);

void pisoc_destroy(pisoc_ctx* ctx);
const char* pisoc_last_error(const pisoc_ctx* ctx);
const char* pisoc_status_string(pisoc_status st);

/* ---- per-kernel timing ----------------------------------------------------
 * When enabled, every kernel launch of pisoc_step is bracketed by HIP events
 * on the context's stream and attributed to its kernel class, together with
 * its algorithmic HBM bytes (each field word the kernel must read or write
 * once).  The back-to-back CG launches issued between two host waits of a
 * solve are bracketed together instead, and their time goes to the working
 * ones: CG launches that return at once because the solve has converged are
 * not counted as launches (their few microseconds stay in the time).  The
 * events are timing-only (no system-scope fence).  Enabling resets the
 * counters. */
#define PISOC_MAX_KSTATS 24
typedef struct {
    char name[32];
    int64_t launches;
    double ms;     /* summed event time of the counted launches */
    double bytes;  /* summed algorithmic bytes of the counted launches */
} pisoc_kernel_stat;

pisoc_status pisoc_profile(pisoc_ctx* ctx, int32_t enable);
/* Copies up to max entries (classes with launches > 0); returns the count. */
int32_t pisoc_profile_read(const pisoc_ctx* ctx, pisoc_kernel_stat* h_out, int32_t max);

/* ---- ensembles -------------------------------------------------------------
 * Independent realisations stepped together: members of the same grid size form
 * a size class whose kernels cover all its members in one launch (members
 * stacked along z, each with its own dt, reference state, particle response
 * times and pressure-solve state), and the classes run as parallel branches.
 * Members may differ in n, C (hence the Mach number) and tau_p; every other
 * parameter must be equal.  The ensemble creates and owns its HIP streams; the
 * calls that step or read it synchronise them.
 *
 * PISOC_ENS_EAGER steps like pisoc_step, per class.  PISOC_ENS_GRAPH replays
 * one captured HIP graph per step for each size class, on the class's stream
 * (the classes' replays overlap): each pressure solve
 * runs a fixed number of CG iterations (sized from the iterations the members
 * needed, +25% + 2) of which every launch after a member's own convergence
 * returns at once, the FP32 refinement runs a fixed number of rounds, and the
 * step is committed on the device.  The first captured call begins with one
 * eager step that measures those iterations (two where a class audits its
 * learned guess and has not yet measured both choices; a call too short for
 * them returns before capturing, and the next one goes on).  The caps follow
 * the iterations the members need (they grow as the flow decays): when a call
 * ends with a solve within 10 % + 2 iterations of the caps its graph holds,
 * the graphs are captured again at once with the new caps.  A solve that reaches
 * its cap without converging flags PISOC_FLAG_PCG_MAXIT (status
 * PISOC_WARN_NOT_CONVERGED, the state has advanced); the caps then grow by
 * half and the graphs are captured again at once.  A diverged member cannot be
 * rolled back in this mode (PISOC_ERR_DIVERGED after the fact). */
typedef struct pisoc_ens pisoc_ens;

/* PISOC_ENS_GRAPH_ONE is PISOC_ENS_GRAPH with one graph for the whole ensemble:
 * every size class's step is a branch of it (forked from and joined into the
 * first class's stream), so a step is one graph launch.  Calls of the two
 * captured modes may alternate; each drops the other's graphs and captures
 * its own (after one eager step). */
enum { PISOC_ENS_EAGER = 0, PISOC_ENS_GRAPH = 1, PISOC_ENS_GRAPH_ONE = 2 };

typedef struct {
    int32_t n, members;                 /* grid size, members of the class */
    int32_t block_x, block_y, cells_z;  /* launch shape of the field kernels */
    int32_t blocks;                     /* blocks per launch (all members) */
    int32_t caps[PISOC_MAX_CORR];       /* captured step: CG iterations of each first solve */
    int32_t cap_later;                  /* ... of each later refinement round */
    int32_t rounds;                     /* ... FP64 refinement rounds (FP32_REFINED) */
    int32_t guess_mask;                 /* ... bit c set: corrector c's solve starts from
                                           the learned guess */
    int32_t cg_cells_z;                 /* planes per block of the CG kernel's z-march
                                           (0: its gathered form) */
    int32_t tiled_cells_z;              /* ... of the other tiled z-marches (0: none) */
} pisoc_ens_class;

/* Workspace for the ensemble (0 if the members are invalid); 256-byte aligned. */
size_t pisoc_ens_workspace_bytes(const pisoc_params* h_members, int32_t count);

/* The batch initialisation: as pisoc_init (the same problem statement of the
 * Introduction and Results section, one independent realisation per member)
 * for `count` members: h_members[m] their parameters, and host arrays of
 * device pointers d_rho[m], d_u[m], d_rho_p[m] (d_rho_p may be NULL without
 * dust).  The set-up waits for work already on hip_stream.  Errors as
 * pisoc_init; on an error no ensemble is created. */
pisoc_status pisoc_ens_init(const pisoc_params* h_members, int32_t count, void* d_workspace,
                            size_t ws_bytes, const double* const* d_rho, const double* const* d_u,
                            const double* const* d_rho_p, void* hip_stream, pisoc_ens** out);

/* Advance every member n_steps steps (mode PISOC_ENS_EAGER or PISOC_ENS_GRAPH).
 * h_info (host, may be NULL) receives `count` records: each member's last step,
 * with flags accumulated over the call.  Synchronises. */
pisoc_status pisoc_ens_step(pisoc_ens* ens, int32_t n_steps, int32_t mode, pisoc_step_info* h_info);

/* As pisoc_fields for member m (asynchronous on the member's class stream;
 * pisoc_ens_time or pisoc_ens_get_stats synchronise). */
pisoc_status pisoc_ens_fields(pisoc_ens* ens, int32_t m, uint32_t which, double* const* d_dst);

/* Statistics of every member into h_out[count]; synchronises. */
pisoc_status pisoc_ens_get_stats(pisoc_ens* ens, pisoc_stats* h_out);

/* Simulated time of every member into h_t[count]; synchronises. */
pisoc_status pisoc_ens_time(pisoc_ens* ens, double* h_t);

int64_t pisoc_ens_steps_done(const pisoc_ens* ens);
int32_t pisoc_ens_num_classes(const pisoc_ens* ens);
pisoc_status pisoc_ens_class_info(const pisoc_ens* ens, int32_t cls, pisoc_ens_class* h_out);

/* Launch-shape autotuner: for every size class, times each candidate shape of
 * the field kernels (block bx x 256/bx threads, cz cells per thread along z,
 * at most 4096 blocks per member) on a representative set of the step's
 * kernels -- a predictor sweep, H/A, the corrector set-up, twelve CG
 * iterations and a dust sweep -- run on the systems of the last step, and
 * keeps the fastest; then, with that shape, the planes per block of the
 * tiled z-marches and of the CG kernel's (each its default, 8, 16 or 32) where
 * they run on tiles.  Winners are cached in the JSON file cache_path (may be
 * NULL) as [bx, cz, CG planes, tile planes (0: none)] under a key of grid
 * size, members, precision, dust
 * classes and guess; a cached entry is used without timing unless force != 0.
 * Needs one completed step.  Synchronises; the captured graph is rebuilt on
 * the next call. */
pisoc_status pisoc_ens_autotune(pisoc_ens* ens, const char* cache_path, int32_t force);

void pisoc_ens_destroy(pisoc_ens* ens);
const char* pisoc_ens_last_error(const pisoc_ens* ens);

/* ---- the pressure (Helmholtz) equation on its own -------------------------
 * The operator of each PISO corrector (Results section: PISO with fourth-order
 * central interpolation):
 *   (M x)_P = psidt_P x_P + (1/h^2) sum_{faces f of P} K_f (x_P - x_nb(f)),
 *   K_f = I4(w) on face f,  h = 2 pi / n,
 * with cell fields psidt = psi/dt > 0 and w = rho/a_P > 0.  M is symmetric
 * positive definite when every K_f > 0. */

/* y = M x.  All arrays n^3 FP64 on the device.  Asynchronous. */
pisoc_status pisoc_helm_apply(int32_t n, const double* d_psidt, const double* d_w,
                              const double* d_x, double* d_y, void* hip_stream);

/* Workspace for pisoc_helm_solve. */
size_t pisoc_helm_workspace_bytes(int32_t n);

/* Jacobi-preconditioned CG on M x = b from the x passed in (d_x is input and
 * output).  Stops when ||r||_2 <= tol ||b||_2 or after maxit iterations
 * (PISOC_WARN_NOT_CONVERGED).  *iters and *relres (host) receive the count
 * and ||r||/||b||.  Synchronises. */
pisoc_status pisoc_helm_solve(int32_t n, const double* d_psidt, const double* d_w,
                              const double* d_b, double* d_x, double tol, int32_t maxit,
                              void* d_workspace, size_t ws_bytes, void* hip_stream,
                              int32_t* iters, double* relres);

/* Preconditioners of pisoc_helm_solve_precond. */
enum {
    PISOC_PRECOND_JACOBI = 0, /* z = D^-1 r, D = diag(M): the solve of the step */
    PISOC_PRECOND_CHEB = 1    /* z = p(D^-1 M) D^-1 r, a degree-1 Chebyshev polynomial */
};

/* pisoc_helm_solve with a choice of preconditioner: a non-learned rival of the
 * learned initial guess (not in the paper).  PISOC_PRECOND_CHEB: the spectrum
 * of D^-1 M lies in [a, 2 - a], a = min psidt/diag (Gershgorin); p is the
 * degree-1 polynomial whose residual 1 - lambda p(lambda) is the degree-2
 * Chebyshev polynomial of that interval normalised to 1 at 0 (positive on the
 * interval, so the preconditioner is symmetric positive definite).  Each
 * iteration applies M twice (two launches).  Arguments, stopping rule,
 * workspace and results as pisoc_helm_solve; another precond value is
 * PISOC_ERR_INVALID.  Synchronises. */
pisoc_status pisoc_helm_solve_precond(int32_t n, const double* d_psidt, const double* d_w,
                                      const double* d_b, double* d_x, double tol, int32_t maxit,
                                      int32_t precond, void* d_workspace, size_t ws_bytes,
                                      void* hip_stream, int32_t* iters, double* relres);

/* The pressure solve of pisoc_helm_solve for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same kernels and results, but the scratch comes
 * from a file-scope device array of PISOC_HELM_NOALLOC_BYTES that each GPU the
 * library runs on holds until the process ends, not from a caller's
 * workspace.  The call allocates nothing (no hipMalloc, hipFree, pinned host
 * buffer or allocating library routine); its first call on a device takes the
 * array's address there.  n <= PISOC_HELM_NOALLOC_MAX_N, else
 * PISOC_ERR_WORKSPACE with no work done.  Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one GPU (other host threads, or
 * other streams) race and must not be made; sequential calls are
 * independent.  Arguments, results and the other errors as pisoc_helm_solve;
 * synchronises. */
#define PISOC_HELM_NOALLOC_MAX_N 64
#define PISOC_HELM_NOALLOC_BYTES (20u << 20)
pisoc_status pisoc_helm_solve_noalloc(int32_t n, const double* d_psidt, const double* d_w,
                                      const double* d_b, double* d_x, double tol, int32_t maxit,
                                      void* hip_stream, int32_t* iters, double* relres);

/* ---- diagnostics of the flow ----------------------------------------------
 * The paper's validation quantities (Results section: the energy spectrum, the
 * kinetic energy and enstrophy, the Taylor micro-scale; third figure: iso-
 * surfaces of the second invariant Q of the velocity gradient), for a velocity
 * field d_u (3 n^3 FP64, SoA, as pisoc_fields returns it).
 *
 * Spectrum: u_hat(k) = DFT(u)(k) / n^3 over the integer wavevectors with
 * components in [-n/2, n/2); shell s holds the k with s - 1/2 <= |k| < s + 1/2;
 * E(s) = sum over the shell of |u_hat(k)|^2 / 2, so sum_s E(s) = <|u|^2> / 2.
 * Taylor micro-scale: lambda = sqrt(5 sum_k |u_hat|^2/2 / D) with
 * D = sum_k |k|^2 |u_hat(k)|^2 / 2 (the isotropic lambda^2 = 15 nu u'^2 / eps,
 * u'^2 = (2/3) sum E, eps = 2 nu D).  n must be a power of two (8..1024).
 * Q = (|Omega|^2 - |S|^2)/2 = -(1/2) sum_ij (d_j u_i)(d_i u_j) per cell, with
 * the Gauss-I4 derivatives of the enstrophy statistic. */

/* Shells of the spectrum of an n^3 grid (0 if n is not supported). */
int32_t pisoc_diag_spectrum_bins(int32_t n);
/* Device workspace of pisoc_diag_spectrum and pisoc_diag_qcrit (256-byte aligned). */
size_t pisoc_diag_workspace_bytes(int32_t n);
/* E(s) for s = 0..nbins-1 into h_E (host), nbins = pisoc_diag_spectrum_bins(n);
 * h_taylor, h_dsum (host, may be NULL): lambda and D.  Synchronises. */
pisoc_status pisoc_diag_spectrum(int32_t n, const double* d_u, double* h_E, int32_t nbins,
                                 double* h_taylor, double* h_dsum, void* d_ws, size_t ws_bytes,
                                 void* hip_stream);
/* Q into d_q (n^3 FP64, device).  h_means (host, may be NULL): <Q> and
 * <(div u)^2> (Gauss-I4), then the call synchronises; else asynchronous. */
pisoc_status pisoc_diag_qcrit(int32_t n, const double* d_u, double* d_q, double* h_means,
                              void* d_ws, size_t ws_bytes, void* hip_stream);
/* Filtered (a-priori sub-grid) statistics, the use the Results section plans
 * for the DNS data base: with the separable top-hat filter of width 2h
 * (weights 1/4, 1/2, 1/4 along each axis; transfer prod_d (1 + cos k_d h)/2),
 * u_bar = bar(u), tau_ij = bar(u_i u_j) - u_bar_i u_bar_j,
 * S_bar_ij = (d_j u_bar_i + d_i u_bar_j)/2 (Gauss-I4), Pi = -tau_ij S_bar_ij:
 * h_out[4] (host) = <|u_bar|^2>/2, <tau_ii/2>, <Pi>, fraction of cells with
 * Pi < 0 (backscatter).  Synchronises. */
pisoc_status pisoc_diag_sgs(int32_t n, const double* d_u, double* h_out, void* d_ws,
                            size_t ws_bytes, void* hip_stream);

/* ---- measurement ------------------------------------------------------------
 * Not in the paper: the practical HBM ceiling of a mix of reads and writes,
 * against which the step's memory-bound kernels are read.  A plain streaming
 * kernel computes out_w[i] = (w + 1) * (in_0[i] + ... + in_{reads-1}[i]) in
 * FP32 for w < writes and i < count, walking the arrays in 16-byte vectors
 * with a grid stride and non-temporal loads and stores, in `blocks` blocks of
 * 256 threads (0: 16384).  h_in[reads], h_out[writes]: host arrays of device
 * pointers, each 16-byte aligned, count floats each; outputs must not
 * overlap inputs.  1 <= reads <= 12, 1 <= writes <= 8, count a multiple of 4.
 * count 0 does nothing (the pointers are not read).  Asynchronous on
 * hip_stream.  Errors: PISOC_ERR_INVALID (before any GPU work) for arguments
 * outside these ranges or a NULL or misaligned pointer; PISOC_ERR_HIP when
 * the launch fails. */
pisoc_status pisoc_stream_probe(int32_t reads, int32_t writes, int64_t count,
                                const float* const* h_in, float* const* h_out, int32_t blocks,
                                void* hip_stream);

/* ---- learned initial guess of the pressure correction --------------------
 * Not in the paper: a small network predicts the start of each pressure solve
 * from the corrector's Jacobi-scaled continuity defect and the pressure of the
 * current density iterate; CG then runs to the same ||r|| <= p_tol ||b|| as
 * without it, so the guess can only save iterations.
 *
 * Network: four periodic 3x3x3 convolutions with 2 -> 16 -> 16 -> 16 -> 1
 * channels, ReLU after the first three, no biases (cross-correlation):
 *   out[co](x) = sum_ci sum_d W[co][ci][t(d)] in[ci](x + d),  d in {-1,0,1}^3,
 *   t(d) = (dz+1)*9 + (dy+1)*3 + (dx+1).
 * Weights: PISOC_NET_NWEIGHTS FP32 values, layer after layer, each layer as
 * [co][ci][27].  Evaluation uses BF16 weights and activations with FP32
 * accumulation on the matrix cores.  Grids need n % 16 == 0.
 * Inputs: channel-last FP32 [batch][n^3][2]; outputs FP32 [batch][n^3].
 * Input channels (pisoc_net_inputs): (b/diag(M))/s1 and (p0 - <p0>)/s2, s1, s2
 * their r.m.s.; the target is p'/s1, and the guess is s1 times the output. */
#define PISOC_NET_NWEIGHTS 15120

size_t pisoc_net_workspace_bytes(int32_t n, int32_t batch);

/* y = net(x) for a batch of grids.  Asynchronous. */
pisoc_status pisoc_net_forward(int32_t n, int32_t batch, const float* d_w, const float* d_x,
                               float* d_y, void* d_ws, size_t ws_bytes, void* hip_stream);

/* Mean squared error loss of net(x) against t and its gradient with respect to
 * the weights (d_grad: PISOC_NET_NWEIGHTS FP32, overwritten; summed over the
 * batch deterministically).  h_loss (host, may be NULL) receives the loss;
 * then the call synchronises. */
pisoc_status pisoc_net_grad(int32_t n, int32_t batch, const float* d_w, const float* d_x,
                            const float* d_t, float* d_grad, double* h_loss, void* d_ws,
                            size_t ws_bytes, void* hip_stream);

/* Training on what the solve measures.  For sample i with its captured
 * pressure system (FP64 [batch][n^3] device arrays: right-hand side d_b,
 * diagonal d_diag and w = rho/a_P in d_wk, as pisoc_fields returns them) and
 * g = net(x_i):  u = M g, alpha = g.b / g.u (the rescale the solve applies to
 * a guess), and the loss L_i = |b - alpha u|^2 / |b|^2, the relative residual
 * the solve would start from; L is invariant to the scales of g and b.  The
 * call returns the batch mean of L_i in h_loss (host, may be NULL; then it
 * synchronises) and its gradient with respect to the weights in d_grad
 * (PISOC_NET_NWEIGHTS FP32, overwritten).  A sample with g.u <= 0 or b = 0
 * counts L_i = 1 with zero gradient. */
pisoc_status pisoc_net_grad_residual(int32_t n, int32_t batch, const float* d_w, const float* d_x,
                                     const double* d_b, const double* d_diag, const double* d_wk,
                                     float* d_grad, double* h_loss, void* d_ws, size_t ws_bytes,
                                     void* hip_stream);

/* One Adam update of nw FP32 weights (step counts from 1).  Asynchronous. */
pisoc_status pisoc_net_adam(int32_t nw, float* d_w, const float* d_g, float* d_m, float* d_v,
                            int32_t step, float lr, float beta1, float beta2, float eps,
                            void* hip_stream);

/* Network inputs of one pressure system (FP64 n^3 device arrays b, diag, p0 as
 * captured by pisoc_fields) into d_x (FP32 [n^3][2]); with d_psol non-NULL the
 * training target p'/s1 into d_t.  h_scales (host, may be NULL) receives
 * s1, s2; then the call synchronises.  d_ws: pisoc_helm_workspace_bytes(n). */
pisoc_status pisoc_net_inputs(int32_t n, const double* d_b, const double* d_diag,
                              const double* d_p0, const double* d_psol, float* d_x, float* d_t,
                              double* h_scales, void* d_ws, size_t ws_bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
