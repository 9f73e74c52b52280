/* oracle.h -- FP64 CPU oracle of one barotropic PISO step with
 * Equilibrium-Eulerian dust transport (test infrastructure only).
 *
 * This library exists to check the GPU library.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no code,
 * header, constant or helper with the GPU path.
 *
 * Grid: periodic cube [0, 2 pi)^3 with n cells per side, spacing h = 2 pi / n,
 * cell volume V = h^3, face area A = h^2.  Cell arrays hold n^3 doubles at
 * offset i + n*(j + n*k) (x fastest).  Face array d holds, at the offset of
 * cell P, the value on the face between P and P + e_d (face "P + 1/2 e_d").
 */
#ifndef PISO_ORACLE_H
#define PISO_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAX_CLASSES 8
#define ORA_MAX_CORR 8

/* status codes (same meaning as the GPU library's) */
#define ORA_OK 0
#define ORA_WARN_NOT_CONVERGED 1
#define ORA_WARN_DUST 3            /* a dust flag below (negative density, diagonal) */
#define ORA_ERR_INVALID (-1)
#define ORA_ERR_DIVERGED (-3)

/* info flags */
#define ORA_FLAG_PCG_MAXIT 1
#define ORA_FLAG_NONFINITE 2
#define ORA_FLAG_RHO_NONPOS 4
#define ORA_FLAG_KFACE_NONPOS 8
/* dust (Equilibrium-Eulerian transport, per step, any class):
 * a bulk density rho_j < 0 after the conservative finish (warning) */
#define ORA_FLAG_DUST_NEG 64
/* a non-finite rho_j (the step is rejected) */
#define ORA_FLAG_DUST_NONFINITE 128
/* the implicit mass-ratio equation's diagonal rho^{n+1}/dt + (9/16) div G is
 * <= 0 in some cell (its Jacobi sweeps lose their contraction there; warning) */
#define ORA_FLAG_DUST_DIAG 256
/* the dust's Courant number sigma_j dt, sigma_j = max sum_f |G_f| / (2 rho V), is
 * >= 0.638 for some class: for a uniform drift the update (n_Y = 4 Jacobi sweeps
 * and the conservative finish, the polynomial sum_{l<=5} (-z)^l of the central
 * I4 transport symbol z) amplifies some Fourier mode beyond that (warning) */
#define ORA_FLAG_DUST_COURANT 512
#define ORA_DUST_COURANT_MAX 0.638
/* the momentum predictor's BiCGStab reached mom_maxit before mom_tol (warning) */
#define ORA_FLAG_MOM_MAXIT 1024

typedef struct {
    int32_t n;
    int32_t n_classes;
    double gamma, C, mu;
    double tau_p[ORA_MAX_CLASSES];
    double cfl, dt_growth, dt_fixed, dt_max;
    int32_t n_corr, n_mom_sweeps, n_dust_sweeps;
    double p_tol;
    int32_t p_maxit;
    /* two-way coupling: the gas momentum is the mixture's (density rho + sum rho_j,
     * convected by the gas plus dust mass fluxes, buoyancy (rho_m - <rho_m>) g) */
    int32_t two_way;
    /* gravity: the dust settles with u_j = u + tau_j (g - Du/Dt); with two_way
     * the mixture also feels its buoyancy */
    double gravity[3];
    /* closure: 0 barotropic p = C rho^gamma; 1 Fourier: ideal gas p = rho R T
     * with an energy equation whose heat flux is q = -kappa grad T (c_v: heat
     * capacity at constant volume per unit mass; T0: initial uniform
     * temperature, see ora_set_temperature) */
    int32_t closure;
    double R_gas, cv, kappa, T0;
    /* time scheme: 0 backward Euler (BDF1); 1 BDF2 with variable steps,
     * d/dt y ~ (c0 y^{n+1} - c1 y^n + c2 y^{n-1}) / dt, w = dt / dt_prev,
     * c0 = (1 + 2w)/(1 + w), c1 = 1 + w, c2 = w^2/(1 + w) (the first step,
     * with no previous one, is BDF1: w = 0).  BDF2 takes the barotropic,
     * one-way step only. */
    int32_t time_scheme;
    /* momentum predictor: mom_tol = 0, n_mom_sweeps Jacobi sweeps; mom_tol > 0,
     * the system a_P u + N(u) = s - grad p^n (the three components stacked)
     * solved to ||r|| <= mom_tol ||s - grad p^n|| from u^n by BiCGStab
     * (van der Vorst 1992) preconditioned with diag(a_P), at most mom_maxit
     * iterations (not converged: ORA_FLAG_MOM_MAXIT, a warning) */
    double mom_tol;
    int32_t mom_maxit;
} ora_params;

#define ORA_BDF1 0
#define ORA_BDF2 1

#define ORA_BAROTROPIC 0
#define ORA_FOURIER 1

typedef struct {
    double t, dt, courant;
    int32_t pcg_iters[ORA_MAX_CORR];
    double pcg_relres[ORA_MAX_CORR];
    int32_t flags;
    double mass_gas;
    double mass_p[ORA_MAX_CLASSES];
    double courant_dust;   /* max over the classes of sigma_j dt */
    int32_t mom_iters;     /* BiCGStab iterations of the momentum predictor (mom_tol > 0) */
    double mom_relres;     /* its final ||r|| / ||s - grad p^n|| */
} ora_info;

/* statistics, in this order */
#define ORA_STAT_KE 0
#define ORA_STAT_ENSTROPHY 1
#define ORA_STAT_RHO_RMS 2
#define ORA_STAT_MACH_RMS 3
#define ORA_STAT_MASS_GAS 4
#define ORA_STAT_CONC_VAR 5              /* n_classes entries */
#define ORA_STAT_MASS_P (5 + ORA_MAX_CLASSES)  /* n_classes entries */
#define ORA_N_STATS (5 + 2 * ORA_MAX_CLASSES)

/* field selectors for ora_get */
enum {
    ORA_RHO = 0,      /* n^3 */
    ORA_U = 1,        /* 3 n^3 */
    ORA_PHI = 2,      /* 3 n^3 faces */
    ORA_RHO_P = 3,    /* n_classes n^3 */
    ORA_P = 4,        /* n^3: C rho^gamma (Fourier: rho R T) */
    ORA_T = 5,        /* n^3: temperature (Fourier closure) */
    /* pressure system of corrector `corr` of the last step */
    ORA_SYS_B = 10,   /* right-hand side b */
    ORA_SYS_W = 11,   /* rho/a_P at cell centres (face coefficient source) */
    ORA_SYS_PSIDT = 12, /* psi/dt */
    ORA_SYS_K = 13,   /* 3 n^3 face coefficients */
    ORA_SYS_X = 14,   /* solution p' */
    ORA_SYS_P0 = 15,  /* p(rho) at the corrector's start */
    ORA_SYS_DIAG = 16, /* diagonal of M */
    ORA_SYS_USTAR = 17 /* 3 n^3: momentum-predictor output u* of the last step */
};

typedef struct ora_state ora_state;

/* ---- whole step ---- */
int ora_create(const ora_params* prm, const double* rho, const double* u,
               const double* rho_p, ora_state** out);
int ora_step(ora_state* s, int32_t n_steps, ora_info* info);
int ora_get(const ora_state* s, int32_t which, int32_t corr, double* dst);
int ora_stats(const ora_state* s, double* out);
double ora_time(const ora_state* s);
void ora_destroy(ora_state* s);
/* keep copies of each corrector's pressure system (b, w, psi/dt, K, p', p0, diag) */
void ora_set_capture(ora_state* s, int32_t on);
/* Fourier closure: the temperature field (n^3) before the first step. */
int ora_set_temperature(ora_state* s, const double* T);
int ora_num_threads(void);

/* ---- operators (exposed for the pins) ---- */
void ora_i4(int32_t n, int32_t d, const double* q, double* out);
void ora_sngrad(int32_t n, int32_t d, const double* q, double* out);
void ora_div_flux(int32_t n, const double* f0, const double* f1, const double* f2, double* out);
void ora_grad(int32_t n, const double* q, double* g0, double* g1, double* g2);
void ora_div_vel(int32_t n, const double* u0, const double* u1, const double* u2, double* out);
void ora_lap(int32_t n, const double* q, double* out);
void ora_kfaces(int32_t n, const double* w, double* k0, double* k1, double* k2);
void ora_helm_apply(int32_t n, const double* psidt, const double* k0, const double* k1,
                    const double* k2, const double* x, double* y);
int32_t ora_pcg(int32_t n, const double* psidt, const double* k0, const double* k1,
                const double* k2, const double* b, double* x, double tol, int32_t maxit,
                double* relres);
void ora_cheb_coef(int32_t n, const double* psidt, const double* k0, const double* k1,
                   const double* k2, double* c);
void ora_cheb_apply(int32_t n, const double* psidt, const double* k0, const double* k1,
                    const double* k2, const double* r, double* z);
int32_t ora_pcg_cheb(int32_t n, const double* psidt, const double* k0, const double* k1,
                     const double* k2, const double* b, double* x, double tol, int32_t maxit,
                     double* relres);

/* ---- learned pressure guess: inputs and solve start (guess.c) ---- */
int ora_net_inputs(int32_t n, const double* b, const double* diag, const double* p0, double* x,
                   double* scales);
int ora_guess_start(int32_t n, const double* psidt, const double* k0, const double* k1,
                    const double* k2, const double* b, const double* g, double* x0, double* alpha,
                    double* res_ratio);

/* ---- learned pressure-guess network (conv.c) ---- */
int32_t ora_conv_nweights(void);
int ora_conv_forward(int32_t n, int32_t batch, const double* w, const double* x, double* y);
int ora_conv_backward(int32_t n, int32_t batch, const double* w, const double* x, const double* t,
                      double* grad_w, double* loss);
int ora_conv_backward_dy(int32_t n, int32_t batch, const double* w, const double* x, const double* dy,
                         double* grad_w);

#ifdef __cplusplus
}
#endif
#endif
