/* oracle.c -- FP64 CPU oracle of one PISO time step of a barotropic gas with
 * Equilibrium-Eulerian dust (test infrastructure only: the tests, the smoke
 * check and the benchmark's CPU-baseline leg load it; the GPU library never
 * does, and the two share no code).
 *
 * What the paper fixes (Results section): a collocated finite-volume PISO
 * pressure-based solver with fourth-order central interpolation and an
 * adaptive time step; a barotropic closure p = C rho^gamma (second footnote);
 * dust carried by the Equilibrium-Eulerian model, i.e. the particle velocity
 * to first order in the Stokes number under Stokes drag, u_p = u - tau_p Du/Dt,
 * whose zero-order version is Marble's dusty gas u_p = u (third footnote).
 * The paper prints no discrete equations.  Every discrete choice below is a
 * reading of those statements, written next to the code it governs:
 *
 *   time scheme        backward Euler in every equation;
 *   interpolation      I4(q)_{P+1/2} = (-q_{P-1} + 9 q_P + 9 q_{P+1} - q_{P+2}) / 16;
 *   face gradient      compact (q_{P+1} - q_P) / h;
 *   cell gradient      Gauss theorem over I4 face values;
 *   momentum           I4 convection with the old mass fluxes and the compact
 *                      viscous Laplacian implicit (Jacobi sweeps, fixed count),
 *                      (mu/3) grad(div u) explicit, Stokes hypothesis;
 *   pressure equation  continuity defect as the right-hand side, Newton
 *                      linearisation drho = psi dp with psi = 1/(gamma C rho^(gamma-1)),
 *                      face coefficient K_f = I4(rho / a_P), Jacobi-preconditioned
 *                      CG stopped at ||r||_2 <= tol ||b||_2;
 *   time step          dt = min(cfl / sigma, growth dt_prev, dt_max) with the
 *                      convective Courant rate sigma = max_P sum_f |phi_f| / (2 rho_P V);
 *   dust               one-way coupled; the mass ratio Y = rho_j / rho is carried
 *                      by the particle mass flux G_f = phi_f - tau_j I4(rho) I4(a) A,
 *                      a = Du/Dt, with implicit Jacobi sweeps, then a conservative
 *                      flux-form update of rho_j.
 *
 * Plain loops over cells with modular periodic indexing.  OpenMP only splits the
 * outer (k) loop; every reduction sums per-plane partials in plane order, so
 * results do not depend on the thread count.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* grid helpers                                                              */
/* ------------------------------------------------------------------------- */

static const double TWO_PI = 6.283185307179586476925286766559;

static inline double spacing(int n) { return TWO_PI / (double)n; }

static inline int wrapi(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

static inline size_t cell(int n, int i, int j, int k) {
    return (size_t)wrapi(i, n) + (size_t)n * ((size_t)wrapi(j, n) + (size_t)n * (size_t)wrapi(k, n));
}

/* offset of the cell reached from (i,j,k) by s steps along axis d */
static inline size_t shifted(int n, int i, int j, int k, int d, int s) {
    int c[3] = {i, j, k};
    c[d] += s;
    return cell(n, c[0], c[1], c[2]);
}

static inline size_t ncell(int n) { return (size_t)n * (size_t)n * (size_t)n; }

static double* alloc_field(size_t count) {
    double* p = (double*)calloc(count ? count : 1, sizeof(double));
    return p;
}

/* Sum of f over all cells in a fixed order: per k-plane partials, then planes in order. */
static double sum_field(int n, const double* f) {
    double* part = alloc_field((size_t)n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) s += f[cell(n, i, j, k)];
        part[k] = s;
    }
    double tot = 0.0;
    for (int k = 0; k < n; ++k) tot += part[k];
    free(part);
    return tot;
}

static double dot_field(int n, const double* a, const double* b) {
    double* part = alloc_field((size_t)n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t P = cell(n, i, j, k);
                s += a[P] * b[P];
            }
        part[k] = s;
    }
    double tot = 0.0;
    for (int k = 0; k < n; ++k) tot += part[k];
    free(part);
    return tot;
}

/* ------------------------------------------------------------------------- */
/* discrete operators                                                        */
/* ------------------------------------------------------------------------- */

/* Fourth-order central interpolation to the faces P + 1/2 e_d (Results section:
 * "fourth order central interpolation"): the symmetric 4-point Lagrange weights
 * (-1, 9, 9, -1)/16 on the cells P - e_d, P, P + e_d, P + 2 e_d. */
void ora_i4(int32_t n, int32_t d, const double* q, double* out) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double qm = q[shifted(n, i, j, k, d, -1)];
                double q0 = q[shifted(n, i, j, k, d, 0)];
                double q1 = q[shifted(n, i, j, k, d, 1)];
                double q2 = q[shifted(n, i, j, k, d, 2)];
                out[cell(n, i, j, k)] = (-qm + 9.0 * q0 + 9.0 * q1 - q2) / 16.0;
            }
}

/* Compact face-normal gradient at P + 1/2 e_d. */
void ora_sngrad(int32_t n, int32_t d, const double* q, double* out) {
    double h = spacing(n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                out[cell(n, i, j, k)] = (q[shifted(n, i, j, k, d, 1)] - q[cell(n, i, j, k)]) / h;
}

/* Finite-volume divergence of face fluxes (per unit volume): sum over the six
 * faces of the outward flux, divided by V. */
void ora_div_flux(int32_t n, const double* f0, const double* f1, const double* f2, double* out) {
    double h = spacing(n);
    double V = h * h * h;
    const double* f[3] = {f0, f1, f2};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    s += f[d][cell(n, i, j, k)] - f[d][shifted(n, i, j, k, d, -1)];
                out[cell(n, i, j, k)] = s / V;
            }
}

/* Cell-centred gradient by the Gauss theorem with I4 face values:
 * (grad q)_d = (I4(q)_{P+1/2} - I4(q)_{P-1/2}) / h. */
void ora_grad(int32_t n, const double* q, double* g0, double* g1, double* g2) {
    double h = spacing(n);
    double* g[3] = {g0, g1, g2};
    double* face = alloc_field(ncell(n));
    for (int d = 0; d < 3; ++d) {
        ora_i4(n, d, q, face);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i)
                    g[d][cell(n, i, j, k)] =
                        (face[cell(n, i, j, k)] - face[shifted(n, i, j, k, d, -1)]) / h;
    }
    free(face);
}

/* Cell divergence of a velocity field by the Gauss theorem with I4 face values. */
void ora_div_vel(int32_t n, const double* u0, const double* u1, const double* u2, double* out) {
    double h = spacing(n);
    const double* u[3] = {u0, u1, u2};
    double* face = alloc_field(ncell(n));
    memset(out, 0, ncell(n) * sizeof(double));
    for (int d = 0; d < 3; ++d) {
        ora_i4(n, d, u[d], face);
#pragma omp parallel for schedule(static)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i)
                    out[cell(n, i, j, k)] +=
                        (face[cell(n, i, j, k)] - face[shifted(n, i, j, k, d, -1)]) / h;
    }
    free(face);
}

/* Compact 7-point Laplacian. */
void ora_lap(int32_t n, const double* q, double* out) {
    double h = spacing(n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    s += q[shifted(n, i, j, k, d, 1)] - 2.0 * q[cell(n, i, j, k)] +
                         q[shifted(n, i, j, k, d, -1)];
                out[cell(n, i, j, k)] = s / (h * h);
            }
}

/* Face coefficients of the pressure Laplacian: K_d = I4 of the cell field w. */
void ora_kfaces(int32_t n, const double* w, double* k0, double* k1, double* k2) {
    ora_i4(n, 0, w, k0);
    ora_i4(n, 1, w, k1);
    ora_i4(n, 2, w, k2);
}

/* Pressure (Helmholtz) operator:
 * (M x)_P = psidt_P x_P + (1/h^2) sum_faces K_f (x_P - x_nb). */
void ora_helm_apply(int32_t n, const double* psidt, const double* k0, const double* k1,
                    const double* k2, const double* x, double* y) {
    double h = spacing(n);
    const double* K[3] = {k0, k1, k2};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t P = cell(n, i, j, k);
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    size_t E = shifted(n, i, j, k, d, 1);
                    size_t W = shifted(n, i, j, k, d, -1);
                    s += K[d][P] * (x[P] - x[E]) + K[d][W] * (x[P] - x[W]);
                }
                y[P] = psidt[P] * x[P] + s / (h * h);
            }
}

static void helm_diag(int32_t n, const double* psidt, const double* const K[3], double* diag) {
    double h = spacing(n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t P = cell(n, i, j, k);
                double s = 0.0;
                for (int d = 0; d < 3; ++d) s += K[d][P] + K[d][shifted(n, i, j, k, d, -1)];
                diag[P] = psidt[P] + s / (h * h);
            }
}

/* Jacobi-preconditioned conjugate gradients on M x = b, starting from the x
 * passed in.  Stops when ||r||_2 <= tol ||b||_2 (measured against b, so that a
 * better starting point can only save iterations).  Returns the number of
 * iterations, or -maxit - 1 if maxit iterations did not reach the tolerance.
 * relres receives ||r||_2 / ||b||_2 (0 when b = 0). */
int32_t ora_pcg(int32_t n, const double* psidt, const double* k0, const double* k1,
                const double* k2, const double* b, double* x, double tol, int32_t maxit,
                double* relres) {
    size_t N = ncell(n);
    const double* K[3] = {k0, k1, k2};
    double* diag = alloc_field(N);
    double* r = alloc_field(N);
    double* z = alloc_field(N);
    double* p = alloc_field(N);
    double* q = alloc_field(N);
    helm_diag(n, psidt, K, diag);

    ora_helm_apply(n, psidt, k0, k1, k2, x, q);
    for (size_t P = 0; P < N; ++P) r[P] = b[P] - q[P];
    double bb = dot_field(n, b, b);
    double rr = dot_field(n, r, r);
    double lim = tol * tol * bb;
    int32_t it = 0;
    int converged = rr <= lim;
    if (!converged) {
        for (size_t P = 0; P < N; ++P) {
            z[P] = r[P] / diag[P];
            p[P] = z[P];
        }
        double rz = dot_field(n, r, z);
        while (it < maxit) {
            ora_helm_apply(n, psidt, k0, k1, k2, p, q);
            double alpha = rz / dot_field(n, p, q);
            for (size_t P = 0; P < N; ++P) {
                x[P] += alpha * p[P];
                r[P] -= alpha * q[P];
            }
            ++it;
            rr = dot_field(n, r, r);
            if (rr <= lim) {
                converged = 1;
                break;
            }
            for (size_t P = 0; P < N; ++P) z[P] = r[P] / diag[P];
            double rz_new = dot_field(n, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
            for (size_t P = 0; P < N; ++P) p[P] = z[P] + beta * p[P];
        }
    }
    if (relres) *relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    free(diag);
    free(r);
    free(z);
    free(p);
    free(q);
    return converged ? it : -maxit - 1;
}

/* Degree-1 Chebyshev polynomial preconditioner, a non-learned rival of the
 * learned guess (not in the paper).  With D = diag(M) the spectrum of D^-1 M
 * lies in [a, b], a = min_P psidt_P / diag_P, b = 2 - a (Gershgorin: the
 * off-diagonal entries of a row of D^-1 M sum in magnitude to
 * 1 - psidt/diag).  z = p(D^-1 M) D^-1 r with the degree-1 p whose residual
 * polynomial 1 - lambda p(lambda) is the degree-2 Chebyshev polynomial of
 * [a, b] normalised to 1 at lambda = 0:
 *   1 - lambda p(lambda) = T2((b + a - 2 lambda)/(b - a)) / T2(mu),
 *   T2(s) = 2 s^2 - 1, mu = (b + a)/(b - a),
 * i.e. p(lambda) = c0 + c1 lambda, c0 = 8 mu / ((b - a) T2(mu)),
 * c1 = -8 / ((b - a)^2 T2(mu)).  p(b) = 8 a / ((b - a)^2 T2(mu)) > 0, so p is
 * positive on [a, b] and the preconditioner symmetric positive definite.
 * c receives c0, c1 and a. */
void ora_cheb_coef(int32_t n, const double* psidt, const double* k0, const double* k1,
                   const double* k2, double* c) {
    size_t N = ncell(n);
    const double* K[3] = {k0, k1, k2};
    double* diag = alloc_field(N);
    helm_diag(n, psidt, K, diag);
    double a = 1.0;
    for (size_t P = 0; P < N; ++P) {
        double t = psidt[P] / diag[P];
        if (t < a) a = t;
    }
    double b = 2.0 - a, mu = (b + a) / (b - a), t2 = 2.0 * mu * mu - 1.0;
    c[0] = 8.0 * mu / ((b - a) * t2);
    c[1] = -8.0 / ((b - a) * (b - a) * t2);
    c[2] = a;
    free(diag);
}

/* z = c0 D^-1 r + c1 D^-1 M D^-1 r (scratch: diag and t, N values each). */
static void cheb_apply(int32_t n, const double* psidt, const double* const K[3], const double* c,
                       const double* diag, const double* r, double* t, double* z) {
    size_t N = ncell(n);
    for (size_t P = 0; P < N; ++P) t[P] = r[P] / diag[P];
    ora_helm_apply(n, psidt, K[0], K[1], K[2], t, z);
    for (size_t P = 0; P < N; ++P) z[P] = c[0] * t[P] + c[1] * z[P] / diag[P];
}

void ora_cheb_apply(int32_t n, const double* psidt, const double* k0, const double* k1,
                    const double* k2, const double* r, double* z) {
    size_t N = ncell(n);
    const double* K[3] = {k0, k1, k2};
    double c[3];
    ora_cheb_coef(n, psidt, k0, k1, k2, c);
    double* diag = alloc_field(N);
    double* t = alloc_field(N);
    helm_diag(n, psidt, K, diag);
    cheb_apply(n, psidt, K, c, diag, r, t, z);
    free(diag);
    free(t);
}

/* Conjugate gradients on M x = b preconditioned by the Chebyshev polynomial
 * above; otherwise as ora_pcg (start, stopping rule, return value). */
int32_t ora_pcg_cheb(int32_t n, const double* psidt, const double* k0, const double* k1,
                     const double* k2, const double* b, double* x, double tol, int32_t maxit,
                     double* relres) {
    size_t N = ncell(n);
    const double* K[3] = {k0, k1, k2};
    double c[3];
    ora_cheb_coef(n, psidt, k0, k1, k2, c);
    double* diag = alloc_field(N);
    double* r = alloc_field(N);
    double* z = alloc_field(N);
    double* p = alloc_field(N);
    double* q = alloc_field(N);
    double* t = alloc_field(N);
    helm_diag(n, psidt, K, diag);
    ora_helm_apply(n, psidt, k0, k1, k2, x, q);
    for (size_t P = 0; P < N; ++P) r[P] = b[P] - q[P];
    double bb = dot_field(n, b, b);
    double rr = dot_field(n, r, r);
    double lim = tol * tol * bb;
    int32_t it = 0;
    int converged = rr <= lim;
    if (!converged) {
        cheb_apply(n, psidt, K, c, diag, r, t, z);
        for (size_t P = 0; P < N; ++P) p[P] = z[P];
        double rz = dot_field(n, r, z);
        while (it < maxit) {
            ora_helm_apply(n, psidt, k0, k1, k2, p, q);
            double alpha = rz / dot_field(n, p, q);
            for (size_t P = 0; P < N; ++P) {
                x[P] += alpha * p[P];
                r[P] -= alpha * q[P];
            }
            ++it;
            rr = dot_field(n, r, r);
            if (rr <= lim) {
                converged = 1;
                break;
            }
            cheb_apply(n, psidt, K, c, diag, r, t, z);
            double rz_new = dot_field(n, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
            for (size_t P = 0; P < N; ++P) p[P] = z[P] + beta * p[P];
        }
    }
    if (relres) *relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    free(diag);
    free(r);
    free(z);
    free(p);
    free(q);
    free(t);
    return converged ? it : -maxit - 1;
}

/* ------------------------------------------------------------------------- */
/* state                                                                     */
/* ------------------------------------------------------------------------- */

struct ora_state {
    ora_params p;
    int n;
    size_t N;
    double h, V, A;
    double t, dt_prev;
    int capture;
    /* state at t^n */
    double* rho;
    double* u[3];
    double* phi[3];
    double* rho_p[ORA_MAX_CLASSES];
    /* two-way: the dust mass fluxes of the last step, summed over the classes */
    double* fd[3];
    /* Fourier closure: temperature */
    double* T;
    /* BDF2: the state at t^{n-1} */
    double* rho_m1;
    double* u_m1[3];
    double* rho_p_m1[ORA_MAX_CLASSES];
    /* captured pressure systems of the last step, one set per corrector */
    double* sys_b[ORA_MAX_CORR];
    double* sys_w[ORA_MAX_CORR];
    double* sys_psidt[ORA_MAX_CORR];
    double* sys_k[ORA_MAX_CORR][3];
    double* sys_x[ORA_MAX_CORR];
    double* sys_p0[ORA_MAX_CORR];
    double* sys_diag[ORA_MAX_CORR];
    double* sys_ustar[3];
    /* work arrays of the step, allocated on first use and kept */
    double* pool[256];
};

static double* pool_get(ora_state* s, int slot) {
    if (!s->pool[slot]) s->pool[slot] = alloc_field(s->N);
    return s->pool[slot];
}

static int check_params(const ora_params* p) {
    if (p->n < 4 || p->n > 1024) return 0;
    if (p->n_classes < 0 || p->n_classes > ORA_MAX_CLASSES) return 0;
    if (!(p->gamma > 1.0) || !(p->C > 0.0) || !(p->mu >= 0.0)) return 0;
    if (p->closure != ORA_BAROTROPIC && p->closure != ORA_FOURIER) return 0;
    if (p->time_scheme != ORA_BDF1 && p->time_scheme != ORA_BDF2) return 0;
    if (!(p->mom_tol >= 0.0) || !(p->mom_tol < 1.0) || (p->mom_tol > 0.0 && p->mom_maxit < 1))
        return 0;
    if (p->time_scheme == ORA_BDF2 && (p->closure != ORA_BAROTROPIC || p->two_way)) return 0;
    if (p->closure == ORA_FOURIER &&
        (!(p->R_gas > 0.0) || !(p->cv > 0.0) || !(p->kappa >= 0.0) || !(p->T0 > 0.0)))
        return 0;
    if (p->n_corr < 1 || p->n_corr > ORA_MAX_CORR) return 0;
    if (p->n_mom_sweeps < 1 || p->n_dust_sweeps < 1) return 0;
    if (!(p->p_tol > 0.0) || p->p_maxit < 1) return 0;
    if (!(p->dt_fixed > 0.0) && !(p->cfl > 0.0 && p->dt_growth > 0.0)) return 0;
    for (int c = 0; c < p->n_classes; ++c)
        if (!(p->tau_p[c] >= 0.0)) return 0;
    return 1;
}

static void free_state(ora_state* s) {
    if (!s) return;
    free(s->rho);
    free(s->T);
    free(s->rho_m1);
    for (int d = 0; d < 3; ++d) free(s->u_m1[d]);
    for (int c = 0; c < ORA_MAX_CLASSES; ++c) free(s->rho_p_m1[c]);
    for (int d = 0; d < 3; ++d) {
        free(s->u[d]);
        free(s->phi[d]);
        free(s->fd[d]);
    }
    for (int c = 0; c < ORA_MAX_CLASSES; ++c) free(s->rho_p[c]);
    for (int c = 0; c < ORA_MAX_CORR; ++c) {
        free(s->sys_b[c]);
        free(s->sys_w[c]);
        free(s->sys_psidt[c]);
        for (int d = 0; d < 3; ++d) free(s->sys_k[c][d]);
        free(s->sys_x[c]);
        free(s->sys_p0[c]);
        free(s->sys_diag[c]);
    }
    for (int d = 0; d < 3; ++d) free(s->sys_ustar[d]);
    for (int i = 0; i < 256; ++i) free(s->pool[i]);
    free(s);
}

int ora_num_threads(void) { return omp_get_max_threads(); }

/* Initial mass fluxes: phi_d = I4(rho) I4(u_d) A on every face; with two-way
 * coupling also the dust's, fd_d = I4(sum_j rho_j) I4(u_d) A (the dust moving
 * with the gas: its drift needs Du/Dt, unknown before the first step). */
static void initial_fluxes(ora_state* s) {
    double* fr = alloc_field(s->N);
    double* fu = alloc_field(s->N);
    double* rd = alloc_field(s->N);
    for (int c = 0; c < s->p.n_classes; ++c)
        for (size_t P = 0; P < s->N; ++P) rd[P] += s->rho_p[c][P];
    for (int d = 0; d < 3; ++d) {
        ora_i4(s->n, d, s->rho, fr);
        ora_i4(s->n, d, s->u[d], fu);
        for (size_t P = 0; P < s->N; ++P) s->phi[d][P] = fr[P] * fu[P] * s->A;
        if (s->p.two_way) {
            s->fd[d] = alloc_field(s->N);
            ora_i4(s->n, d, rd, fr);
            for (size_t P = 0; P < s->N; ++P) s->fd[d][P] = fr[P] * fu[P] * s->A;
        }
    }
    free(fr);
    free(fu);
    free(rd);
}

int ora_create(const ora_params* prm, const double* rho, const double* u, const double* rho_p,
               ora_state** out) {
    if (!prm || !rho || !u || !out || !check_params(prm)) return ORA_ERR_INVALID;
    if (prm->n_classes > 0 && !rho_p) return ORA_ERR_INVALID;
    ora_state* s = (ora_state*)calloc(1, sizeof(ora_state));
    s->p = *prm;
    s->n = prm->n;
    s->N = ncell(prm->n);
    s->h = spacing(prm->n);
    s->V = s->h * s->h * s->h;
    s->A = s->h * s->h;
    s->t = 0.0;
    s->dt_prev = INFINITY;
    s->rho = alloc_field(s->N);
    memcpy(s->rho, rho, s->N * sizeof(double));
    for (int d = 0; d < 3; ++d) {
        s->u[d] = alloc_field(s->N);
        memcpy(s->u[d], u + (size_t)d * s->N, s->N * sizeof(double));
        s->phi[d] = alloc_field(s->N);
    }
    for (int c = 0; c < prm->n_classes; ++c) {
        s->rho_p[c] = alloc_field(s->N);
        memcpy(s->rho_p[c], rho_p + (size_t)c * s->N, s->N * sizeof(double));
    }
    initial_fluxes(s);
    if (prm->closure == ORA_FOURIER) {
        s->T = alloc_field(s->N);
        for (size_t P = 0; P < s->N; ++P) s->T[P] = prm->T0;
    }
    if (prm->time_scheme == ORA_BDF2) {   /* unused until a step has been taken */
        s->rho_m1 = alloc_field(s->N);
        for (int d = 0; d < 3; ++d) s->u_m1[d] = alloc_field(s->N);
        for (int c = 0; c < prm->n_classes; ++c) s->rho_p_m1[c] = alloc_field(s->N);
    }
    *out = s;
    return ORA_OK;
}

int ora_set_temperature(ora_state* s, const double* T) {
    if (!s || !T || s->p.closure != ORA_FOURIER) return ORA_ERR_INVALID;
    memcpy(s->T, T, s->N * sizeof(double));
    return ORA_OK;
}

void ora_destroy(ora_state* s) { free_state(s); }

double ora_time(const ora_state* s) { return s->t; }

void ora_set_capture(ora_state* s, int32_t on) { s->capture = on; }

/* ------------------------------------------------------------------------- */
/* the step                                                                  */
/* ------------------------------------------------------------------------- */

/* Off-diagonal part of the implicit momentum operator for one velocity
 * component q (per unit volume):
 *   N(q)_P = (1/V) sum_f F_f^out I4(q)_f - (9/16) div(phi)_P q_P
 *            - mu [Lap(q)_P + 6 q_P / h^2],
 * i.e. the I4 convection with the old mass fluxes F = phi^n plus the compact
 * viscous Laplacian, without their q_P coefficients (which sit in a_P). */
static void mom_offdiag(const ora_state* s, double* const phi[3], const double* divphi,
                        const double* q, double* out, double* t_face[3], double* t_lap) {
    int n = s->n;
    double h = s->h;
    double mu = s->p.mu;
    for (int d = 0; d < 3; ++d) {
        ora_i4(n, d, q, t_face[d]);
        for (size_t P = 0; P < s->N; ++P) t_face[d][P] *= phi[d][P];
    }
    ora_div_flux(n, t_face[0], t_face[1], t_face[2], out);
    ora_lap(n, q, t_lap);
    for (size_t P = 0; P < s->N; ++P)
        out[P] += -(9.0 / 16.0) * divphi[P] * q[P] - mu * (t_lap[P] + 6.0 * q[P] / (h * h));
}

/* y = A x for the stacked momentum system: y_d = a_P x_d + N(x_d). */
static void mom_apply(const ora_state* s, double* const fm[3], const double* divfm,
                      const double* aP, double* const x[3], double* const y[3], double* t_face[3],
                      double* t_lap) {
    for (int d = 0; d < 3; ++d) {
        mom_offdiag(s, fm, divfm, x[d], y[d], t_face, t_lap);
        for (size_t P = 0; P < s->N; ++P) y[d][P] += aP[P] * x[d][P];
    }
}

static double dot3(int n, double* const a[3], double* const b[3]) {
    return dot_field(n, a[0], b[0]) + dot_field(n, a[1], b[1]) + dot_field(n, a[2], b[2]);
}

static void keep(double** slot, size_t N, const double* src) {
    if (!*slot) *slot = alloc_field(N);
    memcpy(*slot, src, N * sizeof(double));
}

static int one_step(ora_state* s, ora_info* info) {
    const ora_params* pr = &s->p;
    const int n = s->n;
    const size_t N = s->N;
    const double h = s->h, V = s->V, A = s->A;
    const double g = pr->gamma, Cc = pr->C, mu = pr->mu;
    int flags = 0;
    int status = ORA_OK;
    int slot = 0;
    memset(info, 0, sizeof(*info));

#define NEWF(name) double* name = pool_get(s, slot++)
    /* ---- 1. adaptive time step (Results section: adaptive time step) ---- */
    NEWF(sig);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t P = cell(n, i, j, k);
                double f = 0.0;
                for (int d = 0; d < 3; ++d)
                    f += fabs(s->phi[d][P]) + fabs(s->phi[d][shifted(n, i, j, k, d, -1)]);
                sig[P] = f / (2.0 * s->rho[P] * V);
            }
    double sigma = 0.0;
    for (size_t P = 0; P < N; ++P)
        if (sig[P] > sigma) sigma = sig[P];
    double dt;
    if (pr->dt_fixed > 0.0) {
        dt = pr->dt_fixed;
    } else {
        dt = sigma > 0.0 ? pr->cfl / sigma : INFINITY;
        if (pr->dt_growth * s->dt_prev < dt) dt = pr->dt_growth * s->dt_prev;
        if (pr->dt_max > 0.0 && pr->dt_max < dt) dt = pr->dt_max;
    }
    if (!(dt > 0.0) || !isfinite(dt)) return ORA_ERR_INVALID;
    /* time derivative d/dt y ~ (c0 y^{n+1} - c1 y^n + c2 y^{n-1}) / dt */
    const int bdf2 = pr->time_scheme == ORA_BDF2;
    const double om = bdf2 && isfinite(s->dt_prev) ? dt / s->dt_prev : 0.0;
    const double c0 = (1.0 + 2.0 * om) / (1.0 + om), c1 = 1.0 + om, c2 = om * om / (1.0 + om);

    /* ---- 2. density predictor: rho* = rho^n - dt div(phi^n) ---- */
    NEWF(divphi);
    NEWF(rhos);
    ora_div_flux(n, s->phi[0], s->phi[1], s->phi[2], divphi);
    if (bdf2)
        for (size_t P = 0; P < N; ++P)
            rhos[P] = (c1 * s->rho[P] - c2 * s->rho_m1[P] - dt * divphi[P]) / c0;
    else
        for (size_t P = 0; P < N; ++P) rhos[P] = s->rho[P] - dt * divphi[P];

    /* ---- two-way coupling: the momentum equation is the mixture's.  Its
     * density rho_m = rho + rho_d (rho_d = sum_j rho_j), predicted as
     * rho_m* = rho_m^n - dt div(F_m^n), convected by the mixture mass flux
     * F_m = phi + fd (fd: the dust's mass fluxes of the last step), with the
     * buoyancy (rho_m^n - <rho_m^n>) g.  One-way: rho_m = rho, F_m = phi. ---- */
    double* fm[3] = {s->phi[0], s->phi[1], s->phi[2]};
    double* divfm = divphi;
    double* rms = rhos;             /* predicted density of the momentum equation */
    double* rmn = s->rho;           /* its density at t^n */
    double mean_m = 0.0;
    if (pr->two_way) {
        NEWF(rdn);
        memset(rdn, 0, N * sizeof(double));   /* pool arrays keep the last step's values */
        for (int c = 0; c < pr->n_classes; ++c)
            for (size_t P = 0; P < N; ++P) rdn[P] += s->rho_p[c][P];
        NEWF(fm0); NEWF(fm1); NEWF(fm2);
        fm[0] = fm0; fm[1] = fm1; fm[2] = fm2;
        for (int d = 0; d < 3; ++d)
            for (size_t P = 0; P < N; ++P) fm[d][P] = s->phi[d][P] + s->fd[d][P];
        NEWF(dfm);
        divfm = dfm;
        ora_div_flux(n, fm[0], fm[1], fm[2], divfm);
        NEWF(rmn_);
        NEWF(rms_);
        rmn = rmn_;
        rms = rms_;
        for (size_t P = 0; P < N; ++P) {
            rmn[P] = s->rho[P] + rdn[P];
            rms[P] = rmn[P] - dt * divfm[P];
        }
        mean_m = sum_field(n, rmn) / (double)N;
    }

    /* ---- 3. momentum coefficients and explicit source ---- */
    NEWF(aP);
    for (size_t P = 0; P < N; ++P)
        aP[P] = (bdf2 ? c0 : 1.0) * rms[P] / dt + (9.0 / 16.0) * divfm[P] + 6.0 * mu / (h * h);
    NEWF(divu);
    NEWF(gd0); NEWF(gd1); NEWF(gd2);
    double* gdivu[3] = {gd0, gd1, gd2};
    ora_div_vel(n, s->u[0], s->u[1], s->u[2], divu);
    ora_grad(n, divu, gd0, gd1, gd2);
    NEWF(s0); NEWF(s1); NEWF(s2);
    double* src[3] = {s0, s1, s2};
    for (int d = 0; d < 3; ++d)
        for (size_t P = 0; P < N; ++P) {
            src[d][P] = (bdf2 ? c1 * rmn[P] * s->u[d][P] - c2 * s->rho_m1[P] * s->u_m1[d][P]
                              : rmn[P] * s->u[d][P]) / dt +
                        (mu / 3.0) * gdivu[d][P];
            if (pr->two_way) src[d][P] += (rmn[P] - mean_m) * pr->gravity[d];
        }
    NEWF(pn);
    const int fourier = pr->closure == ORA_FOURIER;
    const double Rg = pr->R_gas;
    for (size_t P = 0; P < N; ++P)
        pn[P] = fourier ? s->rho[P] * Rg * s->T[P] : Cc * pow(s->rho[P], g);
    NEWF(gp0); NEWF(gp1); NEWF(gp2);
    double* gpn[3] = {gp0, gp1, gp2};
    ora_grad(n, pn, gp0, gp1, gp2);

    /* scratch for the momentum operator */
    NEWF(tf0); NEWF(tf1); NEWF(tf2); NEWF(tlap);
    double* tface[3] = {tf0, tf1, tf2};
    NEWF(noff);

    /* ---- 4. momentum predictor: Jacobi sweeps of a_P u + N(u) = s - grad p^n ---- */
    double* ucur[3];
    double* unew[3];
    for (int d = 0; d < 3; ++d) {
        ucur[d] = pool_get(s, slot++);
        unew[d] = pool_get(s, slot++);
        memcpy(ucur[d], s->u[d], N * sizeof(double));
    }
    if (pr->mom_tol > 0.0) {
        /* BiCGStab on A u = s - grad p^n, right-preconditioned by K = diag(a_P) */
        double *bv[3], *r[3], *rh[3], *p[3], *v[3], *y[3], *sv[3], *z[3], *t[3];
        for (int d = 0; d < 3; ++d) {
            bv[d] = pool_get(s, slot++); r[d] = pool_get(s, slot++); rh[d] = pool_get(s, slot++);
            p[d] = pool_get(s, slot++); v[d] = pool_get(s, slot++); y[d] = pool_get(s, slot++);
            sv[d] = pool_get(s, slot++); z[d] = pool_get(s, slot++); t[d] = pool_get(s, slot++);
            for (size_t P = 0; P < N; ++P) bv[d][P] = src[d][P] - gpn[d][P];
        }
        mom_apply(s, fm, divfm, aP, ucur, t, tface, tlap);
        for (int d = 0; d < 3; ++d)
            for (size_t P = 0; P < N; ++P) {
                r[d][P] = bv[d][P] - t[d][P];
                rh[d][P] = r[d][P];
                p[d][P] = v[d][P] = 0.0;
            }
        const double bb = dot3(n, bv, bv), lim = pr->mom_tol * pr->mom_tol * bb;
        double rr = dot3(n, r, r), rho_old = 1.0, alpha = 1.0, omega = 1.0;
        int it = 0;
        while (!(rr <= lim) && it < pr->mom_maxit) {
            const double rho = dot3(n, rh, r);
            const double beta = (rho / rho_old) * (alpha / omega);
            for (int d = 0; d < 3; ++d)
                for (size_t P = 0; P < N; ++P) {
                    p[d][P] = r[d][P] + beta * (p[d][P] - omega * v[d][P]);
                    y[d][P] = p[d][P] / aP[P];
                }
            mom_apply(s, fm, divfm, aP, y, v, tface, tlap);
            alpha = rho / dot3(n, rh, v);
            for (int d = 0; d < 3; ++d)
                for (size_t P = 0; P < N; ++P) {
                    sv[d][P] = r[d][P] - alpha * v[d][P];
                    z[d][P] = sv[d][P] / aP[P];
                }
            mom_apply(s, fm, divfm, aP, z, t, tface, tlap);
            const double tt = dot3(n, t, t);
            omega = tt > 0.0 ? dot3(n, t, sv) / tt : 0.0;
            for (int d = 0; d < 3; ++d)
                for (size_t P = 0; P < N; ++P) {
                    ucur[d][P] += alpha * y[d][P] + omega * z[d][P];
                    r[d][P] = sv[d][P] - omega * t[d][P];
                }
            rho_old = rho;
            rr = dot3(n, r, r);
            ++it;
        }
        info->mom_iters = it;
        info->mom_relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        if (!(rr <= lim)) {
            flags |= ORA_FLAG_MOM_MAXIT;
            status = ORA_WARN_NOT_CONVERGED;
        }
    } else {
        for (int sweep = 0; sweep < pr->n_mom_sweeps; ++sweep) {
            for (int d = 0; d < 3; ++d) {
                mom_offdiag(s, fm, divfm, ucur[d], noff, tface, tlap);
                for (size_t P = 0; P < N; ++P)
                    unew[d][P] = (src[d][P] - noff[P] - gpn[d][P]) / aP[P];
            }
            for (int d = 0; d < 3; ++d) {
                double* tmp = ucur[d];
                ucur[d] = unew[d];
                unew[d] = tmp;
            }
        }
    }

    if (s->capture)
        for (int d = 0; d < 3; ++d) keep(&s->sys_ustar[d], N, ucur[d]);

    /* ---- 4b. Fourier closure: energy predictor.  The internal energy
     * e = c_v T of the gas, backward Euler with the old mass fluxes (the
     * momentum predictor's discretisation: I4 convection split into the
     * diagonal (9/16) div(phi) and the rest, compact Laplacian for the heat
     * flux q = -kappa grad T):
     *   c_v [(rho* T - rho^n T^n)/dt + div(phi^n I4(T))] = -p^n div(u^n) + kappa Lap(T),
     * solved by the same number of Jacobi sweeps from T^n.  The correctors
     * then use p = rho R T* and psi = d rho / d p = 1/(R T*). ---- */
    double* Ts = NULL;
    if (fourier) {
        const double cv = pr->cv, kap = pr->kappa;
        NEWF(aT);
        NEWF(sT);
        NEWF(toff);
        for (size_t P = 0; P < N; ++P) {
            aT[P] = cv * (rhos[P] / dt + (9.0 / 16.0) * divphi[P]) + 6.0 * kap / (h * h);
            sT[P] = cv * s->rho[P] * s->T[P] / dt - pn[P] * divu[P];
        }
        double* tcur = pool_get(s, slot++);
        double* tnew = pool_get(s, slot++);
        memcpy(tcur, s->T, N * sizeof(double));
        for (int sweep = 0; sweep < pr->n_mom_sweeps; ++sweep) {
            /* c_v times the convective off-diagonal part, minus the conduction's */
            for (int d = 0; d < 3; ++d) {
                ora_i4(n, d, tcur, tface[d]);
                for (size_t P = 0; P < N; ++P) tface[d][P] *= s->phi[d][P];
            }
            ora_div_flux(n, tface[0], tface[1], tface[2], toff);
            ora_lap(n, tcur, tlap);
            for (size_t P = 0; P < N; ++P) {
                double off = cv * (toff[P] - (9.0 / 16.0) * divphi[P] * tcur[P]) -
                             kap * (tlap[P] + 6.0 * tcur[P] / (h * h));
                tnew[P] = (sT[P] - off) / aT[P];
            }
            double* tmp = tcur;
            tcur = tnew;
            tnew = tmp;
        }
        Ts = tcur;
    }

    /* ---- 5. PISO correctors ---- */
    NEWF(rhok);
    memcpy(rhok, rhos, N * sizeof(double));
    NEWF(p0); NEWF(psidt); NEWF(w); NEWF(b); NEWF(x); NEWF(pk); NEWF(diag);
    NEWF(hb0); NEWF(hb1); NEWF(hb2);
    double* hbya[3] = {hb0, hb1, hb2};
    NEWF(ph0); NEWF(ph1); NEWF(ph2);
    double* phiH[3] = {ph0, ph1, ph2};
    NEWF(kf0); NEWF(kf1); NEWF(kf2);
    double* Kf[3] = {kf0, kf1, kf2};
    NEWF(fa0); NEWF(fa1); NEWF(fa2);
    double* fa[3] = {fa0, fa1, fa2};
    NEWF(ir); NEWF(ih); NEWF(sg); NEWF(dv);
    double* phin[3];
    for (int d = 0; d < 3; ++d) phin[d] = pool_get(s, slot++);

    for (int corr = 0; corr < pr->n_corr; ++corr) {
        /* 5.1 pressure and compressibility of the current density iterate */
        for (size_t P = 0; P < N; ++P) {
            if (fourier) {
                p0[P] = rhok[P] * Rg * Ts[P];
                psidt[P] = 1.0 / (Rg * Ts[P]) / dt;
            } else {
                p0[P] = Cc * pow(rhok[P], g);
                psidt[P] = (bdf2 ? c0 : 1.0) / (g * Cc * pow(rhok[P], g - 1.0)) / dt;
            }
        }
        /* 5.2 HbyA = H(u)/a_P with H(u) = s - N(u) */
        for (int d = 0; d < 3; ++d) {
            mom_offdiag(s, fm, divfm, ucur[d], noff, tface, tlap);
            for (size_t P = 0; P < N; ++P) hbya[d][P] = (src[d][P] - noff[P]) / aP[P];
        }
        /* 5.3-5.5 predicted fluxes, face coefficients, continuity defect */
        for (size_t P = 0; P < N; ++P) w[P] = rhok[P] / aP[P];
        ora_kfaces(n, w, Kf[0], Kf[1], Kf[2]);
        for (int d = 0; d < 3; ++d) {
            ora_i4(n, d, rhok, ir);
            ora_i4(n, d, hbya[d], ih);
            ora_sngrad(n, d, p0, sg);
            for (size_t P = 0; P < N; ++P) {
                phiH[d][P] = ir[P] * ih[P] * A;
                fa[d][P] = phiH[d][P] - Kf[d][P] * A * sg[P];
                if (!(Kf[d][P] > 0.0)) flags |= ORA_FLAG_KFACE_NONPOS;
            }
        }
        ora_div_flux(n, fa[0], fa[1], fa[2], dv);
        if (bdf2)
            for (size_t P = 0; P < N; ++P)
                b[P] = -((c0 * rhok[P] - c1 * s->rho[P] + c2 * s->rho_m1[P]) / dt + dv[P]);
        else
            for (size_t P = 0; P < N; ++P) b[P] = -((rhok[P] - s->rho[P]) / dt + dv[P]);
        /* 5.6-5.7 solve M p' = b from p' = 0 */
        memset(x, 0, N * sizeof(double));
        double relres = 0.0;
        int32_t it = ora_pcg(n, psidt, Kf[0], Kf[1], Kf[2], b, x, pr->p_tol, pr->p_maxit, &relres);
        if (it < 0) {
            flags |= ORA_FLAG_PCG_MAXIT;
            status = ORA_WARN_NOT_CONVERGED;
            it = pr->p_maxit;
        }
        info->pcg_iters[corr] = it;
        info->pcg_relres[corr] = relres;
        if (s->capture) {
            const double* Kc[3] = {Kf[0], Kf[1], Kf[2]};
            helm_diag(n, psidt, Kc, diag);
            keep(&s->sys_b[corr], N, b);
            keep(&s->sys_w[corr], N, w);
            keep(&s->sys_psidt[corr], N, psidt);
            for (int d = 0; d < 3; ++d) keep(&s->sys_k[corr][d], N, Kf[d]);
            keep(&s->sys_x[corr], N, x);
            keep(&s->sys_p0[corr], N, p0);
            keep(&s->sys_diag[corr], N, diag);
        }
        /* 5.8-5.11 pressure, flux correction, conservative density, velocity */
        for (size_t P = 0; P < N; ++P) pk[P] = p0[P] + x[P];
        for (int d = 0; d < 3; ++d) {
            ora_sngrad(n, d, pk, sg);
            for (size_t P = 0; P < N; ++P) phin[d][P] = phiH[d][P] - Kf[d][P] * A * sg[P];
        }
        ora_div_flux(n, phin[0], phin[1], phin[2], dv);
        if (bdf2)
            for (size_t P = 0; P < N; ++P)
                rhok[P] = (c1 * s->rho[P] - c2 * s->rho_m1[P] - dt * dv[P]) / c0;
        else
            for (size_t P = 0; P < N; ++P) rhok[P] = s->rho[P] - dt * dv[P];
        ora_grad(n, pk, tface[0], tface[1], tface[2]);
        for (int d = 0; d < 3; ++d)
            for (size_t P = 0; P < N; ++P) ucur[d][P] = hbya[d][P] - tface[d][P] / aP[P];
    }

    /* ---- 7. Equilibrium-Eulerian dust, one class at a time ---- */
    int fd_slot = -1;
    double* rpn[ORA_MAX_CLASSES] = {0};
    if (pr->n_classes > 0) {
        /* particle-velocity correction source: a = Du/Dt, backward-Euler time
         * derivative plus (u.grad)u with Gauss-I4 gradients of u^{n+1} */
        double* acc[3];
        double* gu[3][3];
        for (int d = 0; d < 3; ++d) {
            acc[d] = pool_get(s, slot++);
            for (int e = 0; e < 3; ++e) gu[d][e] = pool_get(s, slot++);
            ora_grad(n, ucur[d], gu[d][0], gu[d][1], gu[d][2]);
        }
        for (int d = 0; d < 3; ++d)
            for (size_t P = 0; P < N; ++P) {
                double conv = 0.0;
                for (int e = 0; e < 3; ++e) conv += ucur[e][P] * gu[d][e][P];
                acc[d][P] = (bdf2 ? c0 * ucur[d][P] - c1 * s->u[d][P] + c2 * s->u_m1[d][P]
                                  : ucur[d][P] - s->u[d][P]) / dt + conv;
            }
        /* class-independent face factor D_d = I4(rho^{n+1}) (I4(a_d) - g_d) A:
         * the drift u_j - u = tau_j (g - Du/Dt) at the faces */
        double* Dfa[3];
        for (int d = 0; d < 3; ++d) {
            Dfa[d] = pool_get(s, slot++);
            ora_i4(n, d, rhok, ir);
            ora_i4(n, d, acc[d], ih);
            for (size_t P = 0; P < N; ++P) Dfa[d][P] = ir[P] * (ih[P] - pr->gravity[d]) * A;
        }
        double* fdn[3] = {NULL, NULL, NULL};   /* two-way: the dust mass fluxes of this step */
        if (pr->two_way) {
            fd_slot = slot;
            for (int d = 0; d < 3; ++d) fdn[d] = pool_get(s, slot++);
        }
        NEWF(G0); NEWF(G1); NEWF(G2);
        double* G[3] = {G0, G1, G2};
        NEWF(divG); NEWF(Y); NEWF(Yn); NEWF(ry);
        for (int c = 0; c < pr->n_classes; ++c) {
            double tau = pr->tau_p[c];
            const double* rj = s->rho_p[c];
            /* particle mass flux per unit mass ratio: u_p = u - tau a at the faces */
            for (int d = 0; d < 3; ++d)
                for (size_t P = 0; P < N; ++P) G[d][P] = phin[d][P] - tau * Dfa[d][P];
            ora_div_flux(n, G[0], G[1], G[2], divG);
            /* the dust's Courant number, as the gas's with G in place of phi */
            for (int k = 0; k < n; ++k)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        const size_t P = cell(n, i, j, k);
                        double f = 0.0;
                        for (int d = 0; d < 3; ++d)
                            f += fabs(G[d][P]) + fabs(G[d][shifted(n, i, j, k, d, -1)]);
                        const double cd = f / (2.0 * rhok[P] * V) * dt;
                        if (cd > info->courant_dust) info->courant_dust = cd;
                    }
            /* the diagonal of the implicit equation below must stay positive */
            for (size_t P = 0; P < N; ++P)
                if (!((bdf2 ? c0 : 1.0) * rhok[P] / dt + (9.0 / 16.0) * divG[P] > 0.0))
                    flags |= ORA_FLAG_DUST_DIAG;
            for (size_t P = 0; P < N; ++P) Y[P] = rj[P] / s->rho[P];
            /* implicit Euler for rho Y: Jacobi sweeps */
            for (int sweep = 0; sweep < pr->n_dust_sweeps; ++sweep) {
                for (int d = 0; d < 3; ++d) {
                    ora_i4(n, d, Y, tface[d]);
                    for (size_t P = 0; P < N; ++P) tface[d][P] *= G[d][P];
                }
                ora_div_flux(n, tface[0], tface[1], tface[2], ry);
                for (size_t P = 0; P < N; ++P) {
                    double off = ry[P] - (9.0 / 16.0) * divG[P] * Y[P];
                    if (bdf2)
                        Yn[P] = ((c1 * rj[P] - c2 * s->rho_p_m1[c][P]) / dt - off) /
                                (c0 * rhok[P] / dt + (9.0 / 16.0) * divG[P]);
                    else
                        Yn[P] = (rj[P] / dt - off) / (rhok[P] / dt + (9.0 / 16.0) * divG[P]);
                }
                double* tmp = Y;
                Y = Yn;
                Yn = tmp;
            }
            /* conservative finish with the face fluxes of the last iterate */
            for (int d = 0; d < 3; ++d) {
                ora_i4(n, d, Y, tface[d]);
                for (size_t P = 0; P < N; ++P) tface[d][P] *= G[d][P];
                if (pr->two_way)
                    for (size_t P = 0; P < N; ++P)
                        fdn[d][P] = (c == 0 ? 0.0 : fdn[d][P]) + tface[d][P];
            }
            ora_div_flux(n, tface[0], tface[1], tface[2], ry);
            rpn[c] = pool_get(s, slot++);
            for (size_t P = 0; P < N; ++P) {
                rpn[c][P] = bdf2 ? (c1 * rj[P] - c2 * s->rho_p_m1[c][P] - dt * ry[P]) / c0
                                 : rj[P] - dt * ry[P];
                if (!isfinite(rpn[c][P])) flags |= ORA_FLAG_DUST_NONFINITE;
                else if (rpn[c][P] < 0.0) flags |= ORA_FLAG_DUST_NEG;
            }
        }
    }

    /* ---- checks and commit ---- */
    double m_gas = sum_field(n, rhok) * V;
    double usq = dot_field(n, ucur[0], ucur[0]) + dot_field(n, ucur[1], ucur[1]) +
                 dot_field(n, ucur[2], ucur[2]);
    double rmin = INFINITY;
    for (size_t P = 0; P < N; ++P)
        if (rhok[P] < rmin) rmin = rhok[P];
    if (!isfinite(m_gas) || !isfinite(usq)) flags |= ORA_FLAG_NONFINITE;
    if (fourier && !isfinite(sum_field(n, Ts))) flags |= ORA_FLAG_NONFINITE;
    if (!(rmin > 0.0)) flags |= ORA_FLAG_RHO_NONPOS;
    info->dt = dt;
    info->courant = sigma * dt;
    info->flags = flags;
    info->mass_gas = m_gas;
    if (!(info->courant_dust < ORA_DUST_COURANT_MAX) && pr->n_classes > 0)
        flags |= ORA_FLAG_DUST_COURANT;
    info->flags = flags;
    if (flags & (ORA_FLAG_NONFINITE | ORA_FLAG_RHO_NONPOS | ORA_FLAG_DUST_NONFINITE)) {
        status = ORA_ERR_DIVERGED;
    } else {
        if ((flags & (ORA_FLAG_DUST_NEG | ORA_FLAG_DUST_DIAG | ORA_FLAG_DUST_COURANT)) &&
            status == ORA_OK)
            status = ORA_WARN_DUST;
        if (bdf2) {   /* t^n becomes t^{n-1} */
            memcpy(s->rho_m1, s->rho, N * sizeof(double));
            for (int d = 0; d < 3; ++d) memcpy(s->u_m1[d], s->u[d], N * sizeof(double));
            for (int c = 0; c < pr->n_classes; ++c)
                memcpy(s->rho_p_m1[c], s->rho_p[c], N * sizeof(double));
        }
        memcpy(s->rho, rhok, N * sizeof(double));
        if (fourier) memcpy(s->T, Ts, N * sizeof(double));
        for (int d = 0; d < 3; ++d) {
            memcpy(s->u[d], ucur[d], N * sizeof(double));
            memcpy(s->phi[d], phin[d], N * sizeof(double));
        }
        for (int c = 0; c < pr->n_classes; ++c) {
            memcpy(s->rho_p[c], rpn[c], N * sizeof(double));
            info->mass_p[c] = sum_field(n, s->rho_p[c]) * V;
        }
        if (pr->two_way && fd_slot >= 0)
            for (int d = 0; d < 3; ++d)
                memcpy(s->fd[d], pool_get(s, fd_slot + d), N * sizeof(double));
        s->t += dt;
        s->dt_prev = dt;
    }
    info->t = s->t;

#undef NEWF
    return status;
}

int ora_step(ora_state* s, int32_t n_steps, ora_info* info) {
    if (!s || n_steps < 0) return ORA_ERR_INVALID;
    int worst = ORA_OK;
    for (int i = 0; i < n_steps; ++i) {
        ora_info local;
        int st = one_step(s, info ? &info[i] : &local);
        if (st < 0) return st;
        /* a solve that hit its cap outranks the dust warnings, as in the GPU library */
        if (st == ORA_WARN_NOT_CONVERGED || worst == ORA_WARN_NOT_CONVERGED)
            worst = ORA_WARN_NOT_CONVERGED;
        else if (st > worst)
            worst = st;
    }
    return worst;
}

/* ------------------------------------------------------------------------- */
/* outputs                                                                   */
/* ------------------------------------------------------------------------- */

int ora_get(const ora_state* s, int32_t which, int32_t corr, double* dst) {
    size_t N = s->N;
    if (corr < 0 || corr >= ORA_MAX_CORR) return ORA_ERR_INVALID;
    switch (which) {
        case ORA_RHO: memcpy(dst, s->rho, N * sizeof(double)); return ORA_OK;
        case ORA_U:
            for (int d = 0; d < 3; ++d) memcpy(dst + d * N, s->u[d], N * sizeof(double));
            return ORA_OK;
        case ORA_PHI:
            for (int d = 0; d < 3; ++d) memcpy(dst + d * N, s->phi[d], N * sizeof(double));
            return ORA_OK;
        case ORA_RHO_P:
            for (int c = 0; c < s->p.n_classes; ++c)
                memcpy(dst + c * N, s->rho_p[c], N * sizeof(double));
            return ORA_OK;
        case ORA_P:
            for (size_t P = 0; P < N; ++P)
                dst[P] = s->p.closure == ORA_FOURIER ? s->rho[P] * s->p.R_gas * s->T[P]
                                                     : s->p.C * pow(s->rho[P], s->p.gamma);
            return ORA_OK;
        case ORA_T:
            if (s->p.closure != ORA_FOURIER) return ORA_ERR_INVALID;
            memcpy(dst, s->T, N * sizeof(double));
            return ORA_OK;
        default: break;
    }
    const double* src = NULL;
    switch (which) {
        case ORA_SYS_B: src = s->sys_b[corr]; break;
        case ORA_SYS_W: src = s->sys_w[corr]; break;
        case ORA_SYS_PSIDT: src = s->sys_psidt[corr]; break;
        case ORA_SYS_X: src = s->sys_x[corr]; break;
        case ORA_SYS_P0: src = s->sys_p0[corr]; break;
        case ORA_SYS_DIAG: src = s->sys_diag[corr]; break;
        case ORA_SYS_USTAR:
            if (!s->sys_ustar[0]) return ORA_ERR_INVALID;
            for (int d = 0; d < 3; ++d) memcpy(dst + d * N, s->sys_ustar[d], N * sizeof(double));
            return ORA_OK;
        case ORA_SYS_K:
            if (!s->sys_k[corr][0]) return ORA_ERR_INVALID;
            for (int d = 0; d < 3; ++d) memcpy(dst + d * N, s->sys_k[corr][d], N * sizeof(double));
            return ORA_OK;
        default: return ORA_ERR_INVALID;
    }
    if (!src) return ORA_ERR_INVALID;
    memcpy(dst, src, N * sizeof(double));
    return ORA_OK;
}

/* Volume-averaged statistics (the paper's Figs. 1-2 quantities; their
 * definitions are not printed, so the usual ones are taken):
 * KE = <rho |u|^2 / 2>, enstrophy = <|curl u|^2 / 2> with Gauss-I4 derivatives,
 * density r.m.s. = sqrt(<(rho - <rho>)^2>) / <rho>, Mach r.m.s. =
 * sqrt(<|u|^2>) / c0 with c0^2 = gamma C <rho>^(gamma-1), particle
 * concentration variance = <(rho_j/<rho_j> - 1)^2>, masses = sum V. */
int ora_stats(const ora_state* s, double* out) {
    int n = s->n;
    size_t N = s->N;
    double invN = 1.0 / (double)N;
    for (int i = 0; i < ORA_N_STATS; ++i) out[i] = 0.0;
    double* t = alloc_field(N);
    double* gu[3][3];
    for (int d = 0; d < 3; ++d) {
        for (int e = 0; e < 3; ++e) gu[d][e] = alloc_field(N);
        ora_grad(n, s->u[d], gu[d][0], gu[d][1], gu[d][2]);
    }
    for (size_t P = 0; P < N; ++P) {
        double q = 0.0;
        for (int d = 0; d < 3; ++d) q += s->u[d][P] * s->u[d][P];
        t[P] = 0.5 * s->rho[P] * q;
    }
    out[ORA_STAT_KE] = sum_field(n, t) * invN;
    for (size_t P = 0; P < N; ++P) {
        double wx = gu[2][1][P] - gu[1][2][P];
        double wy = gu[0][2][P] - gu[2][0][P];
        double wz = gu[1][0][P] - gu[0][1][P];
        t[P] = 0.5 * (wx * wx + wy * wy + wz * wz);
    }
    out[ORA_STAT_ENSTROPHY] = sum_field(n, t) * invN;
    double rmean = sum_field(n, s->rho) * invN;
    for (size_t P = 0; P < N; ++P) t[P] = (s->rho[P] - rmean) * (s->rho[P] - rmean);
    out[ORA_STAT_RHO_RMS] = sqrt(sum_field(n, t) * invN) / rmean;
    for (size_t P = 0; P < N; ++P) {
        double q = 0.0;
        for (int d = 0; d < 3; ++d) q += s->u[d][P] * s->u[d][P];
        t[P] = q;
    }
    /* sound speed of the mean state: barotropic gamma C <rho>^(gamma-1); Fourier
     * (ideal gas) gamma' R <T> with gamma' = c_p/c_v = 1 + R/c_v */
    double c0;
    if (s->p.closure == ORA_FOURIER) {
        double tm = sum_field(n, s->T) * invN;
        c0 = sqrt((1.0 + s->p.R_gas / s->p.cv) * s->p.R_gas * tm);
    } else {
        c0 = sqrt(s->p.gamma * s->p.C * pow(rmean, s->p.gamma - 1.0));
    }
    out[ORA_STAT_MACH_RMS] = sqrt(sum_field(n, t) * invN) / c0;
    out[ORA_STAT_MASS_GAS] = rmean * (double)N * s->V;
    for (int c = 0; c < s->p.n_classes; ++c) {
        double m = sum_field(n, s->rho_p[c]) * invN;
        for (size_t P = 0; P < N; ++P) {
            double r = m != 0.0 ? s->rho_p[c][P] / m - 1.0 : 0.0;
            t[P] = r * r;
        }
        out[ORA_STAT_CONC_VAR + c] = sum_field(n, t) * invN;
        out[ORA_STAT_MASS_P + c] = m * (double)N * s->V;
    }
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) free(gu[d][e]);
    free(t);
    return ORA_OK;
}
