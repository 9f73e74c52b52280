/* guess.c -- FP64 oracle of the learned initial guess's two non-network
 * parts: the scaled network inputs of one pressure system, and the start of
 * the pressure solve from a guess (test infrastructure only; the network
 * itself is conv.c).
 *
 * Neither part is in the paper, which solves the pressure equation of each
 * PISO corrector (Results section) from zero.  The definitions followed here
 * are those stated for the learned guess: the inputs are the corrector's
 * Jacobi-scaled continuity defect b/diag(M) and the pressure p0 of the current
 * density iterate less its mean, each divided by its root mean square; the
 * solve starts from the multiple alpha g of the guess g that minimises the
 * energy norm of the error along g, alpha = g.b / g.(M g) (the first conjugate
 * gradient step along g), unless that start does not lower the residual norm,
 * ||b - alpha M g|| >= ||b||, in which case it starts from zero.
 *
 * Sums run sequentially in cell order, in FP64.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#include "oracle.h"

/* x[2P] = (b_P / diag_P) / s1, x[2P+1] = (p0_P - <p0>) / s2 with s1, s2 the
 * root mean squares of b/diag and of p0 - <p0> (a channel whose r.m.s. is 0
 * is left at 0).  scales[0] = s1, scales[1] = s2. */
int ora_net_inputs(int32_t n, const double* b, const double* diag, const double* p0, double* x,
                   double* scales) {
    if (n < 1 || !b || !diag || !p0 || !x || !scales) return ORA_ERR_INVALID;
    const size_t N = (size_t)n * n * n;
    double szz = 0.0, sp = 0.0;
    for (size_t P = 0; P < N; ++P) {
        const double z = b[P] / diag[P];
        szz += z * z;
        sp += p0[P];
    }
    const double mean = sp / (double)N;
    double sdd = 0.0;
    for (size_t P = 0; P < N; ++P) {
        const double d = p0[P] - mean;
        sdd += d * d;
    }
    const double s1 = sqrt(szz / (double)N), s2 = sqrt(sdd / (double)N);
    for (size_t P = 0; P < N; ++P) {
        x[2 * P] = s1 > 0.0 ? (b[P] / diag[P]) / s1 : 0.0;
        x[2 * P + 1] = s2 > 0.0 ? (p0[P] - mean) / s2 : 0.0;
    }
    scales[0] = s1;
    scales[1] = s2;
    return ORA_OK;
}

/* Start of the solve M x = b from the guess g (M from psi/dt and the face
 * coefficients k0..k2, as ora_helm_apply): alpha = g.b / g.(M g) (0 when
 * g.(M g) is not positive), x0 = alpha g; when ||b - M x0|| >= ||b|| the start
 * falls back to x0 = 0.  *alpha receives alpha, *res_ratio the ratio
 * ||b - M x0|| / ||b|| of the start that was rejected or taken (before the
 * fallback); returns 1 on a fallback, 0 otherwise, or ORA_ERR_INVALID. */
int ora_guess_start(int32_t n, const double* psidt, const double* k0, const double* k1,
                    const double* k2, const double* b, const double* g, double* x0, double* alpha,
                    double* res_ratio) {
    if (n < 1 || !psidt || !k0 || !k1 || !k2 || !b || !g || !x0) return ORA_ERR_INVALID;
    const size_t N = (size_t)n * n * n;
    double* mg = (double*)malloc(N * sizeof(double));
    if (!mg) return ORA_ERR_INVALID;
    ora_helm_apply(n, psidt, k0, k1, k2, g, mg);
    double gb = 0.0, gmg = 0.0;
    for (size_t P = 0; P < N; ++P) {
        gb += g[P] * b[P];
        gmg += g[P] * mg[P];
    }
    const double a = gmg > 0.0 ? gb / gmg : 0.0;
    double rr = 0.0, bb = 0.0;
    for (size_t P = 0; P < N; ++P) {
        const double r = b[P] - a * mg[P];
        rr += r * r;
        bb += b[P] * b[P];
    }
    free(mg);
    if (alpha) *alpha = a;
    if (res_ratio) *res_ratio = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    const int fallback = !(rr < bb);
    for (size_t P = 0; P < N; ++P) x0[P] = fallback ? 0.0 : a * g[P];
    return fallback;
}
