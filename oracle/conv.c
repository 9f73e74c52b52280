/* conv.c -- FP64 CPU oracle of the learned pressure-guess network (test
 * infrastructure only; shares no code with the GPU kernels).
 *
 * The network: four periodic 3x3x3 convolutions with 2 -> 16 -> 16 -> 16 -> 1
 * channels, ReLU after the first three, no biases.  Convention (cross-
 * correlation):
 *   out[co](x) = sum_ci sum_d W[co][ci][t(d)] in[ci](x + d),  d in {-1,0,1}^3,
 *   t(d) = (dz+1)*9 + (dy+1)*3 + (dx+1),
 * with periodic wrap.  Weights are layer-major, layer l stored as
 * [co][ci][27].  Activations are channel-last: a[b][cell][c], cell = i + n(j + n k).
 * The loss is the mean over batch and cells of (y - t)^2.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static const int kCh[5] = {2, 16, 16, 16, 1};

int32_t ora_conv_nweights(void) {
    int32_t s = 0;
    for (int l = 0; l < 4; ++l) s += kCh[l] * kCh[l + 1] * 27;
    return s;
}

static size_t woff(int l) {
    size_t s = 0;
    for (int m = 0; m < l; ++m) s += (size_t)kCh[m] * kCh[m + 1] * 27;
    return s;
}

static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

/* cell reached from (i,j,k) by tap t */
static inline size_t tap_cell(int n, int i, int j, int k, int t) {
    int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    return (size_t)wrap(i + dx, n) + (size_t)n * ((size_t)wrap(j + dy, n) + (size_t)n * wrap(k + dz, n));
}

/* one layer, forward: out[cell][co] = sum W in[cell + d][ci]; optional ReLU */
static void layer_fwd(int n, int cin, int cout, const double* W, const double* in, double* out,
                      int relu) {
    size_t N = (size_t)n * n * n;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t P = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * k);
                for (int co = 0; co < cout; ++co) {
                    double s = 0.0;
                    for (int ci = 0; ci < cin; ++ci)
                        for (int t = 0; t < 27; ++t)
                            s += W[((size_t)co * cin + ci) * 27 + t] * in[tap_cell(n, i, j, k, t) * cin + ci];
                    out[P * cout + co] = relu && s < 0.0 ? 0.0 : s;
                }
            }
    (void)N;
}

/* Forward pass: x [batch][n^3][2] -> y [batch][n^3]. */
int ora_conv_forward(int32_t n, int32_t batch, const double* w, const double* x, double* y) {
    size_t N = (size_t)n * n * n;
    double* a = (double*)malloc(sizeof(double) * N * 16);
    double* b = (double*)malloc(sizeof(double) * N * 16);
    for (int bi = 0; bi < batch; ++bi) {
        layer_fwd(n, 2, 16, w + woff(0), x + (size_t)bi * N * 2, a, 1);
        layer_fwd(n, 16, 16, w + woff(1), a, b, 1);
        layer_fwd(n, 16, 16, w + woff(2), b, a, 1);
        layer_fwd(n, 16, 1, w + woff(3), a, y + (size_t)bi * N, 0);
    }
    free(a);
    free(b);
    return 0;
}

/* Weight gradient of one layer: gW[co][ci][t] += sum_cells g[cell][co] in[cell+d][ci]. */
static void layer_gradw(int n, int cin, int cout, const double* in, const double* g, double* gW) {
    int nw = cin * cout * 27;
    double* part = (double*)calloc((size_t)n * nw, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        double* pk = part + (size_t)k * nw;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t P = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * k);
                for (int co = 0; co < cout; ++co) {
                    double gv = g[P * cout + co];
                    if (gv == 0.0) continue;
                    for (int ci = 0; ci < cin; ++ci)
                        for (int t = 0; t < 27; ++t)
                            pk[((size_t)co * cin + ci) * 27 + t] += gv * in[tap_cell(n, i, j, k, t) * cin + ci];
                }
            }
    }
    for (int k = 0; k < n; ++k)
        for (int q = 0; q < nw; ++q) gW[q] += part[(size_t)k * nw + q];
    free(part);
}

/* Input gradient of one layer: gin[cell'][ci] = sum_{co,t} W[co][ci][t] g[cell' - d(t)][co],
 * written as a scatter-free gather: the cell P receives from every P - d. */
static void layer_gradin(int n, int cin, int cout, const double* W, const double* g, double* gin) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                size_t P = (size_t)i + (size_t)n * ((size_t)j + (size_t)n * k);
                for (int ci = 0; ci < cin; ++ci) {
                    double s = 0.0;
                    for (int t = 0; t < 27; ++t) {
                        /* the cell Q with Q + d(t) = P */
                        int ft = 26 - t; /* d(ft) = -d(t) */
                        size_t Q = tap_cell(n, i, j, k, ft);
                        for (int co = 0; co < cout; ++co)
                            s += W[((size_t)co * cin + ci) * 27 + t] * g[Q * cout + co];
                    }
                    gin[P * cin + ci] = s;
                }
            }
}

/* Loss and weight gradient (15120 entries, summed over the batch). */
int ora_conv_backward(int32_t n, int32_t batch, const double* w, const double* x, const double* t,
                      double* grad_w, double* loss) {
    size_t N = (size_t)n * n * n;
    int nw = ora_conv_nweights();
    memset(grad_w, 0, sizeof(double) * nw);
    double* a1 = (double*)malloc(sizeof(double) * N * 16);
    double* a2 = (double*)malloc(sizeof(double) * N * 16);
    double* a3 = (double*)malloc(sizeof(double) * N * 16);
    double* y = (double*)malloc(sizeof(double) * N);
    double* g = (double*)malloc(sizeof(double) * N * 16);
    double* gin = (double*)malloc(sizeof(double) * N * 16);
    double total = 0.0;
    double scale = 2.0 / ((double)batch * (double)N);
    for (int bi = 0; bi < batch; ++bi) {
        const double* xb = x + (size_t)bi * N * 2;
        const double* tb = t + (size_t)bi * N;
        layer_fwd(n, 2, 16, w + woff(0), xb, a1, 1);
        layer_fwd(n, 16, 16, w + woff(1), a1, a2, 1);
        layer_fwd(n, 16, 16, w + woff(2), a2, a3, 1);
        layer_fwd(n, 16, 1, w + woff(3), a3, y, 0);
        for (size_t P = 0; P < N; ++P) {
            double d = y[P] - tb[P];
            total += d * d;
            g[P] = scale * d;
        }
        /* layer 4 (linear) */
        layer_gradw(n, 16, 1, a3, g, grad_w + woff(3));
        layer_gradin(n, 16, 1, w + woff(3), g, gin);
        for (size_t q = 0; q < N * 16; ++q) g[q] = a3[q] > 0.0 ? gin[q] : 0.0;
        /* layer 3 */
        layer_gradw(n, 16, 16, a2, g, grad_w + woff(2));
        layer_gradin(n, 16, 16, w + woff(2), g, gin);
        for (size_t q = 0; q < N * 16; ++q) g[q] = a2[q] > 0.0 ? gin[q] : 0.0;
        /* layer 2 */
        layer_gradw(n, 16, 16, a1, g, grad_w + woff(1));
        layer_gradin(n, 16, 16, w + woff(1), g, gin);
        for (size_t q = 0; q < N * 16; ++q) g[q] = a1[q] > 0.0 ? gin[q] : 0.0;
        /* layer 1 */
        layer_gradw(n, 2, 16, xb, g, grad_w + woff(0));
    }
    if (loss) *loss = total / ((double)batch * (double)N);
    free(a1);
    free(a2);
    free(a3);
    free(y);
    free(g);
    free(gin);
    return 0;
}

/* Weight gradient of sum_b sum_P dy[b][P] y[b][P] for a given output
 * gradient dy [batch][n^3]: back-propagation of any loss whose derivative with
 * respect to the network output is dy (summed over the batch). */
int ora_conv_backward_dy(int32_t n, int32_t batch, const double* w, const double* x, const double* dy,
                         double* grad_w) {
    size_t N = (size_t)n * n * n;
    int nw = ora_conv_nweights();
    memset(grad_w, 0, sizeof(double) * nw);
    double* a1 = (double*)malloc(sizeof(double) * N * 16);
    double* a2 = (double*)malloc(sizeof(double) * N * 16);
    double* a3 = (double*)malloc(sizeof(double) * N * 16);
    double* g = (double*)malloc(sizeof(double) * N * 16);
    double* gin = (double*)malloc(sizeof(double) * N * 16);
    for (int bi = 0; bi < batch; ++bi) {
        const double* xb = x + (size_t)bi * N * 2;
        layer_fwd(n, 2, 16, w + woff(0), xb, a1, 1);
        layer_fwd(n, 16, 16, w + woff(1), a1, a2, 1);
        layer_fwd(n, 16, 16, w + woff(2), a2, a3, 1);
        memcpy(g, dy + (size_t)bi * N, sizeof(double) * N);
        layer_gradw(n, 16, 1, a3, g, grad_w + woff(3));
        layer_gradin(n, 16, 1, w + woff(3), g, gin);
        for (size_t q = 0; q < N * 16; ++q) g[q] = a3[q] > 0.0 ? gin[q] : 0.0;
        layer_gradw(n, 16, 16, a2, g, grad_w + woff(2));
        layer_gradin(n, 16, 16, w + woff(2), g, gin);
        for (size_t q = 0; q < N * 16; ++q) g[q] = a2[q] > 0.0 ? gin[q] : 0.0;
        layer_gradw(n, 16, 16, a1, g, grad_w + woff(1));
        layer_gradin(n, 16, 16, w + woff(1), g, gin);
        for (size_t q = 0; q < N * 16; ++q) g[q] = a1[q] > 0.0 ? gin[q] : 0.0;
        layer_gradw(n, 2, 16, xb, g, grad_w + woff(0));
    }
    free(a1);
    free(a2);
    free(a3);
    free(g);
    free(gin);
    return 0;
}
