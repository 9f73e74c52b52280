// diag.hip -- diagnostics of the velocity field on gfx950: the energy
// spectrum and the Taylor micro-scale (through a radix-2 Stockham FFT done in
// LDS, one line per LDS row), and the second invariant Q of the velocity
// gradient.  These are the paper's validation quantities of the flow (Results
// section: energy spectrum, Taylor micro-scale; third figure: Q iso-surfaces).
//
// Filtered statistics: the separable top-hat of width 2h (weights 1/4, 1/2,
// 1/4 per axis), the sub-grid stress, its energy and the energy flux to the
// sub-grid scales (the a-priori tests the paper plans for its DNS data base).
//
// Spectrum: u_hat(k) = DFT(u)(k) / n^3 over integer wavevectors with
// components in [-n/2, n/2); shell s gathers the k with s - 1/2 <= |k| <
// s + 1/2, E(s) = sum over the shell of |u_hat|^2 / 2, so sum_s E(s) =
// <|u|^2>/2.  Taylor micro-scale lambda = sqrt(5 sum E / D) with D = sum_k
// |k|^2 |u_hat(k)|^2 / 2.  Every sum runs in a fixed order (bitwise
// reproducible): per row of wavevectors, per plane, then over the planes.
//
// Also here: the plain streaming kernel that measures the practical HBM
// ceiling of a given mix of reads and writes (no stencil, no reduction).
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdint>
#include <new>
#include <utility>

#include "../../include/pisoc.h"
#include "device.hpp"

namespace pisoc {
namespace {

using cplx = double2;

constexpr int kFftThreads = 256;
constexpr int kFftLds = 1024;        // complex values per LDS buffer (two buffers)

bool pow2(int n) { return n >= 8 && n <= 1024 && (n & (n - 1)) == 0; }
int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}
// lines per FFT block: the two LDS buffers hold L lines of n complex values
int fft_lines(int n) {
    int L = kFftLds / n;
    return L > n ? n : (L < 1 ? 1 : L);
}

// Shell of an integer |k|^2: s with s - 1/2 <= sqrt(k2) < s + 1/2, in integers
// ((s + 1/2)^2 <= k2 <=> k2 >= s^2 + s + 1 for integer k2).
__host__ __device__ inline int shell_of(int64_t k2) {
    int64_t s = (int64_t)sqrt((double)k2);
    while (s * s > k2) --s;
    while ((s + 1) * (s + 1) <= k2) ++s;
    return (int)(s + (k2 >= s * s + s + 1 ? 1 : 0));
}

// One FFT pass along axis AX (0 x, 1 y, 2 z) of the n^3 complex field f, in
// place: block b loads L whole lines into LDS, runs log2(n) radix-2 Stockham
// stages (stage with sub-transforms of size Ns: y[2(j - k) + k] = a + w b,
// y[2(j - k) + k + Ns] = a - w b, a = x[j], b = x[j + n/2], k = j mod Ns,
// w = exp(-i pi k / Ns)) and writes the lines back in natural order.  Along
// x the lines are rows (contiguous); along y and z a block takes L lines at
// consecutive x, so that each element's loads are L consecutive values.
// With re (pass x only) the input is the real field re, imaginary part 0.
template <int AX>
__global__ void __launch_bounds__(kFftThreads) k_fft_axis(cplx* f, const double* re, int n,
                                                         int logn, int L) {
    extern __shared__ cplx lds_fft[];
    cplx* A = lds_fft;
    cplx* B = lds_fft + L * n;
    cplx* W = lds_fft + 2 * L * n;   // twiddles exp(-2 pi i m / n), m < n/2
    const int tid = threadIdx.x;
    for (int m = tid; m < n / 2; m += kFftThreads) {
        double sn, cs;
        sincospi(-2.0 * (double)m / (double)n, &sn, &cs);
        W[m] = {cs, sn};
    }
    const size_t nn = (size_t)n * n;
    const int first = blockIdx.x * L;          // first line of the block
    auto addr = [&](int l, int e) -> size_t {
        if (AX == 0) {
            const int idx = first + l, j = idx % n, k = idx / n;
            return (size_t)e + (size_t)n * j + nn * k;
        }
        const int i0 = first % n, o = first / n;   // o: z (AX = 1) or y (AX = 2)
        if (AX == 1) return (size_t)(i0 + l) + (size_t)n * e + nn * o;
        return (size_t)(i0 + l) + (size_t)n * o + nn * e;
    };
    for (int t = tid; t < L * n; t += kFftThreads) {
        const int l = AX == 0 ? t / n : t % L;
        const int e = AX == 0 ? t % n : t / L;
        const size_t a = addr(l, e);
        A[l * n + e] = re ? cplx{re[a], 0.0} : f[a];
    }
    __syncthreads();
    const int half = n >> 1;
    for (int s = 0, Ns = 1; s < logn; ++s, Ns <<= 1) {
        for (int t = tid; t < L * half; t += kFftThreads) {
            const int l = t / half, j = t - l * half;
            const int k = j & (Ns - 1);
            // exp(-i pi k / Ns) = exp(-2 pi i (k n / (2 Ns)) / n)
            const cplx tw = W[k * (half / Ns)];
            const double cs = tw.x, sn = tw.y;
            const cplx a = A[l * n + j], x = A[l * n + j + half];
            const cplx wb = {x.x * cs - x.y * sn, x.x * sn + x.y * cs};
            const int base = l * n + 2 * (j - k) + k;
            B[base] = {a.x + wb.x, a.y + wb.y};
            B[base + Ns] = {a.x - wb.x, a.y - wb.y};
        }
        __syncthreads();
        cplx* t = A;
        A = B;
        B = t;
    }
    for (int t = tid; t < L * n; t += kFftThreads) {
        const int l = AX == 0 ? t / n : t % L;
        const int e = AX == 0 ? t % n : t / L;
        f[addr(l, e)] = A[l * n + e];
    }
}

// Signed wavenumber of DFT index i (components in [-n/2, n/2)).
__device__ inline int wavenumber(int i, int n) { return i < n / 2 ? i : i - n; }

// Shell binning of one component's transform f, in three fixed-order passes.
// 1. One thread per x-row of wavevectors (fixed ky, kz): walking kx in order of
//    |kx| (0, 1, -1, 2, -2, ..., -n/2) the shell index never decreases, so the
//    row's energies e = |f|^2 / (2 n^6) sum into runs, one per shell, written to
//    rowpart[row][s - s0] with s0 the shell of kx = 0 (W = n/2 + 2 entries per
//    row hold every shell the row reaches; shells it skips stay 0); rowd[row]
//    receives the row's sum of |k|^2 e.
__global__ void __launch_bounds__(kFftThreads) k_spectrum_rows(const cplx* f, int n, int W,
                                                             double inv_n6, double* rowpart,
                                                             double* rowd) {
    const size_t row = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= (size_t)n * n) return;
    const int ky = wavenumber((int)(row % n), n), kz = wavenumber((int)(row / n), n);
    const int64_t kyz = (int64_t)ky * ky + (int64_t)kz * kz;
    const int s0 = shell_of(kyz);
    double* out = rowpart + row * (size_t)W;
    for (int t = 0; t < W; ++t) out[t] = 0.0;
    const cplx* line = f + row * (size_t)n;
    int cur = s0;
    double acc = 0.0, dk = 0.0;
    for (int m = 0; m < n; ++m) {
        const int kx = m == 0 ? 0 : m == n - 1 ? -n / 2 : (m & 1) ? (m + 1) / 2 : -(m / 2);
        const cplx v = line[kx >= 0 ? kx : kx + n];
        const double e = 0.5 * (v.x * v.x + v.y * v.y) * inv_n6;
        const int64_t k2 = kyz + (int64_t)kx * kx;
        const int sh = shell_of(k2);
        if (sh != cur) {
            out[cur - s0] = acc;
            acc = 0.0;
            cur = sh;
        }
        acc += e;
        dk += (double)k2 * e;
    }
    out[cur - s0] = acc;
    rowd[row] = dk;
}

// 2. Per plane kz and shell s: the sum over the plane's rows in row order
//    (s = bins: the rows' |k|^2 e sums) into plane[kz * (bins + 1) + s].
__global__ void __launch_bounds__(64) k_spectrum_planes(const double* rowpart, const double* rowd,
                                                        int n, int W, int bins, double* plane) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int zi = blockIdx.y;
    if (s > bins) return;
    const int kz = wavenumber(zi, n);
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
        const size_t row = (size_t)j + (size_t)n * zi;
        if (s == bins) {
            acc += rowd[row];
            continue;
        }
        const int ky = wavenumber(j, n);
        const int t = s - shell_of((int64_t)ky * ky + (int64_t)kz * kz);
        if (t >= 0 && t < W) acc += rowpart[row * (size_t)W + t];
    }
    plane[(size_t)zi * (bins + 1) + s] = acc;
}

// 3. Totals over the planes (in plane order) and over the three components'
//    plane sets (in component order): out[s] = E(s), out[bins] = D.
__global__ void __launch_bounds__(kFftThreads) k_spectrum_total(const double* part, int nblk,
                                                              int bins, double* out) {
    const size_t set = (size_t)nblk * (bins + 1);
    for (int s = threadIdx.x; s <= bins; s += kFftThreads) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < nblk; ++b) acc += part[c * set + (size_t)b * (bins + 1) + s];
        out[s] = acc;
    }
}

// Q = -(1/2) sum_ij (d_j u_i)(d_i u_j) per cell with the Gauss-I4 cell
// derivative d_j q = (I4(q)_{P+1/2 e_j} - I4(q)_{P-1/2 e_j}) / h; partial sums
// of Q and of (d_i u_i)^2 (the discrete identity sum Q = -(1/2) sum (div u)^2
// holds for these antisymmetric, commuting difference operators).
__global__ void __launch_bounds__(kBlock) k_qcrit(int n, double inv_h, const double* __restrict__ u,
                                                  double* __restrict__ q, double* part) {
    const size_t N = (size_t)n * n * n;
    double v[2] = {0.0, 0.0};
    for (size_t P = (size_t)blockIdx.x * blockDim.x + threadIdx.x; P < N;
         P += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(P % n), j = (int)((P / n) % n), k = (int)(P / ((size_t)n * n));
        const CellIdx c(n, i, j, k, 0);
        double G[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double g[13];
            gather13(u + a * N, c, g);
#pragma unroll
            for (int b = 0; b < 3; ++b) G[a][b] = dgauss13(g, b, inv_h);
        }
        double Q = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Q -= 0.5 * G[a][b] * G[b][a];
        q[P] = Q;
        const double div = G[0][0] + G[1][1] + G[2][2];
        v[0] += Q;
        v[1] += div * div;
    }
    block_partials<2, 0u>(v, part);
}

__global__ void __launch_bounds__(kBlock) k_qcrit_total(const double* part, unsigned nb,
                                                        double* out) {
    double t[2];
    reduce_partials<2, 0u>(part, nb, t);
    if (flat_tid() == 0) {
        out[0] = t[0];
        out[1] = t[1];
    }
}

// Filtered (a-priori sub-grid) statistics: the separable top-hat of width 2h
// (weights 1/4, 1/2, 1/4 along each axis) of u_i and of u_i u_j, into nine
// fields F (u_bar x, y, z; bar(u u) xx, xy, xz, yy, yz, zz).
__global__ void __launch_bounds__(kBlock) k_sgs_filter(int n, const double* __restrict__ u,
                                                       double* __restrict__ F) {
    const size_t N = (size_t)n * n * n;
    for (size_t P = (size_t)blockIdx.x * blockDim.x + threadIdx.x; P < N;
         P += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(P % n), j = (int)((P / n) % n), k = (int)(P / ((size_t)n * n));
        const CellIdx c(n, i, j, k, 0);
        double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const double w = (dx ? 0.25 : 0.5) * (dy ? 0.25 : 0.5) * (dz ? 0.25 : 0.5);
                    const size_t Q = c.self() + (size_t)(ptrdiff_t)(c.off[0][dx + 2] +
                                                                    c.off[1][dy + 2] +
                                                                    c.off[2][dz + 2]);
                    const double a = u[Q], b = u[N + Q], e = u[2 * N + Q];
                    acc[0] += w * a;
                    acc[1] += w * b;
                    acc[2] += w * e;
                    acc[3] += w * a * a;
                    acc[4] += w * a * b;
                    acc[5] += w * a * e;
                    acc[6] += w * b * b;
                    acc[7] += w * b * e;
                    acc[8] += w * e * e;
                }
#pragma unroll
        for (int f = 0; f < 9; ++f) F[f * N + P] = acc[f];
    }
}

// Per cell tau_ij = bar(u_i u_j) - u_bar_i u_bar_j, k_sgs = tau_ii / 2,
// S_bar_ij = (d_j u_bar_i + d_i u_bar_j) / 2 (Gauss-I4), Pi = -tau_ij S_bar_ij;
// partial sums of |u_bar|^2 / 2, k_sgs, Pi and of the cells with Pi < 0.
__global__ void __launch_bounds__(kBlock) k_sgs_stats(int n, double inv_h,
                                                      const double* __restrict__ F,
                                                      double* part) {
    const size_t N = (size_t)n * n * n;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t P = (size_t)blockIdx.x * blockDim.x + threadIdx.x; P < N;
         P += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(P % n), j = (int)((P / n) % n), k = (int)(P / ((size_t)n * n));
        const CellIdx c(n, i, j, k, 0);
        double G[3][3], ub[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double g[13];
            gather13(F + a * N, c, g);
            ub[a] = g[0];
#pragma unroll
            for (int b = 0; b < 3; ++b) G[a][b] = dgauss13(g, b, inv_h);
        }
        // bar(u u) in the order xx, xy, xz, yy, yz, zz
        const int slot[3][3] = {{3, 4, 5}, {4, 6, 7}, {5, 7, 8}};
        double ks = 0.0, pi = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double tau = F[slot[a][b] * N + P] - ub[a] * ub[b];
                if (a == b) ks += 0.5 * tau;
                pi -= tau * 0.5 * (G[a][b] + G[b][a]);
            }
        v[0] += 0.5 * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
        v[1] += ks;
        v[2] += pi;
        v[3] += pi < 0.0 ? 1.0 : 0.0;
    }
    block_partials<4, 0u>(v, part);
}

__global__ void __launch_bounds__(kBlock) k_sgs_total(const double* part, unsigned nb,
                                                      double* out) {
    double t[4];
    reduce_partials<4, 0u>(part, nb, t);
    if (flat_tid() == 0)
        for (int c = 0; c < 4; ++c) out[c] = t[c];
}

constexpr unsigned kQBlocks = 2048;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace: complex field, per-component plane partials, totals.
struct DiagLayout {
    size_t field, part, total_out, qpart, bytes;
};
DiagLayout diag_layout(int n) {
    DiagLayout d{};
    const size_t N = (size_t)n * n * n;
    const int bins = shell_of(3LL * (n / 2) * (n / 2)) + 1;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = align256(off + b);
        return o;
    };
    // the spectrum's complex field or the nine filtered fields (never both at once)
    // (the spectrum's row sums follow its complex field inside the same region)
    d.field = take(sizeof(double) * 9 * N);
    d.part = take(sizeof(double) * 3 * (size_t)n * (bins + 1));
    d.total_out = take(sizeof(double) * (bins + 1));
    d.qpart = take(sizeof(double) * (4 * kQBlocks + 16));
    d.bytes = off;
    return d;
}

// Streaming probe: out_w[i] = (w + 1) * (in_0[i] + ... + in_{R-1}[i]) over
// 16-byte vectors, a flat grid walking the arrays with a grid stride,
// non-temporal loads and stores (as the step's kernels stream their fields).
constexpr int kStreamThreads = 256, kStreamBlocks = 16384;
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kStreamMaxReads = 12, kStreamMaxWrites = 8;
struct StreamPtrs {
    const f4v* in[kStreamMaxReads];
    f4v* out[kStreamMaxWrites];
};

template <int R, int W>
__global__ void __launch_bounds__(kStreamThreads) k_stream(StreamPtrs p, size_t n4) {
    const size_t stride = (size_t)gridDim.x * kStreamThreads;
    for (size_t i = (size_t)blockIdx.x * kStreamThreads + threadIdx.x; i < n4; i += stride) {
        f4v a = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < R; ++r) a += __builtin_nontemporal_load(p.in[r] + i);
#pragma unroll
        for (int w = 0; w < W; ++w) __builtin_nontemporal_store(a * (float)(w + 1), p.out[w] + i);
    }
}

template <int R, int W>
void launch_stream_rw(dim3 g, hipStream_t s, const StreamPtrs& p, size_t n4) {
    hipLaunchKernelGGL((k_stream<R, W>), g, dim3(kStreamThreads), 0, s, p, n4);
}

// launchers of k_stream<R, W>, R = 1..kStreamMaxReads, W = 1..kStreamMaxWrites
using StreamLaunch = void (*)(dim3, hipStream_t, const StreamPtrs&, size_t);
template <int R, int... Ws>
constexpr std::array<StreamLaunch, sizeof...(Ws)> stream_row(std::integer_sequence<int, Ws...>) {
    return {{&launch_stream_rw<R, Ws + 1>...}};
}
template <int... Rs>
constexpr std::array<std::array<StreamLaunch, kStreamMaxWrites>, sizeof...(Rs)> stream_table(
    std::integer_sequence<int, Rs...>) {
    return {{stream_row<Rs + 1>(std::make_integer_sequence<int, kStreamMaxWrites>{})...}};
}
constexpr auto kStreamLaunch = stream_table(std::make_integer_sequence<int, kStreamMaxReads>{});

}  // namespace
}  // namespace pisoc

using namespace pisoc;

extern "C" {

int32_t pisoc_diag_spectrum_bins(int32_t n) {
    if (!pow2(n)) return 0;
    return shell_of(3LL * (n / 2) * (n / 2)) + 1;
}

size_t pisoc_diag_workspace_bytes(int32_t n) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N) return 0;
    return diag_layout(n).bytes;
}

pisoc_status pisoc_diag_spectrum(int32_t n, const double* d_u, double* h_E, int32_t nbins,
                                 double* h_taylor, double* h_dsum, void* d_ws, size_t ws_bytes,
                                 void* hip_stream) {
    if (!pow2(n) || !d_u || !h_E || nbins != pisoc_diag_spectrum_bins(n)) return PISOC_ERR_INVALID;
    const DiagLayout Ly = diag_layout(n);
    if (!d_ws || ws_bytes < Ly.bytes || (reinterpret_cast<uintptr_t>(d_ws) % 256) != 0)
        return PISOC_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    char* ws = reinterpret_cast<char*>(d_ws);
    cplx* f = reinterpret_cast<cplx*>(ws + Ly.field);
    double* part = reinterpret_cast<double*>(ws + Ly.part);
    double* tot = reinterpret_cast<double*>(ws + Ly.total_out);
    const size_t N = (size_t)n * n * n;
    const int L = fft_lines(n), logn = ilog2(n);
    const unsigned blocks = (unsigned)((size_t)n * n / L);
    const size_t lds = sizeof(cplx) * (2 * (size_t)L * n + n / 2);
    const double inv_n6 = 1.0 / ((double)N * (double)N);
    const int W = n / 2 + 2;
    double* rowpart = reinterpret_cast<double*>(ws + Ly.field + sizeof(cplx) * N);
    double* rowd = rowpart + (size_t)n * n * W;
    const size_t set = (size_t)n * (nbins + 1);
    const unsigned rowblocks = (unsigned)(((size_t)n * n + kFftThreads - 1) / kFftThreads);
    for (int c = 0; c < 3; ++c) {
        hipLaunchKernelGGL(k_fft_axis<0>, dim3(blocks), dim3(kFftThreads), lds, s, f, d_u + c * N,
                           n, logn, L);
        hipLaunchKernelGGL(k_fft_axis<1>, dim3(blocks), dim3(kFftThreads), lds, s, f, nullptr, n,
                           logn, L);
        hipLaunchKernelGGL(k_fft_axis<2>, dim3(blocks), dim3(kFftThreads), lds, s, f, nullptr, n,
                           logn, L);
        hipLaunchKernelGGL(k_spectrum_rows, dim3(rowblocks), dim3(kFftThreads), 0, s, f, n, W,
                           inv_n6, rowpart, rowd);
        hipLaunchKernelGGL(k_spectrum_planes, dim3((nbins + 64) / 64, n), dim3(64), 0, s, rowpart,
                           rowd, n, W, nbins, part + c * set);
    }
    hipLaunchKernelGGL(k_spectrum_total, dim3(1), dim3(kFftThreads), 0, s, part, n, nbins, tot);
    if (hipGetLastError() != hipSuccess) return PISOC_ERR_HIP;
    // the totals come back through pageable memory after the stream has drained
    if (hipStreamSynchronize(s) != hipSuccess) return PISOC_ERR_HIP;
    double* host = new (std::nothrow) double[nbins + 1];
    if (!host) return PISOC_ERR_INVALID;
    const bool ok = hipMemcpy(host, tot, sizeof(double) * (nbins + 1), hipMemcpyDeviceToHost) ==
                    hipSuccess;
    if (ok) {
        double e = 0.0;
        for (int b = 0; b < nbins; ++b) {
            h_E[b] = host[b];
            e += host[b];
        }
        const double D = host[nbins];
        if (h_taylor) *h_taylor = D > 0.0 ? std::sqrt(5.0 * e / D) : 0.0;
        if (h_dsum) *h_dsum = D;
    }
    delete[] host;
    return ok ? PISOC_OK : PISOC_ERR_HIP;
}

pisoc_status pisoc_diag_qcrit(int32_t n, const double* d_u, double* d_q, double* h_means,
                              void* d_ws, size_t ws_bytes, void* hip_stream) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_u || !d_q) return PISOC_ERR_INVALID;
    const DiagLayout Ly = diag_layout(n);
    if (!d_ws || ws_bytes < Ly.bytes || (reinterpret_cast<uintptr_t>(d_ws) % 256) != 0)
        return PISOC_ERR_WORKSPACE;
    const size_t N = (size_t)n * n * n;
    double* qpart = reinterpret_cast<double*>(reinterpret_cast<char*>(d_ws) + Ly.qpart);
    double* out = qpart + 2 * kQBlocks;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const double inv_h = (double)n / 6.283185307179586476925286766559;
    hipLaunchKernelGGL(k_qcrit, dim3(kQBlocks), dim3(kBlock), 0, s, n, inv_h, d_u, d_q, qpart);
    if (!h_means) return hipGetLastError() == hipSuccess ? PISOC_OK : PISOC_ERR_HIP;
    hipLaunchKernelGGL(k_qcrit_total, dim3(1), dim3(kBlock), 0, s, qpart, kQBlocks, out);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return PISOC_ERR_HIP;
    double t[2];
    if (hipMemcpy(t, out, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess) return PISOC_ERR_HIP;
    h_means[0] = t[0] / (double)N;
    h_means[1] = t[1] / (double)N;
    return PISOC_OK;
}

pisoc_status pisoc_diag_sgs(int32_t n, const double* d_u, double* h_out, void* d_ws,
                            size_t ws_bytes, void* hip_stream) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_u || !h_out) return PISOC_ERR_INVALID;
    const DiagLayout Ly = diag_layout(n);
    if (!d_ws || ws_bytes < Ly.bytes || (reinterpret_cast<uintptr_t>(d_ws) % 256) != 0)
        return PISOC_ERR_WORKSPACE;
    const size_t N = (size_t)n * n * n;
    char* ws = reinterpret_cast<char*>(d_ws);
    double* F = reinterpret_cast<double*>(ws + Ly.field);
    double* part = reinterpret_cast<double*>(ws + Ly.qpart);
    double* out = part + 4 * kQBlocks;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const double inv_h = (double)n / 6.283185307179586476925286766559;
    hipLaunchKernelGGL(k_sgs_filter, dim3(kQBlocks), dim3(kBlock), 0, s, n, d_u, F);
    hipLaunchKernelGGL(k_sgs_stats, dim3(kQBlocks), dim3(kBlock), 0, s, n, inv_h, F, part);
    hipLaunchKernelGGL(k_sgs_total, dim3(1), dim3(kBlock), 0, s, part, kQBlocks, out);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return PISOC_ERR_HIP;
    double t[4];
    if (hipMemcpy(t, out, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess) return PISOC_ERR_HIP;
    for (int c = 0; c < 4; ++c) h_out[c] = t[c] / (double)N;
    return PISOC_OK;
}

pisoc_status pisoc_stream_probe(int32_t reads, int32_t writes, int64_t count,
                                const float* const* h_in, float* const* h_out, int32_t blocks,
                                void* hip_stream) {
    if (reads < 1 || reads > kStreamMaxReads || writes < 1 || writes > kStreamMaxWrites || count < 0 ||
        count % 4 != 0 ||
        blocks < 0)
        return PISOC_ERR_INVALID;
    if (count == 0) return PISOC_OK;
    if (!h_in || !h_out) return PISOC_ERR_INVALID;
    StreamPtrs p{};
    for (int r = 0; r < reads; ++r) {
        if (!h_in[r] || reinterpret_cast<uintptr_t>(h_in[r]) % 16 != 0) return PISOC_ERR_INVALID;
        p.in[r] = reinterpret_cast<const f4v*>(h_in[r]);
    }
    for (int w = 0; w < writes; ++w) {
        if (!h_out[w] || reinterpret_cast<uintptr_t>(h_out[w]) % 16 != 0) return PISOC_ERR_INVALID;
        p.out[w] = reinterpret_cast<f4v*>(h_out[w]);
    }
    const size_t n4 = (size_t)count / 4;
    const dim3 g((unsigned)(blocks > 0 ? blocks : kStreamBlocks));
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    kStreamLaunch[reads - 1][writes - 1](g, s, p, n4);
    return hipGetLastError() == hipSuccess ? PISOC_OK : PISOC_ERR_HIP;
}

}  // extern "C"
