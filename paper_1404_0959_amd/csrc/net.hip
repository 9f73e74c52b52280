// net.hip -- the learned pressure-guess network on gfx950: four periodic
// 3x3x3 convolutions (2 -> 16 -> 16 -> 16 -> 1, ReLU after the first three, no
// biases) evaluated with BF16 operands and FP32 accumulation on the matrix
// cores (v_mfma_f32_16x16x32_bf16 in the forward 16 -> 16 layers,
// v_mfma_f32_16x16x16_bf16 elsewhere), plus the training kernels (data and
// weight gradients, MSE and residual losses, Adam) and the C ABI of the
// network.
//
// GEMM view of one layer: for 16 consecutive cells along x (one wavefront),
// D[cell][co] = sum over K of A[cell][k] B[k][co] with k = (tap, ci).  With 16
// input channels a K-block of 16 is one tap; with 4 (padded) input channels a
// K-block holds 4 taps.  Lane l loads 4 consecutive channels (8 bytes) of one
// neighbour cell, so activations are stored channel-last in BF16.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/pisoc.h"
#include "device.hpp"
#include "launch.hpp"
#include "net.hpp"

namespace pisoc {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline float bf2f(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__device__ inline int wrapn(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// FP32 -> BF16, round to nearest even, with gfx950's conversion instruction
// (v_cvt_pk_bf16_f32): the same rounding as f2bf for finite values, without
// its branch for NaN.
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ inline uint32_t bf16x2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{a, b}, v2bf));
}
__device__ inline uint16_t bf16x1(float a) { return __builtin_bit_cast(uint16_t, (__bf16)a); }

template <int CINP> constexpr int nkb() { return CINP == 16 ? 27 : 7; }

// (tap, channel) of entry kk (0..15) of K-block kb.
template <int CINP>
__host__ __device__ inline void kdecode(int kb, int kk, int& tap, int& ch) {
    if (CINP == 16) {
        tap = kb;
        ch = kk;
    } else {
        tap = 4 * kb + kk / 4;
        ch = kk % 4;
    }
}

// One convolution layer on a channel-last BF16 input with CINP channels.
// Output: BF16 [cell][16] (ReLU, or masked by mask > 0 for a data gradient), or
// with FINAL the FP32 channel 0 times yscale.
template <int CINP, bool FINAL>
__global__ void __launch_bounds__(256) k_conv(int n, int batch, const uint16_t* __restrict__ in,
                                              const v4s* __restrict__ wpk,
                                              const uint16_t* __restrict__ mask, int relu,
                                              uint16_t* __restrict__ out, float* __restrict__ yout,
                                              float yscale) {
    constexpr int NKB = nkb<CINP>();
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int segs = n / 16;
    const long nseg = (long)batch * n * n * segs;
    if (wave >= nseg) return;  // whole wavefront; no block barrier below
    const int iseg = (int)(wave % segs);
    long rest = wave / segs;
    const int j = (int)(rest % n);
    rest /= n;
    const int k = (int)(rest % n);
    const int b = (int)(rest / n);
    const size_t N = (size_t)n * n * n;
    const int m = lane & 15, g = lane >> 4;
    const int i = iseg * 16 + m;
    v4s B[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) B[kb] = wpk[kb * 64 + lane];
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
        const int tap = CINP == 16 ? kb : 4 * kb + g;
        v4s a = {0, 0, 0, 0};
        if (tap < 27) {
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const size_t cell = (size_t)wrapn(i + dx, n) +
                                (size_t)n * ((size_t)wrapn(j + dy, n) + (size_t)n * wrapn(k + dz, n));
            const int c0 = CINP == 16 ? 4 * g : 0;
            a = *reinterpret_cast<const v4s*>(in + ((size_t)b * N + cell) * CINP + c0);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, B[kb], acc, 0, 0, 0);
    }
    // lane holds D[4g + e][lane & 15]
    const int nn = lane & 15;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const size_t cell = (size_t)(iseg * 16 + 4 * g + e) + (size_t)n * ((size_t)j + (size_t)n * k);
        const size_t P = (size_t)b * N + cell;
        float v = acc[e];
        if (FINAL) {
            if (nn == 0) yout[P] = v * yscale;
        } else {
            if (mask) {
                const uint16_t mb = mask[P * 16 + nn];
                if (!((mb & 0x7fffu) != 0 && (mb & 0x8000u) == 0)) v = 0.f;
            } else if (relu) {
                v = v > 0.f ? v : 0.f;
            }
            out[P * 16 + nn] = bf16x1(v);
        }
    }
}

// Every layer marches along z: a wavefront owns 16 cells along x times kRY
// rows along y and walks a chunk of output planes.
constexpr int kRY = 4;

// The 16 -> 16 layers run on gfx950's K = 32 product
// (v_mfma_f32_16x16x32_bf16, twice the work of the K = 16 form per issue).
// Within one input plane the (kRY + 2) x 3 (row, x shift) items r = 3 iy + q
// are taken two at a time: pair p holds item 2p in lane groups 0-1 and item
// 2p + 1 in groups 2-3, 8 channels (16 bytes) of one cell per lane.  Output row
// oy reads items 3 oy .. 3 oy + 8, the 5 pairs from floor(3 oy / 2) on, whose
// weight operand depends only on the parity c of oy, the pair's slot s in that
// run and dz: 30 operands, held in registers.  60 products per output plane of
// 16 x kRY cells (108 with K = 16), 10 % of their entries the zero halves at
// the ends of odd and even runs.
constexpr int kItems = 3 * (kRY + 2), kPairs = kItems / 2, kSlots = 5;
static_assert(kItems % 2 == 0, "items pair up within a plane");

__device__ inline v4f mfma_k32(v8s a, v8s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// The 16 -> 16 layer as a z-march.  A wavefront owns 16 cells along x times
// kRY rows along y and walks a chunk of ZC output planes: input plane by input
// plane (ZC + 2 of them, each loaded once, 9 pair items of 16 bytes per
// lane), it issues the products of the three output planes the input plane
// reaches (dz = -1, 0, 1) into a ring of three planes of accumulators, and
// stores an output plane once its last input plane (dz = +1) is done.  The
// weight operands are loaded once per wavefront; each item of the next input
// plane is loaded into its register right after the item's last product, so
// a whole plane of products covers the load.  The plane loop is unrolled in
// full (ZC a template parameter), so that every ring slot and edge test is a
// constant and the loads stay in flight across planes (with run-time tests the
// compiler drained them at every branch: 1.65 against 1.12 ms for the
// network at 256^3).  Against one wavefront per 16 x 4 x 4 tile, which
// reread 6 input planes per 4 output planes and reloaded the weights per
// tile, the layer takes about 290 instead of 480 us at 256^3.
__device__ inline void store_plane_rows(const v4f (&acc)[kRY], uint16_t* __restrict__ out, int n,
                                        int x, int j0, int kz, int g, int relu) {
#pragma unroll
    for (int oy = 0; oy < kRY; ++oy) {
        const size_t cell = (size_t)x + (size_t)n * ((size_t)(j0 + oy) + (size_t)n * kz);
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float a = acc[oy][e];
            v[e] = relu && !(a > 0.f) ? 0.f : a;
        }
        uint2 q;
        q.x = bf16x2(v[0], v[1]);
        q.y = bf16x2(v[2], v[3]);
        *reinterpret_cast<uint2*>(out + cell * 16 + 4 * g) = q;
    }
}

template <int ZC>
__global__ void __launch_bounds__(256, 2) k_conv16_zm(int n, int batch,
                                                      const uint16_t* __restrict__ in,
                                                      const v8s* __restrict__ wpp, int relu,
                                                      uint16_t* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int segs = n / 16, nyb = n / kRY, nzc = n / ZC;
    const long nwaves = (long)batch * nzc * nyb * segs;
    if (wave >= nwaves) return;  // whole wavefront; no block barrier below
    const int iseg = (int)(wave % segs);
    long rest = wave / segs;
    const int j0 = (int)(rest % nyb) * kRY;
    rest /= nyb;
    const int k0 = (int)(rest % nzc) * ZC;
    const int b = (int)(rest / nzc);
    const size_t N = (size_t)n * n * n, nn = (size_t)n * n;
    const int m = lane & 15, g = lane >> 4, h = g >> 1;
    v8s B[2][kSlots][3];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int s = 0; s < kSlots; ++s)
#pragma unroll
            for (int dz = 0; dz < 3; ++dz) B[c][s][dz] = wpp[((c * kSlots + s) * 3 + dz) * 64 + lane];
    // this lane's element offset of each pair item within a plane
    int off[kPairs];
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        const int r = 2 * p + h, iy = r / 3, q = r % 3;
        off[p] = (n * wrapn(j0 - 1 + iy, n) + wrapn(iseg * 16 + m + q - 1, n)) * 16 + 8 * (g & 1);
    }
    const uint16_t* inb = in + (size_t)b * N * 16;
    uint16_t* outb = out + (size_t)b * N * 16;
    auto plane_ptr = [&](int t) { return inb + nn * 16 * (size_t)wrapn(k0 - 1 + t, n); };
    v8s a[kPairs];
    {
        const uint16_t* pb = plane_ptr(0);
#pragma unroll
        for (int p = 0; p < kPairs; ++p) a[p] = *reinterpret_cast<const v8s*>(pb + off[p]);
    }
    v4f acc[3][kRY];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int oy = 0; oy < kRY; ++oy) acc[r][oy] = v4f{0.f, 0.f, 0.f, 0.f};
    // fully unrolled: every plane's output rows and ring slots are constants
#pragma unroll
    for (int t = 0; t < ZC + 2; ++t) {
        const bool more = t + 1 < ZC + 2;
        const uint16_t* pn = plane_ptr(more ? t + 1 : t);
#pragma unroll
        for (int p = 0; p < kPairs; ++p) {
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
                const int oz = t - 1 - dz;   // output plane, ring slot oz mod 3
                if (oz < 0 || oz >= ZC) continue;
#pragma unroll
                for (int oy = 0; oy < kRY; ++oy) {
                    const int s = p - (3 * oy) / 2;
                    if (s < 0 || s >= kSlots) continue;
                    acc[oz % 3][oy] = mfma_k32(B[oy & 1][s][dz + 1], a[p], acc[oz % 3][oy]);
                }
            }
            if (more) a[p] = *reinterpret_cast<const v8s*>(pn + off[p]);
        }
        // output plane t - 2 has had its last input plane (dz = +1)
        if (t >= 2) {
            store_plane_rows(acc[(t - 2) % 3], outb, n, iseg * 16 + m, j0, k0 + t - 2, g, relu);
#pragma unroll
            for (int oy = 0; oy < kRY; ++oy) acc[(t - 2) % 3][oy] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    }
}

// The last layer's weights sit in LDS on a zero-padded (dz, dy) grid of [-4, 4]^2.
constexpr int kPadW = 9;   // dy, dz in [-4, 4]

// The last layer as a z-march: a wavefront owns 16 cells along x times kRY
// rows along y and walks ZC output planes.  The matrix columns (output rows of
// the product, weights as the A operand) are the kRY rows of the three output
// planes an input plane reaches, held in a ring: column 4 s + oy is row oy of
// the output plane in slot s (s = plane mod 3; columns 12-15 idle).  Input
// plane by input plane, each of its (kRY + 2) rows and 3 x shifts is one
// product whose weight operand the lane takes from the padded (dz, dy) grid at
// the offsets of its column; a column whose plane lies outside the chunk reads
// the grid's zeros.  After an input plane the output plane of its dz = +1 taps
// is complete: the lanes of its slot store it and clear their accumulators.
// Each input row is loaded once per plane, into its register right after its
// product (a plane of products covers the load).  y = yscale * output, FP32.
template <int ZC>
__global__ void __launch_bounds__(256) k_conv16_final_zm(int n, int batch,
                                                         const uint16_t* __restrict__ in,
                                                         const v4s* __restrict__ wfin,
                                                         float* __restrict__ yout, float yscale) {
    static_assert(kRY == 4, "three planes of kRY rows fit the 16 matrix columns");
    // wl[((dz + 4) kPadW + dy + 4) 3 + q][g]: channels 4g..4g+3 of tap (q - 1, dy, dz)
    __shared__ v4s wl[kPadW * kPadW * 3 * 4];
    for (int i = threadIdx.x; i < kPadW * kPadW * 3 * 4; i += blockDim.x) {
        const int g = i % 4, e = i / 4, q = e % 3, dy = (e / 3) % kPadW - 4, dz = e / (3 * kPadW) - 4;
        const bool reach = dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
        wl[i] = reach ? wfin[((dz + 1) * 9 + (dy + 1) * 3 + q) * 4 + g] : v4s{0, 0, 0, 0};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int segs = n / 16, nyb = n / kRY, nzc = n / ZC;
    const long nwaves = (long)batch * nzc * nyb * segs;
    if (wave >= nwaves) return;  // whole wavefront; no block barrier below
    const int iseg = (int)(wave % segs);
    long rest = wave / segs;
    const int j0 = (int)(rest % nyb) * kRY;
    rest /= nyb;
    const int k0 = (int)(rest % nzc) * ZC;
    const int b = (int)(rest / nzc);
    const size_t N = (size_t)n * n * n, nn = (size_t)n * n;
    const int m = lane & 15, g = lane >> 4;
    const int col = lane & 15, oy = col % kRY, slot = col / kRY;   // this lane's A row (output column)
    const uint16_t* inb = in + (size_t)b * N * 16 + 4 * g;
    // this lane's element offset of input row iy, shift q within a plane
    constexpr int kItemsF = (kRY + 2) * 3;
    int off[kItemsF];
#pragma unroll
    for (int it = 0; it < kItemsF; ++it) {
        const int iy = it / 3, q = it % 3;
        off[it] = (n * wrapn(j0 - 1 + iy, n) + wrapn(iseg * 16 + m + q - 1, n)) * 16;
    }
    auto plane_ptr = [&](int t) { return inb + nn * 16 * (size_t)wrapn(k0 - 1 + t, n); };
    v4s a[kItemsF];
    {
        const uint16_t* pb = plane_ptr(0);
#pragma unroll
        for (int it = 0; it < kItemsF; ++it) a[it] = *reinterpret_cast<const v4s*>(pb + off[it]);
    }
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < ZC + 2; ++t) {
        const bool more = t + 1 < ZC + 2;
        const uint16_t* pn = plane_ptr(more ? t + 1 : t);
        // the output plane of this lane's slot at input plane t: the one of
        // t - 2, t - 1, t congruent to the slot mod 3; its dz = t - 1 - oz, or
        // the grid's zeros (dz = 4) when it is outside the chunk or the slot idle
        const int oz = t - 2 + ((slot - (t - 2) % 3 + 3) % 3);
        const int dz = slot < 3 && oz >= 0 && oz < ZC ? t - 1 - oz : 4;
        const v4s* wb = wl + (((dz + 4) * kPadW + (3 - oy)) * 3) * 4 + g;
#pragma unroll
        for (int it = 0; it < kItemsF; ++it) {
            const int iy = it / 3, q = it % 3;
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wb[(iy * 3 + q) * 4], a[it], acc, 0, 0, 0);
            if (more) a[it] = *reinterpret_cast<const v4s*>(pn + off[it]);
        }
        // output plane t - 2 is complete: lane (g, m) holds rows 4 g + e of
        // cell m, so the lanes of its slot store rows 0..3 and clear them
        if (t >= 2) {
            const int sd = (t - 2) % 3;
            if (g == sd) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const size_t cell = (size_t)(iseg * 16 + m) +
                                        (size_t)n * ((size_t)(j0 + e) + (size_t)n * (k0 + t - 2));
                    yout[(size_t)b * N + cell] = acc[e] * yscale;
                    acc[e] = 0.f;
                }
            }
        }
    }
}

// The first layer (2 input channels, channel-last BF16 [cell][4] input) as a
// z-march like the 16 -> 16 layers.  One K = 16 block per input-row offset
// (dy, dz): lane group g holds the 4 channels of the cell shifted by
// dx = g - 1 (group 3 meets zero weights), so an input row is one 8-byte load
// per lane and the 9 weight operands stay in registers.  A wavefront owns 16
// cells along x times kRY rows along y and walks ZC output planes; each input
// plane's kRY + 2 rows, loaded into their registers right after their last
// product, feed the output rows of the three output planes in reach, held in
// a ring of accumulators.  ReLU, BF16 out.  Against one wavefront per
// 16 x 4 x 4 tile of output rows (36 input rows per 16 output rows) the
// network takes 1.04 instead of 1.07 ms at 256^3.
template <int ZC>
__global__ void __launch_bounds__(256) k_conv4_zm(int n, int batch, const uint16_t* __restrict__ in,
                                                  const v4s* __restrict__ wpk,
                                                  uint16_t* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int segs = n / 16, nyb = n / kRY, nzc = n / ZC;
    const long nwaves = (long)batch * nzc * nyb * segs;
    if (wave >= nwaves) return;  // whole wavefront; no block barrier below
    const int iseg = (int)(wave % segs);
    long rest = wave / segs;
    const int j0 = (int)(rest % nyb) * kRY;
    rest /= nyb;
    const int k0 = (int)(rest % nzc) * ZC;
    const int b = (int)(rest / nzc);
    const size_t N = (size_t)n * n * n, nn = (size_t)n * n;
    const int m = lane & 15, g = lane >> 4;
    v4s B[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) B[t] = wpk[t * 64 + lane];
    constexpr int kRW = kRY + 2;
    const uint16_t* inb = in + (size_t)b * N * 4;
    const int xo = wrapn(iseg * 16 + m + (g < 3 ? g - 1 : 0), n);   // group 3: weights are zero
    int off[kRW];
#pragma unroll
    for (int iy = 0; iy < kRW; ++iy) off[iy] = (n * wrapn(j0 - 1 + iy, n) + xo) * 4;
    auto plane_ptr = [&](int t) { return inb + nn * 4 * (size_t)wrapn(k0 - 1 + t, n); };
    v4s a[kRW];
    {
        const uint16_t* pb = plane_ptr(0);
#pragma unroll
        for (int iy = 0; iy < kRW; ++iy) a[iy] = *reinterpret_cast<const v4s*>(pb + off[iy]);
    }
    v4f acc[3][kRY];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int oy = 0; oy < kRY; ++oy) acc[r][oy] = v4f{0.f, 0.f, 0.f, 0.f};
    uint16_t* outb = out + (size_t)b * N * 16;
#pragma unroll
    for (int t = 0; t < ZC + 2; ++t) {
        const bool more = t + 1 < ZC + 2;
        const uint16_t* pn = plane_ptr(more ? t + 1 : t);
#pragma unroll
        for (int iy = 0; iy < kRW; ++iy) {
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
                const int oz = t - 1 - dz;   // ring slot oz mod 3
                if (oz < 0 || oz >= ZC) continue;
#pragma unroll
                for (int oy = 0; oy < kRY; ++oy) {
                    const int dy = iy - 1 - oy;
                    if (dy < -1 || dy > 1) continue;
                    acc[oz % 3][oy] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                        B[(dz + 1) * 3 + dy + 1], a[iy], acc[oz % 3][oy], 0, 0, 0);
                }
            }
            if (more) a[iy] = *reinterpret_cast<const v4s*>(pn + off[iy]);
        }
        if (t >= 2) {   // output plane t - 2 has had its last input plane
            store_plane_rows(acc[(t - 2) % 3], outb, n, iseg * 16 + m, j0, k0 + t - 2, g, 1);
#pragma unroll
            for (int oy = 0; oy < kRY; ++oy) acc[(t - 2) % 3][oy] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    }
}

// Weight gradient of one layer: partial sums over this wavefront's cells of
// D[co][(tap, ci)] = sum_cells g[cell][co] in[cell + d(tap)][ci], one 16x16 tile
// per K-block, written to part[wave][kb][co][n].
template <int CINP>
__global__ void __launch_bounds__(256) k_conv_wgrad(int n, int batch,
                                                    const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ gr, int gp,
                                                    int cout, float* __restrict__ part, int spw,
                                                    int nwaves) {
    constexpr int NKB = nkb<CINP>();
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int segs = n / 16;
    const long nseg = (long)batch * n * n * segs;
    const size_t N = (size_t)n * n * n;
    const int m = lane & 15, g = lane >> 4, nn = lane & 15;
    v4f acc[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) acc[kb] = v4f{0.f, 0.f, 0.f, 0.f};
    for (long s = (long)wave * spw; s < (long)(wave + 1) * spw && s < nseg; ++s) {
        const int iseg = (int)(s % segs);
        long rest = s / segs;
        const int j = (int)(rest % n);
        rest /= n;
        const int k = (int)(rest % n);
        const int b = (int)(rest / n);
        v4s a;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const size_t P = (size_t)b * N + (size_t)(iseg * 16 + 4 * g + e) +
                             (size_t)n * ((size_t)j + (size_t)n * k);
            a[e] = m < cout ? (short)gr[P * gp + m] : (short)0;
        }
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            int tap, ci;
            kdecode<CINP>(kb, nn, tap, ci);
            v4s bb = {0, 0, 0, 0};
            if (tap < 27) {
                const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
                const size_t yz = (size_t)n * ((size_t)wrapn(j + dy, n) + (size_t)n * wrapn(k + dz, n));
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const size_t cell = (size_t)wrapn(iseg * 16 + 4 * g + e + dx, n) + yz;
                    bb[e] = (short)in[((size_t)b * N + cell) * CINP + ci];
                }
            }
            acc[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[kb], 0, 0, 0);
        }
    }
    float* dst = part + (size_t)wave * NKB * 256;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[kb * 256 + (4 * g + e) * 16 + nn] = acc[kb][e];
}

// Sum the per-wavefront partials in wavefront order and scatter them into the
// FP32 gradient layout [co][ci][27] of one layer (deterministic).
template <int CINP>
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nwaves, int cin, int cout,
                               float* __restrict__ grad) {
    constexpr int NKB = nkb<CINP>();
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= NKB * 256) return;
    const int kb = idx / 256, co = (idx % 256) / 16, nn = idx % 16;
    int tap, ci;
    kdecode<CINP>(kb, nn, tap, ci);
    if (tap >= 27 || ci >= cin || co >= cout) return;
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += (double)part[(size_t)w * NKB * 256 + idx];
    grad[((size_t)co * cin + ci) * 27 + tap] = (float)s;
}

// Pack the first layer (cin input channels, cout <= 16 outputs) for
// k_conv4_zm: one K-block per input-row offset (dy, dz), t9 = (dz+1) 3 + (dy+1);
// its K entry 4 g + c holds channel c of the cell dx = g - 1 along x (g < 3;
// g = 3 and c >= cin are zero).
__global__ void k_pack_rows4(const float* __restrict__ w, int cin, int cout, v4s* __restrict__ wpk) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 9 * 64) return;
    const int kb = t / 64, lane = t % 64;
    const int nn = lane & 15, g = lane >> 4;
    const int tap = (kb / 3) * 9 + (kb % 3) * 3 + g;
    v4s v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float x = 0.f;
        if (g < 3 && e < cin && nn < cout) x = w[((size_t)nn * cin + e) * 27 + tap];
        v[e] = (short)f2bf(x);
    }
    wpk[t] = v;
}

// Pack the last layer (16 inputs, 1 output) for k_conv16_final_zm:
// wfin[tap * 4 + g] = BF16 W[0][4g + e][tap], e = 0..3.
__global__ void k_pack_final(const float* __restrict__ w, v4s* __restrict__ wfin) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 27 * 4) return;
    const int tap = t / 4, g = t % 4;
    v4s v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (short)f2bf(w[(size_t)(4 * g + e) * 27 + tap]);
    wfin[t] = v;
}

// Pack a 16 -> 16 layer for k_conv16_zm: operand (c, s, dz) at lane
// (n = co, g) holds in entry j the weight of channel 8 (g & 1) + j for item
// rr = 2 s + (g >> 1) - c of the output row's run, rr = 3 (dy + 1) + dx + 1,
// zero outside 0..8.
__global__ void k_pack_pairs(const float* __restrict__ w, v8s* __restrict__ wpp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * kSlots * 3 * 64) return;
    const int op = t / 64, lane = t % 64;
    const int dz = op % 3, s = (op / 3) % kSlots, c = op / (3 * kSlots);
    const int co = lane & 15, g = lane >> 4, rr = 2 * s + (g >> 1) - c;
    v8s v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float x = 0.f;
        if (rr >= 0 && rr < 9) x = w[((size_t)co * 16 + 8 * (g & 1) + j) * 27 + dz * 9 + rr];
        v[j] = (short)f2bf(x);
    }
    wpp[t] = v;
}

// Pack one layer's FP32 weights [co][ci][27] into per-lane BF16 B operands.
// Forward: out channel n = co, K entry (tap, ci).  Data gradient (tflip): out
// channel n = ci, K entry (tap', co) with weight W[co][ci][26 - tap'].
template <int CINP>
__global__ void k_pack(const float* __restrict__ w, int cin, int cout, int tflip,
                       v4s* __restrict__ wpk) {
    constexpr int NKB = nkb<CINP>();
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NKB * 64) return;
    const int kb = t / 64, lane = t % 64;
    const int nn = lane & 15, g = lane >> 4;
    v4s v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        int tap, cc;
        kdecode<CINP>(kb, 4 * g + e, tap, cc);
        float x = 0.f;
        if (tap < 27) {
            if (!tflip) {
                if (nn < cout && cc < cin) x = w[((size_t)nn * cin + cc) * 27 + tap];
            } else {
                if (nn < cin && cc < cout) x = w[((size_t)cc * cin + nn) * 27 + (26 - tap)];
            }
        }
        v[e] = (short)f2bf(x);
    }
    wpk[t] = v;
}

// Network input: channel-last BF16 [cell][4] = (x0, x1, 0, 0) from FP32 [cell][2].
__global__ void k_input_bf16(const float* __restrict__ x, uint16_t* __restrict__ xb, size_t cells) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < cells; i += stride) {
        xb[4 * i + 0] = f2bf(x[2 * i + 0]);
        xb[4 * i + 1] = f2bf(x[2 * i + 1]);
        xb[4 * i + 2] = 0;
        xb[4 * i + 3] = 0;
    }
}

// MSE loss partials and the output gradient dy = 2 (y - t) / count as BF16 [cell][4].
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             size_t count, float scale, uint16_t* __restrict__ dy,
                                             double* part) {
    double v[1] = {0.0};
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) {
        const float d = y[i] - t[i];
        v[0] += (double)d * (double)d;
        dy[4 * i + 0] = f2bf(scale * d);
        dy[4 * i + 1] = 0;
        dy[4 * i + 2] = 0;
        dy[4 * i + 3] = 0;
    }
    block_partials<1, 0u>(v, part);
}

// ---- training on the solve's own measure ----
// For one sample with the captured system (b, diag, w) of M x = b and the
// network output g: u = M g, alpha = g.b / g.u (the start rescale of the
// solve), r = b - alpha u and the loss L = |r|^2 / |b|^2, the relative
// residual the solve starts from (invariant to the scale of g and b).  With
// c = g.u:  dL/dg = -(2 / |b|^2) [ (u.r / c) (b - 2 alpha u) + alpha M r ].
// M v = diag v - (1/h^2) sum_f K_f v_nb(f), K_f = I4(w) on face f: the
// pressure operator written with its diagonal.  FP64 arithmetic on the FP32
// network output.
constexpr int kResBlocks = 64;   // blocks per sample (grid kResBlocks x batch)

template <typename V>
__device__ inline double m_offdiag(const double* __restrict__ w, const CellIdx& c, V&& v) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) s += i4(w, c, d, 0) * v(c.sh(d, 1)) + i4(w, c, d, -1) * v(c.sh(d, -1));
    return s;
}

__global__ void __launch_bounds__(256) k_res_u(int n, double inv_h2, const double* __restrict__ b,
                                               const double* __restrict__ diag,
                                               const double* __restrict__ w, const float* __restrict__ y,
                                               double* __restrict__ u, double* part) {
    const BlockXYZ bx = block_xyz();
    const size_t N = (size_t)n * n * n, base = (size_t)bx.y * N;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // g.b, g.u, u.b, u.u, b.b
    for (size_t i = (size_t)bx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const CellIdx c(n, (int)(i % n), (int)((i / n) % n), (int)(i / ((size_t)n * n)), base);
        const size_t P = c.self();
        const double gP = y[P], bP = b[P];
        const double uP = diag[P] * gP - inv_h2 * m_offdiag(w, c, [&](size_t Q) { return (double)y[Q]; });
        u[P] = uP;
        v[0] += gP * bP;
        v[1] += gP * uP;
        v[2] += uP * bP;
        v[3] += uP * uP;
        v[4] += bP * bP;
    }
    block_partials<5, 0u>(v, part);
}

// Per sample: coef = (alpha, u.r / c, -2 / (|b|^2 batch)) and its loss; one
// block walks the samples in order and writes the batch mean to loss.
__global__ void __launch_bounds__(256) k_res_coef(int batch, const double* __restrict__ part,
                                                  double* __restrict__ coef, double* loss) {
    double total = 0.0;
    for (int sm = 0; sm < batch; ++sm) {
        double t[5];
        reduce_partials_strided<5, 0u>(part, (size_t)kResBlocks * batch, (size_t)sm * kResBlocks,
                                       kResBlocks, t);
        if (threadIdx.x == 0) {
            const double gb = t[0], gu = t[1], ub = t[2], uu = t[3], bb = t[4];
            const bool ok = gu > 0.0 && bb > 0.0;
            const double alpha = ok ? gb / gu : 0.0;
            const double ur = ub - alpha * uu;
            coef[3 * sm + 0] = alpha;
            coef[3 * sm + 1] = ok ? ur / gu : 0.0;
            coef[3 * sm + 2] = ok ? -2.0 / (bb * batch) : 0.0;
            total += ok ? (bb - 2.0 * alpha * ub + alpha * alpha * uu) / bb : 1.0;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = total / batch;
}

// Output gradient dL/dg as BF16 [cell][4] (channel 0), for the backward pass.
__global__ void __launch_bounds__(256) k_res_dy(int n, double inv_h2, const double* __restrict__ b,
                                                const double* __restrict__ diag,
                                                const double* __restrict__ w,
                                                const double* __restrict__ u,
                                                const double* __restrict__ coef,
                                                uint16_t* __restrict__ dy) {
    const BlockXYZ bx = block_xyz();
    const size_t N = (size_t)n * n * n, base = (size_t)bx.y * N;
    const double alpha = coef[3 * bx.y], beta = coef[3 * bx.y + 1], sc = coef[3 * bx.y + 2];
    for (size_t i = (size_t)bx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const CellIdx c(n, (int)(i % n), (int)((i / n) % n), (int)(i / ((size_t)n * n)), base);
        const size_t P = c.self();
        auto r = [&](size_t Q) { return b[Q] - alpha * u[Q]; };
        const double Mr = diag[P] * r(P) - inv_h2 * m_offdiag(w, c, r);
        const double g = sc * (beta * (b[P] - 2.0 * alpha * u[P]) + alpha * Mr);
        dy[4 * P + 0] = f2bf((float)g);
        dy[4 * P + 1] = 0;
        dy[4 * P + 2] = 0;
        dy[4 * P + 3] = 0;
    }
}

__global__ void k_adam(int nw, float* __restrict__ w, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------
static const int kCh[5] = {2, 16, 16, 16, 1};

size_t net_weight_offset(int layer) {
    size_t s = 0;
    for (int l = 0; l < layer; ++l) s += (size_t)kCh[l] * kCh[l + 1] * 27;
    return s;
}

// Forward operands: layer 1 for k_conv (7 K-blocks), layers 2-4 (27 each),
// layer 1 again for k_conv4_zm (9 K-blocks), layer 4 for
// k_conv16_final_zm (27 taps x 4 channel groups), then layers 2 and 3 for
// k_conv16_zm (30 K = 32 operands each).
constexpr size_t kPackV4 = (size_t)(7 + 27 + 27 + 27 + 9) * 64 + 27 * 4;
constexpr int kPairOps = 2 * kSlots * 3 * 64;
static_assert(kPackV4 * sizeof(v4s) % sizeof(v8s) == 0, "pair operands stay 16-byte aligned");
size_t net_packed_bytes() { return kPackV4 * sizeof(v4s) + (size_t)2 * kPairOps * sizeof(v8s); }
static const v8s* pair_ops(const void* wpk, int layer) {
    return reinterpret_cast<const v8s*>(reinterpret_cast<const v4s*>(wpk) + kPackV4) +
           (size_t)(layer - 1) * kPairOps;
}

void net_pack_forward(hipStream_t s, const float* w32, void* wpk) {
    v4s* p = reinterpret_cast<v4s*>(wpk);
    hipLaunchKernelGGL(k_pack<4>, dim3((7 * 64 + 255) / 256), dim3(256), 0, s,
                       w32 + net_weight_offset(0), 2, 16, 0, p);
    p += 7 * 64;
    for (int l = 1; l < 4; ++l) {
        hipLaunchKernelGGL(k_pack<16>, dim3((27 * 64 + 255) / 256), dim3(256), 0, s,
                           w32 + net_weight_offset(l), 16, kCh[l + 1], 0, p);
        p += 27 * 64;
    }
    hipLaunchKernelGGL(k_pack_rows4, dim3((9 * 64 + 255) / 256), dim3(256), 0, s,
                       w32 + net_weight_offset(0), 2, 16, p);
    p += 9 * 64;
    hipLaunchKernelGGL(k_pack_final, dim3(1), dim3(128), 0, s, w32 + net_weight_offset(3), p);
    for (int l = 1; l < 3; ++l)
        hipLaunchKernelGGL(k_pack_pairs, dim3((kPairOps + 255) / 256), dim3(256), 0, s,
                           w32 + net_weight_offset(l), const_cast<v8s*>(pair_ops(wpk, l)));
}

static dim3 conv_grid(int n, int batch) {
    const long waves = (long)batch * n * n * (n / 16);
    return dim3((unsigned)((waves + 3) / 4));
}

// Output planes per wavefront of k_conv16_zm: the longest chunk (16, 8 or 4
// planes, dividing n) that still gives at least 4096 wavefronts (32 planes
// would spill registers).
static int zm_chunk(int n, int batch) {
    const long per_plane = (long)batch * (n / kRY) * (n / 16);
    for (int zc = 16; zc > 4; zc /= 2)
        if (n % zc == 0 && per_plane * (n / zc) >= 4096) return zc;
    return 4;
}
static unsigned zm_blocks(int n, int batch, int zc) {
    const long waves = (long)batch * (n / zc) * (n / kRY) * (n / 16);
    return (unsigned)((waves + 3) / 4);
}

void net_forward(hipStream_t s, int n, int batch, const void* wpk, const uint16_t* x4,
                 uint16_t* a, uint16_t* b, float* y, float yscale) {
    const v4s* p = reinterpret_cast<const v4s*>(wpk);
    const dim3 B(256);
    const int zc = zm_chunk(n, batch);
    const dim3 GZ(zm_blocks(n, batch, zc));
    const v4s* w1 = p + (7 + 27 + 27 + 27) * 64;
    switch (zc) {
    case 16: hipLaunchKernelGGL(k_conv4_zm<16>, GZ, B, 0, s, n, batch, x4, w1, a); break;
    case 8: hipLaunchKernelGGL(k_conv4_zm<8>, GZ, B, 0, s, n, batch, x4, w1, a); break;
    default: hipLaunchKernelGGL(k_conv4_zm<4>, GZ, B, 0, s, n, batch, x4, w1, a); break;
    }
    auto layer = [&](const uint16_t* src, const v8s* w, uint16_t* dst) {
        switch (zc) {
        case 16: hipLaunchKernelGGL(k_conv16_zm<16>, GZ, B, 0, s, n, batch, src, w, 1, dst); break;
        case 8: hipLaunchKernelGGL(k_conv16_zm<8>, GZ, B, 0, s, n, batch, src, w, 1, dst); break;
        default: hipLaunchKernelGGL(k_conv16_zm<4>, GZ, B, 0, s, n, batch, src, w, 1, dst); break;
        }
    };
    layer(a, pair_ops(wpk, 1), b);
    layer(b, pair_ops(wpk, 2), a);
    const v4s* wfin = reinterpret_cast<const v4s*>(wpk) + (7 + 27 + 27 + 27 + 9) * 64;
    switch (zc) {
    case 16: hipLaunchKernelGGL(k_conv16_final_zm<16>, GZ, B, 0, s, n, batch, a, wfin, y, yscale); break;
    case 8: hipLaunchKernelGGL(k_conv16_final_zm<8>, GZ, B, 0, s, n, batch, a, wfin, y, yscale); break;
    default: hipLaunchKernelGGL(k_conv16_final_zm<4>, GZ, B, 0, s, n, batch, a, wfin, y, yscale); break;
    }
}

// ---- training workspace ----
struct NetWs {
    size_t x4, a1, a2, a3, y, g1, g2, dy, wf, wb, part, lpart, ru, rpart, rcoef, total;
    int nwaves, spw;
    unsigned lblocks;
};

static NetWs net_layout(int n, int batch) {
    NetWs L{};
    const size_t cells = (size_t)batch * n * n * n;
    const long nseg = (long)batch * n * n * (n / 16);
    L.nwaves = (int)(nseg < 1024 ? nseg : 1024);
    L.spw = (int)((nseg + L.nwaves - 1) / L.nwaves);
    L.lblocks = 1024;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + 255) / 256 * 256;
        return o;
    };
    L.x4 = take(cells * 4 * 2);
    L.a1 = take(cells * 16 * 2);
    L.a2 = take(cells * 16 * 2);
    L.a3 = take(cells * 16 * 2);
    L.y = take(cells * 4);
    L.g1 = take(cells * 16 * 2);
    L.g2 = take(cells * 16 * 2);
    L.dy = take(cells * 4 * 2);
    L.wf = take(net_packed_bytes());
    L.wb = take((size_t)3 * 27 * 64 * sizeof(v4s));
    L.part = take((size_t)L.nwaves * 27 * 256 * sizeof(float));
    L.lpart = take((size_t)L.lblocks * sizeof(double) + sizeof(double));
    L.ru = take(cells * sizeof(double));
    L.rpart = take((size_t)5 * kResBlocks * batch * sizeof(double));
    L.rcoef = take((size_t)3 * batch * sizeof(double));
    L.total = off;
    return L;
}

}  // namespace pisoc

using namespace pisoc;

static bool net_shape_ok(int32_t n, int32_t batch) {
    return n >= 16 && n <= PISOC_MAX_N && n % 16 == 0 && batch >= 1;
}

extern "C" {

size_t pisoc_net_workspace_bytes(int32_t n, int32_t batch) {
    if (!net_shape_ok(n, batch)) return 0;
    return net_layout(n, batch).total;
}

pisoc_status pisoc_net_forward(int32_t n, int32_t batch, const float* d_w, const float* d_x,
                               float* d_y, void* d_ws, size_t ws_bytes, void* stream) {
    if (!net_shape_ok(n, batch) || !d_w || !d_x || !d_y) return PISOC_ERR_INVALID;
    NetWs L = net_layout(n, batch);
    if (!d_ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) % 256) != 0)
        return PISOC_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(d_ws);
    const size_t cells = (size_t)batch * n * n * n;
    uint16_t* x4 = reinterpret_cast<uint16_t*>(ws + L.x4);
    hipLaunchKernelGGL(k_input_bf16, dim3((unsigned)std::min<size_t>((cells + 255) / 256, 65536)),
                       dim3(256), 0, s, d_x, x4, cells);
    net_pack_forward(s, d_w, ws + L.wf);
    net_forward(s, n, batch, ws + L.wf, x4, reinterpret_cast<uint16_t*>(ws + L.a1),
                reinterpret_cast<uint16_t*>(ws + L.a2), d_y, 1.f);
    return hipGetLastError() == hipSuccess ? PISOC_OK : PISOC_ERR_HIP;
}

// Forward pass of a training step keeping every activation in the
// workspace (y at L.y), after packing the forward and data-gradient weights.
static void grad_forward(hipStream_t s, const NetWs& L, char* ws, int n, int batch, const float* d_w,
                         const float* d_x) {
    auto U = [&](size_t off) { return reinterpret_cast<uint16_t*>(ws + off); };
    const size_t cells = (size_t)batch * n * n * n;
    const dim3 G = conv_grid(n, batch), B(256);
    const unsigned lin = (unsigned)std::min<size_t>((cells + 255) / 256, 65536);
    hipLaunchKernelGGL(k_input_bf16, dim3(lin), B, 0, s, d_x, U(L.x4), cells);
    net_pack_forward(s, d_w, ws + L.wf);
    // data-gradient weights of layers 2..4 (transposed, flipped)
    v4s* wb = reinterpret_cast<v4s*>(ws + L.wb);
    for (int l = 1; l < 4; ++l) {
        if (l == 3)
            hipLaunchKernelGGL(k_pack<4>, dim3((7 * 64 + 255) / 256), B, 0, s,
                               d_w + net_weight_offset(l), 16, 1, 1, wb + (l - 1) * 27 * 64);
        else
            hipLaunchKernelGGL(k_pack<16>, dim3((27 * 64 + 255) / 256), B, 0, s,
                               d_w + net_weight_offset(l), 16, 16, 1, wb + (l - 1) * 27 * 64);
    }
    const v4s* wf = reinterpret_cast<const v4s*>(ws + L.wf);
    float* y = reinterpret_cast<float*>(ws + L.y);
    hipLaunchKernelGGL((k_conv<4, false>), G, B, 0, s, n, batch, U(L.x4), wf, (const uint16_t*)nullptr,
                       1, U(L.a1), (float*)nullptr, 1.f);
    hipLaunchKernelGGL((k_conv<16, false>), G, B, 0, s, n, batch, U(L.a1), wf + 7 * 64,
                       (const uint16_t*)nullptr, 1, U(L.a2), (float*)nullptr, 1.f);
    hipLaunchKernelGGL((k_conv<16, false>), G, B, 0, s, n, batch, U(L.a2), wf + 34 * 64,
                       (const uint16_t*)nullptr, 1, U(L.a3), (float*)nullptr, 1.f);
    hipLaunchKernelGGL((k_conv<16, true>), G, B, 0, s, n, batch, U(L.a3), wf + 61 * 64,
                       (const uint16_t*)nullptr, 0, (uint16_t*)nullptr, y, 1.f);
}

// Weight gradient from the output gradient dy (BF16 [cell][4] at L.dy) and
// the activations grad_forward kept.
static void grad_backward(hipStream_t s, const NetWs& L, char* ws, int n, int batch, float* d_grad) {
    auto U = [&](size_t off) { return reinterpret_cast<uint16_t*>(ws + off); };
    const dim3 G = conv_grid(n, batch), B(256);
    const v4s* wb = reinterpret_cast<const v4s*>(ws + L.wb);
    float* part = reinterpret_cast<float*>(ws + L.part);
    const dim3 GW((L.nwaves + 3) / 4);
    auto wgrad16 = [&](const uint16_t* in, const uint16_t* gr, int gp, int cout, int layer) {
        hipLaunchKernelGGL(k_conv_wgrad<16>, GW, B, 0, s, n, batch, in, gr, gp, cout, part, L.spw,
                           L.nwaves);
        hipLaunchKernelGGL(k_wgrad_reduce<16>, dim3((27 * 256 + 255) / 256), B, 0, s, part, L.nwaves,
                           16, cout, d_grad + net_weight_offset(layer));
    };
    // layer 4 (linear), 3, 2, 1
    wgrad16(U(L.a3), U(L.dy), 4, 1, 3);
    hipLaunchKernelGGL((k_conv<4, false>), G, B, 0, s, n, batch, U(L.dy), wb + 2 * 27 * 64, U(L.a3),
                       0, U(L.g1), (float*)nullptr, 1.f);
    wgrad16(U(L.a2), U(L.g1), 16, 16, 2);
    hipLaunchKernelGGL((k_conv<16, false>), G, B, 0, s, n, batch, U(L.g1), wb + 27 * 64, U(L.a2), 0,
                       U(L.g2), (float*)nullptr, 1.f);
    wgrad16(U(L.a1), U(L.g2), 16, 16, 1);
    hipLaunchKernelGGL((k_conv<16, false>), G, B, 0, s, n, batch, U(L.g2), wb, U(L.a1), 0, U(L.g1),
                       (float*)nullptr, 1.f);
    hipLaunchKernelGGL(k_conv_wgrad<4>, GW, B, 0, s, n, batch, U(L.x4), U(L.g1), 16, 16, part, L.spw,
                       L.nwaves);
    hipLaunchKernelGGL(k_wgrad_reduce<4>, dim3((7 * 256 + 255) / 256), B, 0, s, part, L.nwaves, 2, 16,
                       d_grad + net_weight_offset(0));
}

static pisoc_status read_loss(hipStream_t s, const double* loss_dev, double scale, double* h_loss) {
    if (hipGetLastError() != hipSuccess) return PISOC_ERR_HIP;
    if (h_loss) {
        double l = 0.0;
        if (hipMemcpyAsync(&l, loss_dev, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PISOC_ERR_HIP;
        *h_loss = l * scale;
    }
    return PISOC_OK;
}

pisoc_status pisoc_net_grad(int32_t n, int32_t batch, const float* d_w, const float* d_x,
                            const float* d_t, float* d_grad, double* h_loss, void* d_ws,
                            size_t ws_bytes, void* stream) {
    if (!net_shape_ok(n, batch) || !d_w || !d_x || !d_t || !d_grad) return PISOC_ERR_INVALID;
    NetWs L = net_layout(n, batch);
    if (!d_ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) % 256) != 0)
        return PISOC_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(d_ws);
    const size_t cells = (size_t)batch * n * n * n;
    grad_forward(s, L, ws, n, batch, d_w, d_x);
    // loss and output gradient
    double* lpart = reinterpret_cast<double*>(ws + L.lpart);
    hipLaunchKernelGGL(k_mse, dim3(L.lblocks), dim3(256), 0, s, reinterpret_cast<const float*>(ws + L.y),
                       d_t, cells, (float)(2.0 / (double)cells),
                       reinterpret_cast<uint16_t*>(ws + L.dy), lpart);
    double* loss_dev = lpart + L.lblocks;
    sum_partials(s, lpart, L.lblocks, loss_dev);
    grad_backward(s, L, ws, n, batch, d_grad);
    return read_loss(s, loss_dev, 1.0 / (double)cells, h_loss);
}

pisoc_status pisoc_net_grad_residual(int32_t n, int32_t batch, const float* d_w, const float* d_x,
                                     const double* d_b, const double* d_diag, const double* d_wk,
                                     float* d_grad, double* h_loss, void* d_ws, size_t ws_bytes,
                                     void* stream) {
    if (!net_shape_ok(n, batch) || !d_w || !d_x || !d_b || !d_diag || !d_wk || !d_grad)
        return PISOC_ERR_INVALID;
    NetWs L = net_layout(n, batch);
    if (!d_ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) % 256) != 0)
        return PISOC_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(d_ws);
    grad_forward(s, L, ws, n, batch, d_w, d_x);
    const double h = 2.0 * M_PI / n, inv_h2 = 1.0 / (h * h);
    double* u = reinterpret_cast<double*>(ws + L.ru);
    double* rpart = reinterpret_cast<double*>(ws + L.rpart);
    double* coef = reinterpret_cast<double*>(ws + L.rcoef);
    double* loss_dev = reinterpret_cast<double*>(ws + L.lpart);
    const dim3 GR(kResBlocks, batch), B(256);
    hipLaunchKernelGGL(k_res_u, GR, B, 0, s, n, inv_h2, d_b, d_diag, d_wk,
                       reinterpret_cast<const float*>(ws + L.y), u, rpart);
    hipLaunchKernelGGL(k_res_coef, dim3(1), B, 0, s, batch, rpart, coef, loss_dev);
    hipLaunchKernelGGL(k_res_dy, GR, B, 0, s, n, inv_h2, d_b, d_diag, d_wk, u, coef,
                       reinterpret_cast<uint16_t*>(ws + L.dy));
    grad_backward(s, L, ws, n, batch, d_grad);
    return read_loss(s, loss_dev, 1.0, h_loss);
}

pisoc_status pisoc_net_adam(int32_t nw, float* d_w, const float* d_g, float* d_m, float* d_v,
                            int32_t step, float lr, float beta1, float beta2, float eps,
                            void* stream) {
    if (nw < 1 || !d_w || !d_g || !d_m || !d_v || step < 1) return PISOC_ERR_INVALID;
    const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((nw + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), nw, d_w, d_g, d_m, d_v, lr, beta1,
                       beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? PISOC_OK : PISOC_ERR_HIP;
}

}  // extern "C"
