// device.hpp -- device-side building blocks shared by the PISO kernels:
// grid geometry, periodic neighbour indexing, the fourth-order face
// interpolation, and deterministic grid-wide reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pisoc {

constexpr int kBlock = 256;       // threads per block of every field kernel
constexpr int kMaxRed = 8;        // values per grid reduction
constexpr int kMaxCorr = 4;
constexpr int kMaxClasses = 8;
constexpr int kIterInf = 0x7fffffff;

// Constants of one grid size and gas, passed by value to the kernels.  A
// launch covers `batch` members of the same size stacked along z (member m owns
// the blocks with blockIdx.z in [m nz, (m+1) nz) and the cells [m N, (m+1) N) of
// every field; vector components are NT = batch N apart).
struct Phys {
    int n;
    int cz;             // cells per thread along z
    int nz;             // blocks per member along z
    int batch;          // members in the launch
    size_t N, NT;       // cells per member, cells of all members
    double h, inv_h, inv_h2, V, inv_V, A;
    double gamma, C, mu;
    double g[3];        // gravity (settling drift; with two-way coupling also buoyancy)
    // Fourier closure (FP64 single grids): p = rho R T with the energy
    // equation; tn: T^n, ts: T* of the current step (set before each step)
    int fourier;
    double R, cv, kappa;
    const double* tn;
    const double* ts;
    // BDF2 (FP64 single grids, gathered kernels): the state at t^{n-1}
    // (density deviation, velocity, and one class's bulk density, set per
    // class); the coefficients are DevState::bdf
    int bdf2;
    const double* rm1;
    const double* um1;
    const double* rjm1;
};

// Variable-step BDF2 coefficients, d/dt y ~ (c0 y^{n+1} - c1 y^n + c2 y^{n-1}) / dt
// with w = dt / dt_prev (w = 0, backward Euler, when there is no previous step).
__host__ __device__ inline void bdf2_coef(double dt, double dt_prev, double (&c)[3]) {
    const double w = isfinite(dt_prev) ? dt / dt_prev : 0.0;
    c[0] = (1.0 + 2.0 * w) / (1.0 + w);
    c[1] = 1.0 + w;
    c[2] = w * w / (1.0 + w);
}

// The compressibility factor of the corrector: psi = rho / (gamma_psi p) with
// gamma_psi = gamma for the barotropic closure (d rho / d p of C rho^gamma)
// and 1 for the ideal gas at the predicted temperature (1 / (R T)).
__host__ __device__ inline double gamma_psi(const Phys& ph) { return ph.fourier ? 1.0 : ph.gamma; }

// State of one pressure solve, kept on the device so that CG never returns to
// the host between iterations.
struct PcgState {
    double bb;        // reference ||b||^2 of the current solve
    double rr;        // ||r||^2 of the last checked iterate
    double tol2;      // tol^2 of the current (inner) solve
    double tol_final; // p_tol^2: the requested relative residual, squared
    double alphah[2]; // alpha_{k-1}, written by CG iteration k in slot k & 1
    double cheb[2];   // c0, c1 of the Chebyshev polynomial preconditioner
    int32_t it_stop;  // iteration index at which the solve stopped (kIterInf: running)
    int32_t maxit;
    int32_t iters;
    int32_t converged;
    int32_t skip;     // 1: the refinement already meets the tolerance; later rounds do nothing
};

// State of the momentum predictor's BiCGStab (mom_tol > 0), on the device.
struct BicgState {
    double rho, rho_old, alpha, omega;  // (rh, r_k), (rh, r_{k-1}), alpha_k, omega_k
    double bb, rr;                      // ||b||^2 and ||r||^2 of the last checked iterate
    int32_t it_stop;                    // iteration count at the stop (kIterInf: running)
    int32_t iters, converged, pad;
};

// Per-member device state, read back by the host after a batch of work.
struct DevState {
    double dt, dt_prev, sigma, t;
    PcgState pcg;
    int32_t flags;
    int32_t pad0;
    double mass_gas;   // sum rho V of the last step
    double usq;        // sum |u|^2 of the last step
    double rho_min;
    double mass_p[kMaxClasses];
    double red[kMaxRed];
    // constants of the member: rho and p are stored as deviations from
    // (rho_ref, p_ref); particle response times
    double rho_ref, p_ref;
    double tau[kMaxClasses];
    double aff[2];     // per-member affine coefficients of a statistics pass
    // record of the current step, per corrector
    int32_t it_corr[kMaxCorr];     // CG iterations, all rounds
    int32_t rounds_corr[kMaxCorr]; // FP64 refinement rounds
    int32_t it_first[kMaxCorr];    // iterations of the first (fresh) solve
    int32_t it_later[kMaxCorr];    // most iterations of one later refinement round
    double rel_corr[kMaxCorr];     // final ||r|| / ||b||
    // accumulated over the steps since the host last cleared them
    int32_t flags_acc;
    int32_t steps_acc;
    int32_t it_first_max[kMaxCorr];
    int32_t it_later_max[kMaxCorr];
    // two-way coupling: mean mixture density <rho + sum_j rho_j> (a constant of
    // the run: gas and dust masses are conserved exactly)
    double rhom_mean;
    // the dust's Courant number of the step (max over the classes)
    double courant_dust;
    // BDF2 coefficients of the step (c0, c1, c2), written by the predictor
    double bdf[3];
    BicgState bicg;
};

// A cell and the periodic offsets to the cells up to two steps away along
// each axis (every stencil here reaches at most two cells): computed once per
// cell, so that each neighbour address is one add.
struct CellIdx {
    size_t p;               // this cell (member base included)
    int off[3][5];          // off[d][s + 2]: index offset of the cell s steps along d
    __device__ inline CellIdx(int n, int i, int j, int k, size_t base) {
        p = base + (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
        const int nn = n * n;
#pragma unroll
        for (int s = -2; s <= 2; ++s) {
            off[0][s + 2] = wrap_delta(i, s, n);
            off[1][s + 2] = wrap_delta(j, s, n) * n;
            off[2][s + 2] = wrap_delta(k, s, n) * nn;
        }
    }
    static __device__ inline int wrap_delta(int i, int s, int n) {
        int a = i + s;
        a = a < 0 ? a + n : (a >= n ? a - n : a);
        return a - i;
    }
    // cell reached by s steps along axis d (|s| <= 2)
    __device__ inline size_t sh(int d, int s) const {
        return p + (size_t)(ptrdiff_t)off[d][s + 2];
    }
    __device__ inline size_t self() const { return p; }
};

// Fourth-order central interpolation onto face P + (s + 1/2) e_d:
// weights (-1, 9, 9, -1)/16 on cells P+s-1 .. P+s+2 along d.
template <typename T>
__device__ inline T i4(const T* __restrict__ q, const CellIdx& c, int d, int s) {
    T a = q[c.sh(d, s - 1)], b = q[c.sh(d, s)], e = q[c.sh(d, s + 1)], f = q[c.sh(d, s + 2)];
    return (T(9) * (b + e) - (a + f)) * T(0.0625);
}

// I4 of T-stored values evaluated in the arithmetic of R (FP64 evaluation of
// FP32-stored fields).
template <typename R, typename T>
__device__ inline R i4r(const T* __restrict__ q, const CellIdx& c, int d, int s) {
    R a = (R)q[c.sh(d, s - 1)], b = (R)q[c.sh(d, s)], e = (R)q[c.sh(d, s + 1)],
      f = (R)q[c.sh(d, s + 2)];
    return (R(9) * (b + e) - (a + f)) * R(0.0625);
}

// Scheduling fence placed after a cell's gathered loads: the compiler may not
// move the arithmetic that uses them above it, nor the loads below it, so all
// of the cell's loads are in flight before the first wait.
__device__ inline void loads_issued() { __builtin_amdgcn_sched_barrier(0); }

// A field on the cross-shaped stencil of reach 2, gathered into registers so
// that all of its loads are in flight together: v[0] is the cell, v[1 + 4d + t]
// the cells -2, -1, +1, +2 (t = 0..3) steps along axis d.
template <typename T>
__device__ inline void gather13(const T* __restrict__ q, const CellIdx& c, T (&v)[13]) {
    v[0] = q[c.self()];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v[1 + 4 * d] = q[c.sh(d, -2)];
        v[2 + 4 * d] = q[c.sh(d, -1)];
        v[3 + 4 * d] = q[c.sh(d, 1)];
        v[4 + 4 * d] = q[c.sh(d, 2)];
    }
}

// The gathered value s steps along d (|s| <= 2).
template <typename T>
__device__ inline T g13(const T (&v)[13], int d, int s) {
    return s == 0 ? v[0] : v[1 + 4 * d + (s < 0 ? s + 2 : s + 1)];
}

// I4 onto face P + (s + 1/2) e_d from gathered values (same operations as i4).
template <typename T>
__device__ inline T i4g(const T (&v)[13], int d, int s) {
    const T a = g13(v, d, s - 1), b = g13(v, d, s), e = g13(v, d, s + 1), f = g13(v, d, s + 2);
    return (T(9) * (b + e) - (a + f)) * T(0.0625);
}

// I4 of gathered values evaluated in the arithmetic of R (same operations as i4r).
template <typename R, typename T>
__device__ inline R i4gr(const T (&v)[13], int d, int s) {
    const R a = (R)g13(v, d, s - 1), b = (R)g13(v, d, s), e = (R)g13(v, d, s + 1),
            f = (R)g13(v, d, s + 2);
    return (R(9) * (b + e) - (a + f)) * R(0.0625);
}

// Gauss-I4 cell derivative along d from gathered values (same operations as dgauss).
template <typename T>
__device__ inline T dgauss13(const T (&v)[13], int d, T inv_h) {
    return (i4g(v, d, 0) - i4g(v, d, -1)) * inv_h;
}

// The cross of reach 1: v[0] the cell, v[1 + 2d] and v[2 + 2d] the cells -1
// and +1 along axis d.
template <typename T>
__device__ inline void gather7(const T* __restrict__ q, const CellIdx& c, T (&v)[7]) {
    v[0] = q[c.self()];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v[1 + 2 * d] = q[c.sh(d, -1)];
        v[2 + 2 * d] = q[c.sh(d, 1)];
    }
}

// The five cells -2..2 along axis d: v[s + 2].
template <typename T>
__device__ inline void gather_line(const T* __restrict__ q, const CellIdx& c, int d, T (&v)[5]) {
#pragma unroll
    for (int s = -2; s <= 2; ++s) v[s + 2] = q[c.sh(d, s)];
}

// I4 onto face s + 1/2 along the gathered line (same operations as i4r).
template <typename R, typename T>
__device__ inline R i4l(const T (&v)[5], int s) {
    const R a = (R)v[s + 1], b = (R)v[s + 2], e = (R)v[s + 3], f = (R)v[s + 4];
    return (R(9) * (b + e) - (a + f)) * R(0.0625);
}

// Gauss-theorem cell derivative along d from I4 face values.
template <typename T>
__device__ inline T dgauss(const T* __restrict__ q, const CellIdx& c, int d, T inv_h) {
    return (i4(q, c, d, 0) - i4(q, c, d, -1)) * inv_h;
}

__device__ inline int flat_tid() { return threadIdx.x + blockDim.x * threadIdx.y; }
__device__ inline unsigned num_blocks() { return gridDim.x * gridDim.y * gridDim.z; }

constexpr unsigned kXcds = 8;   // accelerator complex dies, each with its own L2

// Logical number of this block.  The blocks of a launch are dealt to the XCDs
// round-robin in order of their hardware number; renumbering them so that each
// XCD receives one contiguous range of logical numbers keeps neighbouring tiles,
// and the halo cells they share, in the same XCD's L2.  Tiles, members and
// reduction partials are all indexed by the logical number.
__device__ inline unsigned flat_bid() {
    const unsigned f = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned B = num_blocks();
    return B % kXcds == 0 ? (f % kXcds) * (B / kXcds) + f / kXcds : f;
}

// Logical 3D block coordinates (x fastest) of this block.
struct BlockXYZ {
    int x, y, z;
};
__device__ inline BlockXYZ block_xyz() {
    const unsigned L = flat_bid();
    return {(int)(L % gridDim.x), (int)((L / gridDim.x) % gridDim.y),
            (int)(L / (gridDim.x * gridDim.y))};
}

// Store that streams past the caches: the written line does not displace
// lines still to be read (a z-march's halo rows and planes) from L2.
template <typename T>
__device__ inline void stream_st(T* p, T v) { __builtin_nontemporal_store(v, p); }

// Load of a value no other tile reads (a z-march's own point values), with
// the same streaming hint.
template <typename T>
__device__ inline T stream_ld(const T* p) { return __builtin_nontemporal_load(p); }

// Barrier that orders only LDS accesses across the block: it waits for this
// wave's LDS operations, not for its global loads in flight, so loads issued
// for a later plane of a z-march stay in flight across it (a plain
// __syncthreads() also waits for every outstanding global access).
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <bool MAX>
__device__ inline double combine(double a, double b) {
    if constexpr (MAX) return a > b ? a : b;
    else return a + b;
}

template <bool MAX>
__device__ inline double wave_reduce(double v) {
    for (int off = 32; off > 0; off >>= 1) v = combine<MAX>(v, __shfl_down(v, off, 64));
    return v;
}

// wave_reduce of NV values at once: each step's shuffles of all components
// are issued together (one LDS round trip per step rather than one per step
// and component), each component combined in wave_reduce's order.
template <int NV, unsigned MAXMASK>
__device__ inline void wave_reduce_all(double (&v)[NV]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double t[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) t[c] = __shfl_down(v[c], off, 64);
#pragma unroll
        for (int c = 0; c < NV; ++c)
            v[c] = ((MAXMASK >> c) & 1u) ? combine<true>(v[c], t[c]) : combine<false>(v[c], t[c]);
    }
}

// Block reduction of NV values over the block's waves (up to 16 waves of 64);
// component c uses max when bit c of MAXMASK is set, else a sum.  Result valid
// in thread 0.  The order of operations is fixed, so the result is bitwise
// reproducible.  LDS_ONLY: the barriers order only LDS accesses (lds_barrier),
// so global loads and stores in flight stay in flight across the reduction.
template <int NV, unsigned MAXMASK, bool LDS_ONLY = false>
__device__ inline void block_reduce(double (&v)[NV], double* lds) {
    const int tid = flat_tid();
    const int lane = tid & 63, wave = tid >> 6;
    const int nw = (blockDim.x * blockDim.y + 63) >> 6;
    wave_reduce_all<NV, MAXMASK>(v);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) lds[wave * NV + c] = v[c];
    if (LDS_ONLY) lds_barrier();
    else __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double acc = lds[c];
            for (int w = 1; w < nw; ++w)
                acc = ((MAXMASK >> c) & 1u) ? combine<true>(acc, lds[w * NV + c]) : acc + lds[w * NV + c];
            v[c] = acc;
        }
    }
    if (LDS_ONLY) lds_barrier();
    else __syncthreads();
}

// Per-block partials of a grid-wide reduction: thread 0 writes the block's
// totals to part[c * num_blocks + block].  No fence is needed: the partials
// are consumed by a later kernel on the same stream.
template <int NV, unsigned MAXMASK, bool LDS_ONLY = false>
__device__ inline void block_partials(double (&v)[NV], double* part) {
    __shared__ double lds[16 * NV];
    block_reduce<NV, MAXMASK, LDS_ONLY>(v, lds);
    if (flat_tid() == 0) {
        const unsigned nb = num_blocks(), bid = flat_bid();
#pragma unroll
        for (int c = 0; c < NV; ++c) part[(size_t)c * nb + bid] = v[c];
    }
}

// Totals of count partials per column starting at `first`, columns nbt apart.
template <int NV, unsigned MAXMASK, bool LDS_ONLY = false>
__device__ inline void reduce_partials_strided(const double* __restrict__ part, size_t nbt,
                                               size_t first, unsigned nb, double (&out)[NV]) {
    __shared__ double lds[16 * NV];
    __shared__ double tot[NV];
    const int tid = flat_tid();
    const int nthr = blockDim.x * blockDim.y;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        const bool mx = (MAXMASK >> c) & 1u;
        double acc = mx ? -__builtin_inf() : 0.0;
        for (unsigned b = tid; b < nb; b += nthr) {
            const double x = part[(size_t)c * nbt + first + b];
            acc = mx ? (x > acc ? x : acc) : acc + x;
        }
        out[c] = acc;
    }
    block_reduce<NV, MAXMASK, LDS_ONLY>(out, lds);
    if (tid == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) tot[c] = out[c];
    if (LDS_ONLY) lds_barrier();
    else __syncthreads();
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c] = tot[c];
}

// Totals of one member's partials: an earlier kernel with nbt blocks in all
// wrote column c of block b at part[c nbt + b]; member m owns the blocks
// [m nbt/batch, (m+1) nbt/batch).
template <int NV, unsigned MAXMASK, bool LDS_ONLY = false>
__device__ inline void reduce_member(const double* __restrict__ part, unsigned nbt, int batch,
                                     int m, double (&out)[NV]) {
    const unsigned per = nbt / (unsigned)batch;
    double tmp[NV];
    reduce_partials_strided<NV, MAXMASK, LDS_ONLY>(part, nbt, (size_t)m * per, per, tmp);
#pragma unroll
    for (int c = 0; c < NV; ++c) out[c] = tmp[c];
}

// Totals of partials written by an earlier kernel with `nb` blocks.  Every
// block of the calling kernel computes the same totals in the same order
// (bitwise identical, deterministic); all threads receive them.
template <int NV, unsigned MAXMASK>
__device__ inline void reduce_partials(const double* __restrict__ part, unsigned nb,
                                       double (&out)[NV]) {
    reduce_partials_strided<NV, MAXMASK>(part, nb, 0, nb, out);
}

// Round to nearest even FP32 -> BF16 (bit pattern); NaN stays NaN.
__host__ __device__ inline uint16_t f2bf(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Pressure deviation p(rho) - p_ref for rho = rho_ref + r (p_ref = C rho_ref^gamma),
// written with log1p/expm1 so that it stays accurate for small r in FP32.
__device__ inline double pdev(double r, double rho_ref, double p_ref, double gamma) {
    return p_ref * expm1(gamma * log1p(r / rho_ref));
}
__device__ inline float pdev(float r, double rho_ref, double p_ref, double gamma) {
    return (float)p_ref * expm1f((float)gamma * log1pf(r / (float)rho_ref));
}

}  // namespace pisoc
