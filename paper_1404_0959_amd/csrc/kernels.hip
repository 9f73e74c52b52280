// kernels.hip -- HIP kernels of one PISO + Equilibrium-Eulerian dust step on
// gfx950, templated on the storage/compute type T (double, or float for the
// FP32 mode whose reductions stay in double).
//
// Density and pressure are stored as deviations r = rho - rho_ref and
// p - p_ref so that FP32 storage keeps the digits of the fluctuations.
// Face mass fluxes are stored once per face (array d at the offset of the cell
// below the face), and every divergence is taken from stored faces, so the
// total gas and dust mass telescope exactly.
#include "device.hpp"
#include "launch.hpp"

namespace pisoc {

// The member of this block (blocks of member m have blockIdx.z in
// [m nz, (m+1) nz)), its z-block and its first cell.
#define MEMBER(ph)                                                           \
    const BlockXYZ bp_ = block_xyz();                                        \
    const int mem_ = bp_.z / (ph).nz;                                        \
    const int bz_ = bp_.z - mem_ * (ph).nz;                                  \
    const size_t base_ = (size_t)mem_ * (ph).N;                              \
    (void)bz_;                                                               \
    (void)base_;
// true in one thread of the member's first block
#define MEMBER_FIRST() (bp_.x == 0 && bp_.y == 0 && bz_ == 0 && flat_tid() == 0)
#define FOR_CELLS(ph)                                                        \
    const int ci_ = bp_.x * blockDim.x + threadIdx.x;                        \
    const int cj_ = bp_.y * blockDim.y + threadIdx.y;                        \
    for (int zz_ = 0; zz_ < (ph).cz; ++zz_) {                                \
        const int ck_ = bz_ * (ph).cz + zz_;                                 \
        if (ci_ >= (ph).n || cj_ >= (ph).n || ck_ >= (ph).n) continue;       \
        const CellIdx c((ph).n, ci_, cj_, ck_, base_);                       \
        const size_t P = c.self();
#define END_CELLS }

__host__ __device__ static inline size_t ncell(const Phys& ph) { return ph.NT; }

// Largest dust Courant number at which the dust update (4 Jacobi sweeps and the
// conservative finish) damps every Fourier mode of a uniform drift: the root
// y = 0.8130 of (1 + y^6)^2 = 1 + y^2 over the I4 transport symbol's maximum
// 1.2739.
constexpr double kDustCourantMax = 0.638;

// ---------------------------------------------------------------- utilities
template <typename T>
__global__ void k_cast_in(const double* __restrict__ src, T* __restrict__ dst, size_t count,
                          double shift) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = (T)(src[i] - shift);
}

template <typename T>
__global__ void k_cast_out(const T* __restrict__ src, double* __restrict__ dst, size_t count,
                           double shift) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = (double)src[i] + shift;
}

// p = p_ref + p_dev(r) as FP64 (one member)
template <typename T>
__global__ void k_pressure_out(double gamma, double rho_ref, double p_ref, const T* __restrict__ r,
                               double* __restrict__ dst, size_t count, const double* temp,
                               double R) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride)
        dst[i] = temp ? (rho_ref + (double)r[i]) * R * temp[i]
                      : p_ref + pdev((double)r[i], rho_ref, p_ref, gamma);
}

// dst[i] = v (FP64 fill).
__global__ void k_fill(double* __restrict__ dst, size_t count, double v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = v;
}

// Initial face mass fluxes phi_d = I4(rho) I4(u_d) A.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_phi(Phys ph, const DevState* st, const T* __restrict__ r,
                                                     const T* __restrict__ u, T* __restrict__ phi) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T rref = (T)(st + mem_)->rho_ref, A = (T)ph.A;
    FOR_CELLS(ph)
#pragma unroll
    for (int d = 0; d < 3; ++d)
        phi[d * N + P] = (rref + i4(r, c, d, 0)) * i4(u + d * N, c, d, 0) * A;
    END_CELLS
}

// Two-way coupling, initial dust mass fluxes fd_d = I4(sum_j rho_j) I4(u_d) A
// (the dust moving with the gas: its drift needs Du/Dt, unknown before the
// first step).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_fd(Phys ph, int ncls, const T* __restrict__ rhoj,
                                                    const T* __restrict__ u, T* __restrict__ fd) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T A = (T)ph.A;
    FOR_CELLS(ph)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T q[4];
#pragma unroll
        for (int s = -1; s <= 2; ++s) {
            T acc = T(0);
            for (int j = 0; j < ncls; ++j) acc += rhoj[j * N + c.sh(d, s)];
            q[s + 1] = acc;
        }
        const T rd = (T(9) * (q[1] + q[2]) - (q[0] + q[3])) * T(0.0625);
        fd[d * N + P] = rd * i4(u + d * N, c, d, 0) * A;
    }
    END_CELLS
}

// ---------------------------------------------------------------- time step
// Convective Courant rate sigma_P = sum_f |phi_f| / (2 rho_P V) of a cell
// from its own (fp) and lower (fm) face fluxes and its density deviation r.
template <typename T>
__device__ inline double courant_rate(const T (&fp)[3], const T (&fm)[3], T r, double rref,
                                      double V) {
    double f = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) f += fabs((double)fp[d]) + fabs((double)fm[d]);
    return f / (2.0 * (rref + (double)r) * V);
}

// Per-block maxima of the Courant rate; the next kernel turns them into dt.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cfl(Phys ph, const DevState* st, const T* __restrict__ r,
                                                const T* __restrict__ phi, double* part) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    double v[1] = {0.0};
    FOR_CELLS(ph)
    T fp[3], fm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        fp[d] = phi[d * N + P];
        fm[d] = phi[d * N + c.sh(d, -1)];
    }
    const T rP = r[P];
    loads_issued();
    const double s = courant_rate(fp, fm, rP, (st + mem_)->rho_ref, ph.V);
    v[0] = s > v[0] ? s : v[0];
    END_CELLS
    block_partials<1, 1u>(v, part);
}

// Adaptive time step dt = min(cfl / sigma, growth dt_prev, dt_max) (or
// dt_fixed) from the Courant partials; density predictor
// rho* = rho^n - dt div(phi^n); momentum diagonal
// a_P = rho*/dt + (9/16) div(phi^n) + 6 mu / h^2; div u^n (Gauss-I4); p(rho^n).
__device__ inline double predict_dt(double sigma, double dt_prev, double dt_fixed, double cfl,
                                    double growth, double dt_max) {
    if (dt_fixed > 0.0) return dt_fixed;
    double dtd = sigma > 0.0 ? cfl / sigma : __builtin_inf();
    if (growth * dt_prev < dtd) dtd = growth * dt_prev;
    if (dt_max > 0.0 && dt_max < dtd) dtd = dt_max;
    return dtd;
}

// From the face fluxes of the cell (own fp, lower fm) and u^n_d on the line
// along d (ul[d][5]): rho*, a_P, div u^n; p(rho^n) from rho^n.
template <typename T>
__device__ inline void predict_cell(const T (&fp)[3], const T (&fm)[3], const T (&ul)[3][5], T rnP,
                                    T dt, T inv_V, T inv_h, T diag_visc, T rref, double pref,
                                    double gamma, T& rs, T& a, T& divu, T& pn) {
    T dphi = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) dphi += fp[d] - fm[d];
    dphi *= inv_V;
    const T r = rnP - dt * dphi;
    rs = r;
    a = (rref + r) / dt + T(0.5625) * dphi + diag_visc;
    T du = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) du += i4l<T>(ul[d], 0) - i4l<T>(ul[d], -1);
    divu = du * inv_h;
    pn = pdev(rnP, (double)rref, pref, gamma);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_predict(Phys ph, DevState* st, const double* part_cfl,
                                                    unsigned nb, double dt_fixed, double cfl,
                                                    double growth, double dt_max,
                                                    const T* __restrict__ rn, const T* __restrict__ un,
                                                    const T* __restrict__ phi, T* __restrict__ rs,
                                                    T* __restrict__ aP, T* __restrict__ divu,
                                                    T* __restrict__ pn) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    double sg[1];
    reduce_member<1, 1u>(part_cfl, nb, ph.batch, mem_, sg);
    const double dtd = predict_dt(sg[0], (st + mem_)->dt_prev, dt_fixed, cfl, growth, dt_max);
    double bc[3] = {1.0, 1.0, 0.0};
    if (ph.bdf2) bdf2_coef(dtd, (st + mem_)->dt_prev, bc);
    if (MEMBER_FIRST()) {
#pragma unroll
        for (int q = 0; q < 3; ++q) (st + mem_)->bdf[q] = bc[q];
        if (!(dtd > 0.0) || !isfinite(dtd)) (st + mem_)->flags |= 16;  // bad dt
        (st + mem_)->sigma = sg[0];
        (st + mem_)->dt = dtd;
    }
    const T dt = (T)dtd;
    const T inv_V = (T)ph.inv_V, inv_h = (T)ph.inv_h;
    const T diag_visc = (T)(6.0 * ph.mu * ph.inv_h2);
    FOR_CELLS(ph)
    T fp[3], fm[3], ul[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        fp[d] = phi[d * N + P];
        fm[d] = phi[d * N + c.sh(d, -1)];
        gather_line(un + d * N, c, d, ul[d]);
    }
    const T rnP = rn[P];
    loads_issued();
    T r, a, dv, p;
    predict_cell(fp, fm, ul, rnP, dt, inv_V, inv_h, diag_visc, (T)(st + mem_)->rho_ref,
                 (st + mem_)->p_ref, ph.gamma, r, a, dv, p);
    if (ph.fourier)   // ideal gas at T^n
        p = (T)(((st + mem_)->rho_ref + (double)rnP) * ph.R * ph.tn[P] - (st + mem_)->p_ref);
    if (ph.bdf2) {    // rho* = (c1 rho^n - c2 rho^{n-1} - dt div phi) / c0, a_P with c0 rho*/dt
        double dphi = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) dphi += (double)fp[d] - (double)fm[d];
        dphi *= ph.inv_V;
        const double rr = (bc[1] * (double)rnP - bc[2] * ph.rm1[P] - dtd * dphi) / bc[0];
        r = (T)rr;
        a = (T)(bc[0] * ((st + mem_)->rho_ref + rr) / dtd + 0.5625 * dphi + 6.0 * ph.mu * ph.inv_h2);
    }
    rs[P] = r;
    aP[P] = a;
    divu[P] = dv;
    pn[P] = p;
    END_CELLS
}

// Explicit momentum source s = rho^n u^n / dt + (mu/3) grad(div u^n).
template <typename T>
__device__ inline void mom_source_cell(const T (&dv)[13], const T (&uv)[3], T rho, T dt, T m3,
                                       T inv_h, T (&out)[3]) {
#pragma unroll
    for (int m = 0; m < 3; ++m) out[m] = rho * uv[m] / dt + m3 * dgauss13(dv, m, inv_h);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_mom_source(Phys ph, const DevState* st,
                                                       const T* __restrict__ rn,
                                                       const T* __restrict__ un,
                                                       const T* __restrict__ divu,
                                                       T* __restrict__ s) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T dt = (T)(st + mem_)->dt;
    const T m3 = (T)(ph.mu / 3.0), inv_h = (T)ph.inv_h;
    FOR_CELLS(ph)
    T dv[13], uv[3];
    gather13(divu, c, dv);
#pragma unroll
    for (int m = 0; m < 3; ++m) uv[m] = un[m * N + P];
    const T rho = (T)(st + mem_)->rho_ref + rn[P];
    loads_issued();
    T out[3];
    mom_source_cell(dv, uv, rho, dt, m3, inv_h, out);
    if (ph.bdf2) {   // (c1 rho^n u^n - c2 rho^{n-1} u^{n-1}) / dt
        const double* bc = (st + mem_)->bdf;
        const double rm = (st + mem_)->rho_ref + ph.rm1[P];
#pragma unroll
        for (int m = 0; m < 3; ++m)
            out[m] = (T)((bc[1] * (double)rho * (double)uv[m] - bc[2] * rm * ph.um1[m * N + P]) /
                         (double)dt + (double)m3 * (double)dgauss13(dv, m, inv_h));
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) s[m * N + P] = out[m];
    END_CELLS
}

// Two-way coupling: the momentum equation becomes the mixture's, density
// rho_m = rho + rho_d (rho_d = sum_j rho_j) convected by the mixture mass flux
// F_m = phi + F_d (F_d: the dust mass fluxes of the last step).  From the gas
// predictor's a_P and source: a_P += rho_d^n / dt - (7/16) div F_d, which makes
// it rho_m*/dt + (9/16) div F_m + 6 mu/h^2 with rho_m* = rho_m^n - dt div F_m;
// s += rho_d^n u^n / dt + (rho_m^n - <rho_m>) g; F_m is written for the
// momentum sweeps and H/a_P.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mixture(Phys ph, const DevState* st, int ncls,
                                                    const T* __restrict__ rn,
                                                    const T* __restrict__ un,
                                                    const T* __restrict__ rhoj,
                                                    const T* __restrict__ phi,
                                                    const T* __restrict__ fd, T* __restrict__ fm,
                                                    T* __restrict__ aP, T* __restrict__ src) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T dt = (T)(st + mem_)->dt, inv_V = (T)ph.inv_V;
    const double rref = (st + mem_)->rho_ref, mean = (st + mem_)->rhom_mean;
    FOR_CELLS(ph)
    T rd = T(0);
    for (int j = 0; j < ncls; ++j) rd += rhoj[j * N + P];
    T dfd = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T fo = fd[d * N + P];
        dfd += fo - fd[d * N + c.sh(d, -1)];
        fm[d * N + P] = phi[d * N + P] + fo;
    }
    dfd *= inv_V;
    aP[P] += rd / dt - T(0.4375) * dfd;
    const double rm = rref + (double)rn[P] + (double)rd;
#pragma unroll
    for (int m = 0; m < 3; ++m)
        src[m * N + P] += rd * un[m * N + P] / dt + (T)((rm - mean) * ph.g[m]);
    END_CELLS
}

// One Jacobi sweep of the momentum predictor,
//   u_out = (s - N(u_in) - grad p^n) / a_P        (HBYA = false), or
// the corrector's HbyA = (s - N(u_in)) / a_P     (HBYA = true), which also
// stores w = rho_k / a_P and p_dev(rho_k) of the current density iterate.
// N(u) = (1/V) sum_f phi_f^out I4(u)_f - (9/16) div(phi) u_P - mu sum_nb u_nb / h^2.
template <typename T, bool HBYA>
__device__ inline void mom_cell(const T (&u)[3][13], const T (&pv)[13], const T (&fp)[3],
                                const T (&fm)[3], const T (&sv)[3], T a, T inv_V, T inv_h,
                                T mu_h2, T (&out)[3], T& ia) {
    T dphi = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) dphi += fp[d] - fm[d];
    dphi *= inv_V;
    ia = T(1) / a;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        T conv = T(0), nb = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            conv += fp[d] * i4g(u[m], d, 0) - fm[d] * i4g(u[m], d, -1);
            nb += g13(u[m], d, 1) + g13(u[m], d, -1);
        }
        T off = conv * inv_V - T(0.5625) * dphi * u[m][0] - mu_h2 * nb;
        T rhs = sv[m] - off;
        if (!HBYA) rhs -= (i4g(pv, m, 0) - i4g(pv, m, -1)) * inv_h;
        out[m] = rhs * ia;
    }
}

template <typename T, bool HBYA>
__global__ void __launch_bounds__(kBlock) k_mom_sweep(Phys ph, const DevState* st, const T* __restrict__ uin,
                                                      T* __restrict__ uout, const T* __restrict__ phi,
                                                      const T* __restrict__ aP, const T* __restrict__ s,
                                                      const T* __restrict__ pn, const T* __restrict__ rk,
                                                      T* __restrict__ w, T* __restrict__ p0) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T inv_V = (T)ph.inv_V, inv_h = (T)ph.inv_h;
    const T mu_h2 = (T)(ph.mu * ph.inv_h2);
    FOR_CELLS(ph)
    // every load of the cell first (the 13-point stencils of the three
    // components and of p^n, the six fluxes), then the arithmetic
    T u[3][13], pv[13], fp[3], fm[3], sv[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) gather13(uin + m * N, c, u[m]);
    if (!HBYA) gather13(pn, c, pv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        fp[d] = phi[d * N + P];
        fm[d] = phi[d * N + c.sh(d, -1)];
        sv[d] = s[d * N + P];
    }
    const T a = aP[P];
    const T rkP = HBYA ? rk[P] : T(0);
    loads_issued();
    T out[3], ia;
    mom_cell<T, HBYA>(u, pv, fp, fm, sv, a, inv_V, inv_h, mu_h2, out, ia);
#pragma unroll
    for (int m = 0; m < 3; ++m) uout[m * N + P] = out[m];
    if (HBYA) {
        w[P] = ((T)(st + mem_)->rho_ref + rkP) * ia;
        p0[P] = ph.fourier   // ideal gas at the predicted temperature T*
                    ? (T)(((st + mem_)->rho_ref + (double)rkP) * ph.R * ph.ts[P] - (st + mem_)->p_ref)
                    : pdev(rkP, (st + mem_)->rho_ref, (st + mem_)->p_ref, ph.gamma);
    }
    END_CELLS
}

// The same sweep as a z-march over a 64 x 8 column tile (n a multiple of
// 64): each velocity component and p^n are read once per cell from HBM;
// their x-y neighbours of the current plane come from LDS tiles (halo 2), the
// z neighbours from five-plane register queues; the fluxes phi_x, phi_y of the
// plane sit in LDS with the one low-side neighbour each needs, phi_z in a
// two-plane queue.  All loads of plane k + 1 (queue heads, own-cell values and
// this thread's share of the halo) are issued before plane k's LDS-only
// barriers.  The per-cell arithmetic is mom_cell, as in k_mom_sweep.
// (FP32: at least four wavefronts per SIMD, two blocks per CU, with the
// halo queue in registers)
template <typename T, bool HBYA>
__global__ void __launch_bounds__(kTX * kTY, sizeof(T) == 4 ? 4 : 2) k_mom_sweep_tiled(
    Phys ph, const DevState* st, const T* __restrict__ uin, T* __restrict__ uout,
    const T* __restrict__ phi, const T* __restrict__ aP, const T* __restrict__ s,
    const T* __restrict__ pn, const T* __restrict__ rk, T* __restrict__ w, T* __restrict__ p0) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T inv_V = (T)ph.inv_V, inv_h = (T)ph.inv_h;
    const T mu_h2 = (T)(ph.mu * ph.inv_h2);
    const int n = ph.n, cz = ph.cz;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + kTX * ty;
    const int i0 = bp_.x * kTX, j0 = bp_.y * kTY;
    const int k0 = bz_ * cz;
    const int k1 = k0 + cz < n ? k0 + cz : n;
    const size_t nn = (size_t)n * n;
    constexpr int NF = HBYA ? 3 : 4;            // fields with a halo-2 tile: u_x, u_y, u_z, p^n
    constexpr int kHalo = 4 * kTX + 4 * kTY;    // halo cells of one such tile
    constexpr int kJobs = NF * kHalo + kTY + kTX;
    constexpr int kPer = (kJobs + kTX * kTY - 1) / (kTX * kTY);
    // one LDS array (so that every store to it is an LDS store): the halo-2
    // tiles of u_x, u_y, u_z (and p^n), phi_x at x = i0 - 1 .. i0 + 63, phi_y at
    // y = j0 - 1 .. j0 + 7, and a scratch slot per thread for idle halo jobs
    constexpr int kUW = kTX + 4, kUS = (kTY + 4) * kUW;
    constexpr int kFX = NF * kUS, kFY = kFX + kTY * (kTX + 1), kDum = kFY + (kTY + 1) * kTX;
    __shared__ T lds[kDum + kTX * kTY];
    auto U = [&](int f, int y, int x) -> T& { return lds[f * kUS + y * kUW + x]; };
    auto FX = [&](int y, int x) -> T& { return lds[kFX + y * (kTX + 1) + x]; };
    auto FY = [&](int y, int x) -> T& { return lds[kFY + y * kTX + x]; };
    auto wr = [n](int a) { return a < 0 ? a + n : (a >= n ? a - n : a); };
    const size_t col = base_ + (size_t)(i0 + tx) + (size_t)n * (j0 + ty);
    // this thread's halo jobs: source array, offset within a plane, LDS slot
    typedef const T __attribute__((address_space(1)))* gptr;   // global memory
    gptr hsrc[kPer];
    size_t hoff[kPer];
    int hdst[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int jb = tid + q * kTX * kTY;
        hsrc[q] = (gptr)uin;
        hoff[q] = col;
        hdst[q] = kDum + tid;
        if (jb < NF * kHalo) {
            const int f = jb / kHalo, h = jb - f * kHalo;
            const gptr src = (gptr)(f < 3 ? uin + (size_t)f * N : pn);
            if (h < 4 * kTX) {                  // rows j0-2, j0-1, j0+8, j0+9
                const int row = h / kTX, x = h - row * kTX;
                const int yy = row < 2 ? row : kTY + row;
                hsrc[q] = src;
                hoff[q] = base_ + (size_t)(i0 + x) + (size_t)n * wr(j0 - 2 + yy);
                hdst[q] = f * kUS + yy * kUW + x + 2;
            } else {                            // columns i0-2, i0-1, i0+64, i0+65
                const int t = h - 4 * kTX, c4 = t / kTY, y = t - c4 * kTY;
                const int xx = c4 < 2 ? c4 : kTX + c4;
                hsrc[q] = src;
                hoff[q] = base_ + (size_t)wr(i0 - 2 + xx) + (size_t)n * (j0 + y);
                hdst[q] = f * kUS + (y + 2) * kUW + xx;
            }
        } else if (jb < NF * kHalo + kTY) {     // phi_x at x = i0 - 1
            const int y = jb - NF * kHalo;
            hsrc[q] = (gptr)phi;
            hoff[q] = base_ + (size_t)wr(i0 - 1) + (size_t)n * (j0 + y);
            hdst[q] = kFX + y * (kTX + 1);
        } else if (jb < kJobs) {                // phi_y at y = j0 - 1
            const int x = jb - NF * kHalo - kTY;
            hsrc[q] = (gptr)(phi + N);
            hoff[q] = base_ + (size_t)(i0 + x) + (size_t)n * wr(j0 - 1);
            hdst[q] = kFY + x;
        }
    }
    // queues and the values of the first plane
    T uq[3][5], pq[5], fzq[2];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int t = 0; t < 5; ++t) uq[m][t] = uin[(size_t)m * N + col + nn * wr(k0 - 2 + t)];
#pragma unroll
    for (int t = 0; t < 5; ++t) pq[t] = HBYA ? T(0) : pn[col + nn * wr(k0 - 2 + t)];
    fzq[0] = phi[2 * N + col + nn * wr(k0 - 1)];
    fzq[1] = phi[2 * N + col + nn * k0];
    T cfx = phi[col + nn * k0], cfy = phi[N + col + nn * k0], ca = aP[col + nn * k0];
    T cs[3], crk = HBYA ? rk[col + nn * k0] : T(0);
#pragma unroll
    for (int m = 0; m < 3; ++m) cs[m] = s[(size_t)m * N + col + nn * k0];
    auto clampk = [](int a, int hi) { return a < hi ? a : hi; };
    // halo values of planes kk .. kk + kHQ - 1 (hq[.][0] goes to LDS at plane
    // kk).  FP32: a halo value is loaded with the owner tile's queue head of
    // the same plane, four planes ahead, so that both reads of the line fall
    // together in L2; FP64 loads it two planes ahead (its registers are full)
    constexpr int kHQ = sizeof(T) == 4 ? 3 : 1;
    T hq[kPer][kHQ];
#pragma unroll
    for (int q = 0; q < kPer; ++q)
#pragma unroll
        for (int t = 0; t < kHQ; ++t)
            hq[q][t] = hsrc[q][nn * (size_t)wr(clampk(k0 + t, k1 - 1)) + hoff[q]];
    // values of plane k0 + 1 and the queue head at k0 + 3, rotated in after plane k0
    T nu[3], np = T(0), nfz, nfx, nfy, na, ns[3], nrk = T(0), nh[kPer];
    // queue heads at plane kq, halo values at kh, own values at kv
    auto prefetch = [&](int kq, int kh, int kv) {
        const size_t pq3 = nn * (size_t)wr(kq), phh = nn * (size_t)wr(kh), pv = nn * (size_t)wr(kv);
#pragma unroll
        for (int m = 0; m < 3; ++m) nu[m] = uin[(size_t)m * N + col + pq3];
        if (!HBYA) np = pn[col + pq3];
        nfz = phi[2 * N + col + pv];
        nfx = phi[col + pv];
        nfy = phi[N + col + pv];
        na = stream_ld(aP + col + pv);
#pragma unroll
        for (int m = 0; m < 3; ++m) ns[m] = stream_ld(s + (size_t)m * N + col + pv);
        if (HBYA) nrk = stream_ld(rk + col + pv);
#pragma unroll
        for (int q = 0; q < kPer; ++q) nh[q] = hsrc[q][phh + hoff[q]];
    };
    // last planes the chunk needs: queue heads k1 + 1, halo and own values k1 - 1
    prefetch(clampk(k0 + 3, k1 + 1), clampk(k0 + kHQ, k1 - 1), clampk(k0 + 1, k1 - 1));
    for (int kk = k0; kk < k1; ++kk) {
        const size_t pl = nn * (size_t)kk;
        // plane kk into LDS
#pragma unroll
        for (int m = 0; m < 3; ++m) U(m, ty + 2, tx + 2) = uq[m][2];
        if (!HBYA) U(NF - 1, ty + 2, tx + 2) = pq[2];
        FX(ty, tx + 1) = cfx;
        FY(ty + 1, tx) = cfy;
#pragma unroll
        for (int q = 0; q < kPer; ++q) lds[hdst[q]] = hq[q][0];
        lds_barrier();
        T u[3][13], pv[13], fp[3], fm[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            u[m][0] = uq[m][2];
            u[m][1] = U(m, ty + 2, tx);
            u[m][2] = U(m, ty + 2, tx + 1);
            u[m][3] = U(m, ty + 2, tx + 3);
            u[m][4] = U(m, ty + 2, tx + 4);
            u[m][5] = U(m, ty, tx + 2);
            u[m][6] = U(m, ty + 1, tx + 2);
            u[m][7] = U(m, ty + 3, tx + 2);
            u[m][8] = U(m, ty + 4, tx + 2);
            u[m][9] = uq[m][0];
            u[m][10] = uq[m][1];
            u[m][11] = uq[m][3];
            u[m][12] = uq[m][4];
        }
        if (!HBYA) {
            constexpr int f = NF - 1;
            pv[0] = pq[2];
            pv[1] = U(f, ty + 2, tx);
            pv[2] = U(f, ty + 2, tx + 1);
            pv[3] = U(f, ty + 2, tx + 3);
            pv[4] = U(f, ty + 2, tx + 4);
            pv[5] = U(f, ty, tx + 2);
            pv[6] = U(f, ty + 1, tx + 2);
            pv[7] = U(f, ty + 3, tx + 2);
            pv[8] = U(f, ty + 4, tx + 2);
            pv[9] = pq[0];
            pv[10] = pq[1];
            pv[11] = pq[3];
            pv[12] = pq[4];
        }
        fp[0] = FX(ty, tx + 1);
        fm[0] = FX(ty, tx);
        fp[1] = FY(ty + 1, tx);
        fm[1] = FY(ty, tx);
        fp[2] = fzq[1];
        fm[2] = fzq[0];
        T out[3], ia;
        mom_cell<T, HBYA>(u, pv, fp, fm, cs, ca, inv_V, inv_h, mu_h2, out, ia);
#pragma unroll
        for (int m = 0; m < 3; ++m) stream_st(uout + ((size_t)m * N + col + pl), out[m]);
        if (HBYA) {
            stream_st(w + (col + pl), ((T)(st + mem_)->rho_ref + crk) * ia);
            stream_st(p0 + (col + pl),
                      ph.fourier   // ideal gas at the predicted temperature T*
                          ? (T)(((st + mem_)->rho_ref + (double)crk) * ph.R * ph.ts[col + pl] -
                                (st + mem_)->p_ref)
                          : pdev(crk, (st + mem_)->rho_ref, (st + mem_)->p_ref, ph.gamma));
        }
        lds_barrier();
        // advance the queues with the values loaded one plane ago, then load
        // the queue head at kk + 4 and the values of plane kk + 2
#pragma unroll
        for (int m = 0; m < 3; ++m) {
#pragma unroll
            for (int t = 0; t < 4; ++t) uq[m][t] = uq[m][t + 1];
            uq[m][4] = nu[m];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) pq[t] = pq[t + 1];
        pq[4] = np;
        fzq[0] = fzq[1];
        fzq[1] = nfz;
        cfx = nfx;
        cfy = nfy;
        ca = na;
#pragma unroll
        for (int m = 0; m < 3; ++m) cs[m] = ns[m];
        crk = nrk;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
#pragma unroll
            for (int t = 0; t + 1 < kHQ; ++t) hq[q][t] = hq[q][t + 1];
            hq[q][kHQ - 1] = nh[q];
        }
        prefetch(clampk(kk + 4, k1 + 1), clampk(kk + 1 + kHQ, k1 - 1), clampk(kk + 2, k1 - 1));
    }
}

// Corrector set-up: predicted fluxes phiH = I4(rho_k) I4(HbyA_d) A on the
// cell's own faces, and the pressure system M p' = b with
//   b = -[(rho_k - rho^n)/dt + div(phiH - K A snGrad p0)],  K = I4(w),
//   diag(M) = psi/dt + sum K / h^2,  psi = rho/(gamma p) = 1/(gamma C rho^(gamma-1)).
// The continuity defect is evaluated in FP64 arithmetic whatever T is (it is
// a small difference of large fluxes).  CG starts from x = 0: r = b and
// partial sums of b.(b/diag), b.b, b.b; x itself is not written (the first
// x update writes rather than adds).  With b64 non-null (FP32 storage) the
// FP64 defect is also kept (the first refinement takes the FP64 accumulator
// as zero).

// The per-cell arithmetic of the corrector set-up, shared by the gathered and
// the tiled kernel: from w and rho_k on the 13-point cross, the HbyA component
// d on the line along d, p0 on the 7-point cross and rho^n of the cell, the
// predicted fluxes on the cell's own faces phf, the FP64 defect b and diag(M).
template <typename T>
__device__ inline void corr_rhs_cell(const T (&wv)[13], const T (&rv)[13], const T (&hl)[3][5],
                                     const T (&pv)[7], T rnP, double dt, double rref, double pref,
                                     double gamma, double A, double inv_V, double inv_h,
                                     double inv_h2, double& b, T& dgT, T (&phf)[3],
                                     const double* bc = nullptr, double rm1P = 0.0) {
    double divF = 0.0, sumK = 0.0;
    const double p0P = (double)pv[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int s = -1; s <= 0; ++s) {
            const double Kf = i4gr<double>(wv, d, s);
            const double ph_f = (rref + i4gr<double>(rv, d, s)) * i4l<double>(hl[d], s) * A;
            const double sn = (s == 0 ? ((double)pv[2 + 2 * d] - p0P)
                                      : (p0P - (double)pv[1 + 2 * d])) * inv_h;
            const double F = ph_f - Kf * A * sn;
            divF += s == 0 ? F : -F;
            sumK += Kf;
            if (s == 0) phf[d] = (T)ph_f;
        }
    }
    if (bc)   // BDF2: (c0 rho_k - c1 rho^n + c2 rho^{n-1}) / dt and c0 psi / dt
        b = -((bc[0] * (double)rv[0] - bc[1] * (double)rnP + bc[2] * rm1P) / dt + divF * inv_V);
    else
        b = -(((double)rv[0] - (double)rnP) / dt + divF * inv_V);
    const double rho = rref + (double)rv[0];
    const double psidt = (bc ? bc[0] : 1.0) * rho / (gamma * (pref + p0P)) / dt;
    dgT = (T)(psidt + sumK * inv_h2);
}

// Outputs of one cell of the corrector set-up and its partial sums.
template <typename T>
__device__ inline void corr_rhs_store(size_t P, size_t N, double b, T dgT, const T (&phf)[3],
                                      double p0abs, T* __restrict__ phiH, T* __restrict__ rvec,
                                      T* __restrict__ diag, double* snap_b, double* snap_diag,
                                      double* snap_p0, double* b64, double (&v)[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) stream_st(phiH + (d * N + P), phf[d]);
    const T bT = (T)b;
    stream_st(rvec + P, bT);
    diag[P] = dgT;   // read again by every CG iteration: through the caches
    const double bd = (double)bT;
    v[0] += bd * (bd / (double)dgT);
    v[1] += b64 ? b * b : bd * bd;
    v[2] += b64 ? b * b : bd * bd;
    if (b64) stream_st(b64 + P, b);
    if (snap_b) {
        snap_b[P] = b;
        snap_diag[P] = (double)dgT;
        snap_p0[P] = p0abs;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_corr_rhs(
    Phys ph, DevState* st, const T* __restrict__ rn, const T* __restrict__ rk,
    const T* __restrict__ w, const T* __restrict__ hbya, const T* __restrict__ p0,
    T* __restrict__ phiH, T* __restrict__ rvec, T* __restrict__ diag, double* part_u,
    double* snap_b, double* snap_diag, double* snap_p0, double* b64) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const double dt = (st + mem_)->dt;
    const double rref = (st + mem_)->rho_ref, pref = (st + mem_)->p_ref;
    double v[3] = {0.0, 0.0, 0.0};
    FOR_CELLS(ph)
    // every load of the cell first, then the FP64 arithmetic
    T wv[13], rv[13], hl[3][5], pv[7];
    gather13(w, c, wv);
    gather13(rk, c, rv);
#pragma unroll
    for (int d = 0; d < 3; ++d) gather_line(hbya + d * N, c, d, hl[d]);
    gather7(p0, c, pv);
    const T rnP = rn[P];
    loads_issued();
    double b;
    T dgT, phf[3];
    corr_rhs_cell(wv, rv, hl, pv, rnP, dt, rref, pref, gamma_psi(ph), ph.A, ph.inv_V, ph.inv_h,
                  ph.inv_h2, b, dgT, phf, ph.bdf2 ? (st + mem_)->bdf : nullptr,
                  ph.bdf2 ? ph.rm1[P] : 0.0);
    corr_rhs_store(P, N, b, dgT, phf, pref + (double)pv[0], phiH, rvec, diag, snap_b, snap_diag,
                   snap_p0, b64, v);
    END_CELLS
    block_partials<3, 0u>(v, part_u);
    if (MEMBER_FIRST()) {
        (st + mem_)->pcg.it_stop = kIterInf;
        (st + mem_)->pcg.converged = 0;
        (st + mem_)->pcg.iters = 0;
    }
}

// The corrector set-up as a z-march over a 64 x 8 column tile (n a multiple
// of 64), for the reason of k_mom_sweep_tiled: w, rho_k, the HbyA x
// and y components and p0 are read once per cell from HBM and their x-y
// neighbours of the current plane come from halo-2 LDS tiles; the z
// neighbours of w, rho_k and HbyA_z come from five-plane register queues, of
// p0 from a three-plane one.  The loads of plane kk + 2 (queue heads at
// kk + 4, resp. kk + 3) are issued after plane kk's work, a plane ahead of
// their use, and clamped to the planes the chunk needs.  The per-cell
// arithmetic is corr_rhs_cell, as in k_corr_rhs.  (FP32: at least four
// wavefronts per SIMD, two blocks per CU, within 128 registers; 218 instead
// of 238 us at 256^3.)
template <typename T>
__global__ void __launch_bounds__(kTX * kTY, sizeof(T) == 4 ? 4 : 2) k_corr_rhs_tiled(
    Phys ph, DevState* st, const T* __restrict__ rn, const T* __restrict__ rk,
    const T* __restrict__ w, const T* __restrict__ hbya, const T* __restrict__ p0,
    T* __restrict__ phiH, T* __restrict__ rvec, T* __restrict__ diag, double* part_u,
    double* snap_b, double* snap_diag, double* snap_p0, double* b64) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const double dt = (st + mem_)->dt;
    const double rref = (st + mem_)->rho_ref, pref = (st + mem_)->p_ref;
    const int n = ph.n, cz = ph.cz;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + kTX * ty;
    const int i0 = bp_.x * kTX, j0 = bp_.y * kTY;
    const int k0 = bz_ * cz;
    const int k1 = k0 + cz < n ? k0 + cz : n;
    const size_t nn = (size_t)n * n;
    constexpr int NF = 5;                       // halo-2 tiles: w, rho_k, HbyA_x, HbyA_y, p0
    constexpr int kHalo = 4 * kTX + 4 * kTY;    // halo cells of one tile
    constexpr int kJobs = NF * kHalo;
    constexpr int kPer = (kJobs + kTX * kTY - 1) / (kTX * kTY);
    constexpr int kUW = kTX + 4, kUS = (kTY + 4) * kUW;
    constexpr int kDum = NF * kUS;              // then a scratch slot per thread for idle jobs
    __shared__ T lds[kDum + kTX * kTY];
    auto U = [&](int f, int y, int x) -> T& { return lds[f * kUS + y * kUW + x]; };
    auto wr = [n](int a) { return a < 0 ? a + n : (a >= n ? a - n : a); };
    const size_t col = base_ + (size_t)(i0 + tx) + (size_t)n * (j0 + ty);
    typedef const T __attribute__((address_space(1)))* gptr;   // global memory
    const gptr fsrc[NF] = {(gptr)w, (gptr)rk, (gptr)hbya, (gptr)(hbya + N), (gptr)p0};
    gptr hsrc[kPer];
    size_t hoff[kPer];
    int hdst[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int jb = tid + q * kTX * kTY;
        hsrc[q] = (gptr)w;
        hoff[q] = col;
        hdst[q] = kDum + tid;
        if (jb < kJobs) {
            const int f = jb / kHalo, h = jb - f * kHalo;
            hsrc[q] = fsrc[f];
            if (h < 4 * kTX) {                  // rows j0-2, j0-1, j0+8, j0+9
                const int row = h / kTX, x = h - row * kTX;
                const int yy = row < 2 ? row : kTY + row;
                hoff[q] = base_ + (size_t)(i0 + x) + (size_t)n * wr(j0 - 2 + yy);
                hdst[q] = f * kUS + yy * kUW + x + 2;
            } else {                            // columns i0-2, i0-1, i0+64, i0+65
                const int t = h - 4 * kTX, c4 = t / kTY, y = t - c4 * kTY;
                const int xx = c4 < 2 ? c4 : kTX + c4;
                hoff[q] = base_ + (size_t)wr(i0 - 2 + xx) + (size_t)n * (j0 + y);
                hdst[q] = f * kUS + (y + 2) * kUW + xx;
            }
        }
    }
    const T* hz = hbya + 2 * N;
    // queues (w, rho_k, HbyA_z at kk - 2 .. kk + 2; p0 at kk - 1 .. kk + 1) and
    // the own values of the first plane
    T wq[5], rq[5], zq[5], pq[3];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        wq[t] = w[col + nn * wr(k0 - 2 + t)];
        rq[t] = rk[col + nn * wr(k0 - 2 + t)];
        zq[t] = hz[col + nn * wr(k0 - 2 + t)];
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) pq[t] = p0[col + nn * wr(k0 - 1 + t)];
    T cx = hbya[col + nn * k0], cy = hbya[N + col + nn * k0], cn = rn[col + nn * k0], ch[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) ch[q] = hsrc[q][nn * (size_t)k0 + hoff[q]];
    T nw, nr, nz, np, nx, ny, nrn, nh[kPer];
    // queue heads at kq5 (w, rho_k, HbyA_z) and kq3 (p0), own and halo values at kv
    auto prefetch = [&](int kq5, int kq3, int kv) {
        const size_t p5 = nn * (size_t)wr(kq5), p3 = nn * (size_t)wr(kq3), pv = nn * (size_t)wr(kv);
        nw = w[col + p5];
        nr = rk[col + p5];
        nz = hz[col + p5];
        np = p0[col + p3];
        nx = hbya[col + pv];
        ny = hbya[N + col + pv];
        nrn = stream_ld(rn + col + pv);
#pragma unroll
        for (int q = 0; q < kPer; ++q) nh[q] = hsrc[q][pv + hoff[q]];
    };
    auto clampk = [](int a, int hi) { return a < hi ? a : hi; };
    // last planes the chunk needs: queue heads k1 + 1 (p0: k1), own values k1 - 1
    prefetch(clampk(k0 + 3, k1 + 1), clampk(k0 + 2, k1), clampk(k0 + 1, k1 - 1));
    double v[3] = {0.0, 0.0, 0.0};
    for (int kk = k0; kk < k1; ++kk) {
        const size_t P = col + nn * (size_t)kk;
        U(0, ty + 2, tx + 2) = wq[2];
        U(1, ty + 2, tx + 2) = rq[2];
        U(2, ty + 2, tx + 2) = cx;
        U(3, ty + 2, tx + 2) = cy;
        U(4, ty + 2, tx + 2) = pq[1];
#pragma unroll
        for (int q = 0; q < kPer; ++q) lds[hdst[q]] = ch[q];
        lds_barrier();
        T wv[13], rv[13], hl[3][5], pv[7];
        auto cross = [&](int f, T c, const T (&zq5)[5], T (&o)[13]) {
            o[0] = c;
            o[1] = U(f, ty + 2, tx);
            o[2] = U(f, ty + 2, tx + 1);
            o[3] = U(f, ty + 2, tx + 3);
            o[4] = U(f, ty + 2, tx + 4);
            o[5] = U(f, ty, tx + 2);
            o[6] = U(f, ty + 1, tx + 2);
            o[7] = U(f, ty + 3, tx + 2);
            o[8] = U(f, ty + 4, tx + 2);
            o[9] = zq5[0];
            o[10] = zq5[1];
            o[11] = zq5[3];
            o[12] = zq5[4];
        };
        cross(0, wq[2], wq, wv);
        cross(1, rq[2], rq, rv);
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            hl[0][t] = U(2, ty + 2, tx + t);
            hl[1][t] = U(3, ty + t, tx + 2);
            hl[2][t] = zq[t];
        }
        pv[0] = pq[1];
        pv[1] = U(4, ty + 2, tx + 1);
        pv[2] = U(4, ty + 2, tx + 3);
        pv[3] = U(4, ty + 1, tx + 2);
        pv[4] = U(4, ty + 3, tx + 2);
        pv[5] = pq[0];
        pv[6] = pq[2];
        lds_barrier();
        double b;
        T dgT, phf[3];
        corr_rhs_cell(wv, rv, hl, pv, cn, dt, rref, pref, gamma_psi(ph), ph.A, ph.inv_V, ph.inv_h,
                      ph.inv_h2, b, dgT, phf, ph.bdf2 ? (st + mem_)->bdf : nullptr,
                      ph.bdf2 ? ph.rm1[P] : 0.0);
        corr_rhs_store(P, N, b, dgT, phf, pref + (double)pv[0], phiH, rvec, diag, snap_b,
                       snap_diag, snap_p0, b64, v);
        // advance the queues with the values loaded one plane ago, then load
        // the queue heads at kk + 4 (p0: kk + 3) and the values of plane kk + 2
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            wq[t] = wq[t + 1];
            rq[t] = rq[t + 1];
            zq[t] = zq[t + 1];
        }
        wq[4] = nw;
        rq[4] = nr;
        zq[4] = nz;
        pq[0] = pq[1];
        pq[1] = pq[2];
        pq[2] = np;
        cx = nx;
        cy = ny;
        cn = nrn;
#pragma unroll
        for (int q = 0; q < kPer; ++q) ch[q] = nh[q];
        prefetch(clampk(kk + 4, k1 + 1), clampk(kk + 3, k1), clampk(kk + 2, k1 - 1));
    }
    block_partials<3, 0u>(v, part_u);
    if (MEMBER_FIRST()) {
        (st + mem_)->pcg.it_stop = kIterInf;
        (st + mem_)->pcg.converged = 0;
        (st + mem_)->pcg.iters = 0;
    }
}

// FP64 residual refinement (FP32 storage): accumulate the inner FP32
// correction, x64_new = x64 + d, evaluate r64 = b64 - M x64_new in FP64
// arithmetic (coefficients K = I4(w) and diag from their FP32 storage), and
// set up the next inner solve's right-hand side float(r64) with partial sums
// r.(r/diag), ||r64||^2, ||r64||^2.  FROM_ZERO: x64 is zero (the first round
// of a solve started from zero) and is not read.  The next inner solve
// starts from d = 0 without d being written.  x64_new is also written
// rounded to T (xf): after the last round that is the corrector's solution.
// store_x = 0 (FROM_ZERO only): x64_new = d exactly, so neither x64_new nor
// xf is written (d itself serves as the solution).
template <typename T>
__device__ inline void refine_cell(const T (&wv)[13], const double (&xv)[7], const T (&dv)[7],
                                   double bP, T dgP, double inv_h2, double& xP, double& r) {
    auto xn = [&](int t) { return xv[t] + (double)dv[t]; };
    xP = xn(0);
    double lap = 0.0, sumK = 0.0;
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
        const double kp = i4gr<double>(wv, dd, 0), km = i4gr<double>(wv, dd, -1);
        lap += kp * (xP - xn(2 + 2 * dd)) + km * (xP - xn(1 + 2 * dd));
        sumK += kp + km;
    }
    r = bP - (((double)dgP - sumK * inv_h2) * xP + lap * inv_h2);
}

template <typename T, bool FROM_ZERO>
__global__ void __launch_bounds__(kBlock) k_refine(Phys ph, DevState* st,
                                                   const double* __restrict__ x64,
                                                   const T* __restrict__ d, double* __restrict__ x64n,
                                                   T* __restrict__ xf,
                                                   const double* __restrict__ b64,
                                                   const T* __restrict__ w, const T* __restrict__ diag,
                                                   T* __restrict__ r32, double* part_u, int store_x) {
    MEMBER(ph)
    if ((st + mem_)->pcg.skip) return;   // converged already: the round does nothing
    const double inv_h2 = ph.inv_h2;
    double v[3] = {0.0, 0.0, 0.0};
    FOR_CELLS(ph)
    T wv[13], dv[7];
    double xv[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    gather13(w, c, wv);
    if (!FROM_ZERO) gather7(x64, c, xv);
    gather7(d, c, dv);
    const double bP = b64[P];
    const T dgP = diag[P];
    loads_issued();
    double xP, r;
    refine_cell(wv, xv, dv, bP, dgP, inv_h2, xP, r);
    if (!FROM_ZERO || store_x) {
        x64n[P] = xP;
        xf[P] = (T)xP;
    }
    const T rT = (T)r;
    r32[P] = rT;
    v[0] += (double)rT * ((double)rT / (double)dgP);
    v[1] += r * r;
    v[2] += r * r;
    END_CELLS
    block_partials<3, 0u>(v, part_u);
    if (MEMBER_FIRST()) {
        (st + mem_)->pcg.it_stop = kIterInf;
        (st + mem_)->pcg.converged = 0;
        (st + mem_)->pcg.iters = 0;
    }
}

// ---------------------------------------------------------------- CG
// Jacobi-PCG with one kernel per iteration.  Iteration k >= 1 forms, on the
// stencil, r_k = r_{k-1} - alpha_{k-1} q_{k-1}, z_k = r_k / diag (not stored)
// and the direction p_k = z_k + beta_k p_{k-1}; iteration 0 takes p_0 = z_0.
// Then q_k = M p_k with the face coefficients K = I4(w) formed on the fly; the
// kernel stores r_k, p_k and q_k and writes the partial sums from which the
// next iteration takes its scalars (cg_head).  The iterates are those of
// textbook PCG; r_k.z_k and ||r_k||^2 are expanded from sums of iteration
// k-1 instead of being summed over r_k, so one global reduction per
// iteration suffices.  x is updated every other iteration: an even k >= 2
// applies x += alpha_{k-2} p_{k-2} + alpha_{k-1} p_{k-1} (p_{k-1} is read
// anyway), an odd k leaves x alone, and the stop iteration adds what is
// still due (one term at an odd k, two at an even k), with the rounding of
// adding the terms one iteration at a time.  r and q alternate between two buffers (iteration k
// reads the k-1 values on the stencil while writing its own), p rotates
// through three (an even k also reads p_{k-2}).  With xzero (the solve
// started from x = 0, not written) the first write of x sets it: at k = 2,
// or on a stop at k = 1 (x = alpha_0 p_0) or k = 0 (x = 0).  XM: 0 for k = 0,
// 1 for odd k, 2 for even k >= 2.

// Partial-sum columns of iteration k (FP64 sums of products of the stored
// values): p.q, q.z, q.(q/diag), q.r, q.q, r.z, r.r over r_k, z_k = r_k / diag
// (the z of the direction), p_k, q_k.
enum CgCol { CG_PQ, CG_QZ, CG_QQD, CG_QR, CG_QQ, CG_RZ, CG_RR, CG_COLS };
static_assert(CG_COLS == kCgCols, "CG partial columns");

// The Jacobi preconditioner z = r / diag is applied as r * jinv(diag): in
// FP32 the hardware reciprocal (within 1 ulp; the preconditioner stays a
// positive diagonal), in FP64 the rounded 1 / diag.  Every block forms a
// cell's z with the same expression, so all see the same direction p.
__device__ inline float jinv(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ inline double jinv(double d) { return 1.0 / d; }

// y = q / diag as y = q * jinv(diag)
template <typename T>
__device__ inline void cg_accumulate(double (&v)[CG_COLS], T p, T q, T r, T z, T id) {
    const double qd = (double)q, rd = (double)r, zd = (double)z, yd = (double)(q * id);
    v[CG_PQ] += (double)p * qd;
    v[CG_QZ] += qd * zd;
    v[CG_QQD] += qd * yd;
    v[CG_QR] += qd * rd;
    v[CG_QQ] += qd * qd;
    v[CG_RZ] += rd * zd;
    v[CG_RR] += rd * rd;
}

// Scalars of iteration k, bitwise the same in every block of the member.
// k = 0: ||r_0||^2 (and ||b||^2 of a fresh solve) from the set-up kernel's
// partials (r.z, r.r, b.b).  k >= 1: from the partials of iteration k-1,
// alpha_{k-1} = r.z / p.q and, with r_k = r_{k-1} - alpha_{k-1} q_{k-1},
//   r_k.z_k   = r.z - 2 alpha q.z + alpha^2 q.(q/diag),
//   ||r_k||^2 = r.r - 2 alpha q.r + alpha^2 q.q,
// each one step from sums over the stored r_{k-1} (no drift accumulates over
// iterations); beta_k = r_k.z_k / r_{k-1}.z_{k-1}.  Stop at
// ||r_k||^2 <= tol^2 ||b||^2 or k = maxit; `recorder` (one thread of the
// member) writes the iteration to the member state.  With pcg.skip (a
// refinement round after the refinement has converged) the solve stops at
// k = 0 without touching x.
struct CgHead {
    double alpha, beta, rr;
    bool stop, skip;
};
__device__ inline CgHead cg_head(const Phys& ph, PcgState& g, bool recorder, int mem, int k,
                                 const double* part_in, unsigned nb_in, int fresh, int maxit) {
    CgHead h{0.0, 0.0, 0.0, false, false};
    if (g.skip) {
        h.stop = h.skip = true;
        if (recorder) {
            g.iters = k;
            g.it_stop = k;
            g.converged = 1;
        }
        return h;
    }
    // reference ||b||^2: from this system's partials on the first iteration of
    // a fresh solve, else the stored one (later refinement rounds measure
    // against the original right-hand side)
    const bool newb = fresh && k == 0;
    double bb;
    if (k == 0) {
        double t[3];
        reduce_member<3, 0u, true>(part_in, nb_in, ph.batch, mem, t);
        h.rr = t[1];
        bb = newb ? t[2] : g.bb;
    } else {
        double t[CG_COLS];
        reduce_member<CG_COLS, 0u, true>(part_in, nb_in, ph.batch, mem, t);
        const double a = t[CG_RZ] / t[CG_PQ];
        const double rz = t[CG_RZ] - 2.0 * a * t[CG_QZ] + a * a * t[CG_QQD];
        const double rr = t[CG_RR] - 2.0 * a * t[CG_QR] + a * a * t[CG_QQ];
        h.alpha = a;
        h.beta = rz / t[CG_RZ];
        h.rr = rr < 0.0 ? 0.0 : rr;   // cancellation at the rounding floor; NaN stays NaN
        bb = g.bb;
    }
    const bool conv = h.rr <= g.tol2 * bb;
    h.stop = conv || k >= maxit;
    if (recorder) {
        g.rr = h.rr;
        g.iters = k;
        if (k >= 1) g.alphah[k & 1] = h.alpha;
        if (newb) g.bb = bb;
        if (h.stop) {
            g.it_stop = k;
            g.converged = conv ? 1 : 0;
        }
    }
    return h;
}

// The x update of iteration k (see above): alpha = alpha_{k-1}, alpha2 =
// alpha_{k-2}; set: x not written yet (xzero and k <= 2).  V: T or a vector of T.
template <typename T>
struct CgX {
    T alpha, alpha2;
    bool set;
    template <typename V>
    __device__ V one(V xo, V p1) const { return set ? alpha * p1 : xo + alpha * p1; }
    template <typename V>
    __device__ V two(V xo, V p2, V p1) const {
        const V t = set ? alpha2 * p2 : xo + alpha2 * p2;
        return t + alpha * p1;
    }
};
template <typename T, int XM>
__device__ inline CgX<T> cg_x(const PcgState& g, int k, double alpha, int xzero) {
    return {(T)alpha, XM == 2 ? (T)g.alphah[(k - 1) & 1] : T(0), xzero != 0 && k <= 2};
}

// Gathered form (any n).
template <typename T, int XM>
__global__ void __launch_bounds__(kBlock) k_pcg_spmv(
    Phys ph, DevState* st, int k, const T* __restrict__ rin, T* __restrict__ rout,
    const T* __restrict__ diag, const T* __restrict__ w, const T* __restrict__ pold,
    const T* __restrict__ pold2, T* __restrict__ pnew, const T* __restrict__ qold,
    T* __restrict__ q, T* __restrict__ x, const double* part_in, unsigned nb_in, double* part_out,
    int fresh, int maxit, int xzero) {
    constexpr bool UPD = XM > 0, XE = XM == 2;
    MEMBER(ph)
    // it_stop == k is this launch's own decision, written by the member's
    // first block: the other blocks must still take the stop path below
    if (k > (st + mem_)->pcg.it_stop) return;
    const CgHead h = cg_head(ph, (st + mem_)->pcg, MEMBER_FIRST(), mem_, k, part_in, nb_in, fresh,
                             maxit);
    const T alpha = (T)h.alpha, beta = (T)h.beta;
    const CgX<T> xu = cg_x<T, XM>((st + mem_)->pcg, k, h.alpha, xzero);
    if (h.stop) {
        if ((UPD || xzero) && !h.skip) {
            FOR_CELLS(ph)
            x[P] = XE ? xu.two(x[P], pold2[P], pold[P]) : UPD ? xu.one(x[P], pold[P]) : T(0);
            END_CELLS
        }
        return;
    }
    const T inv_h2 = (T)ph.inv_h2;
    double v[CG_COLS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    FOR_CELLS(ph)
    auto res = [&](size_t Q) -> T { return UPD ? rin[Q] - alpha * qold[Q] : rin[Q]; };
    auto dir = [&](size_t Q) -> T {
        const T z = res(Q) * jinv(diag[Q]);
        return UPD ? z + beta * pold[Q] : z;
    };
    const T rP = res(P), dP = diag[P], iP = jinv(dP), zP = rP * iP;
    const T pP = UPD ? zP + beta * pold[P] : zP;   // as dir(P)
    // difference form psi/dt p_P + sum K (p_P - p_nb) / h^2 (no cancellation
    // between the diagonal and the neighbour sum for smooth p)
    T lap = T(0), sumK = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T kp = i4(w, c, d, 0), km = i4(w, c, d, -1);
        lap += kp * (pP - dir(c.sh(d, 1))) + km * (pP - dir(c.sh(d, -1)));
        sumK += kp + km;
    }
    const T qP = (dP - sumK * inv_h2) * pP + lap * inv_h2;
    if (UPD) rout[P] = rP;
    if (XE) x[P] = xu.two(x[P], pold2[P], pold[P]);
    pnew[P] = pP;
    q[P] = qP;
    cg_accumulate(v, pP, qP, rP, zP, iP);
    END_CELLS
    block_partials<CG_COLS, 0u>(v, part_out);
}

// Tiled form: a block of TX x NTY threads owns a TX x (NTY RPT) column tile
// (64 x 8 for n a multiple of 64, 16 x 16 for the other multiples of 16) and
// marches along z.  Each of r, q, p_old, diag and w is read once per cell
// from HBM: the x-y neighbours of the current plane come from LDS tiles (halo
// 2 for w; halo 1 for the direction p, formed from r, q, p_old and diag at
// the halo cells), the z neighbours from per-thread register queues.
template <typename T, int RPT, int XM, int TX, int NTY>
__global__ void __launch_bounds__(TX * NTY) k_pcg_spmv_tiled(
    Phys ph, DevState* st, int k, const T* __restrict__ rin, T* __restrict__ rout,
    const T* __restrict__ diag, const T* __restrict__ w, const T* __restrict__ pold,
    const T* __restrict__ pold2, T* __restrict__ pnew, const T* __restrict__ qold,
    T* __restrict__ q, T* __restrict__ x, const double* part_in, unsigned nb_in, double* part_out,
    int fresh, int maxit, int xzero) {
    constexpr bool UPD = XM > 0, XE = XM == 2;
    MEMBER(ph)
    if (k > (st + mem_)->pcg.it_stop) return;   // see k_pcg_spmv
    const CgHead h = cg_head(ph, (st + mem_)->pcg, MEMBER_FIRST(), mem_, k, part_in, nb_in, fresh,
                             maxit);
    const T alpha = (T)h.alpha, beta = (T)h.beta;
    const T inv_h2 = (T)ph.inv_h2;
    const int n = ph.n, cz = ph.cz;
    constexpr int TY = NTY * RPT;               // tile rows; thread row ty owns rows ty + e NTY
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + TX * ty;
    const int i0 = bp_.x * TX, j0 = bp_.y * TY;
    const int k0 = bz_ * cz;
    const int k1 = k0 + cz < n ? k0 + cz : n;
    const size_t nn = (size_t)n * n;
    const CgX<T> xu = cg_x<T, XM>((st + mem_)->pcg, k, h.alpha, xzero);
    if (h.stop) {
        if ((UPD || xzero) && !h.skip) {
#pragma unroll
            for (int e = 0; e < RPT; ++e) {
                const size_t c0 = base_ + (size_t)(i0 + tx) + (size_t)n * (j0 + ty + e * NTY);
                for (int kk = k0; kk < k1; ++kk) {
                    const size_t Q = c0 + nn * (size_t)kk;
                    x[Q] = XE    ? xu.two(x[Q], pold2[Q], pold[Q])
                           : UPD ? xu.one(x[Q], pold[Q])
                                 : T(0);
                }
            }
        }
        return;
    }
    __shared__ T ws[TY + 4][TX + 4];
    __shared__ T ps[TY + 2][TX + 2];
    auto wr = [n](int a) { return a < 0 ? a + n : (a >= n ? a - n : a); };
    // r_k and p_k of a cell from its r_{k-1}, q_{k-1}, diag, p_{k-1}
    auto resf = [&](T ro, T qo) -> T { return UPD ? ro - alpha * qo : ro; };
    auto dirf = [&](T z, T po) -> T { return UPD ? z + beta * po : z; };
    size_t col[RPT];
    T wq0[RPT], wq1[RPT], wq2[RPT], wq3[RPT], wq4[RPT], pm[RPT], pc[RPT], rc[RPT], zc[RPT], dc[RPT];
    T ic[RPT];   // jinv(diag) of the current plane
    T rn1[RPT], qn1[RPT], dn1[RPT], on1[RPT];
    // p_old of the current plane; XE: x and p_{k-2} of the current plane and
    // one plane ahead
    T oc[RPT], xc[RPT], xn1[RPT], o2c[RPT], o2n1[RPT];
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
        col[e] = base_ + (size_t)(i0 + tx) + (size_t)n * (j0 + ty + e * NTY);
        wq0[e] = w[col[e] + nn * wr(k0 - 2)];
        wq1[e] = w[col[e] + nn * wr(k0 - 1)];
        wq2[e] = w[col[e] + nn * k0];
        wq3[e] = w[col[e] + nn * wr(k0 + 1)];
        const size_t Qm = col[e] + nn * wr(k0 - 1), Q0 = col[e] + nn * k0;
        pm[e] = dirf(resf(rin[Qm], UPD ? qold[Qm] : T(0)) * jinv(diag[Qm]), UPD ? pold[Qm] : T(0));
        rc[e] = resf(rin[Q0], UPD ? qold[Q0] : T(0));
        dc[e] = diag[Q0];
        ic[e] = jinv(dc[e]);
        zc[e] = rc[e] * ic[e];
        oc[e] = UPD ? pold[Q0] : T(0);
        pc[e] = dirf(zc[e], oc[e]);
        if (XE) {
            xc[e] = stream_ld(x + Q0);
            o2c[e] = stream_ld(pold2 + Q0);
        }
    }
    // this thread's halo cell, if any (same x-y position on every plane):
    // w rows j0-2, j0-1, j0+TY, j0+TY+1; w columns i0-2, i0-1, i0+TX, i0+TX+1;
    // p rows j0-1, j0+TY; p columns i0-1, i0+TX
    constexpr int nWR = 4 * TX, nWC = 4 * TY, nPR = 2 * TX, nPC = 2 * TY;
    static_assert(nWR + nWC + nPR + nPC <= TX * NTY, "one halo cell per thread");
    int hkind = 0, hy = 0, hx = 0;
    size_t hoff = 0;
    if (tid < nWR) {
        const int row = tid / TX, xx = tid - row * TX;
        hy = row < 2 ? row : TY + row;
        hx = xx + 2;
        hoff = base_ + (size_t)(i0 + xx) + (size_t)n * wr(j0 - 2 + hy);
        hkind = 1;
    } else if (tid < nWR + nWC) {
        const int t2 = tid - nWR, c4 = t2 / TY, y = t2 - c4 * TY;
        hx = c4 < 2 ? c4 : TX + c4;
        hy = y + 2;
        hoff = base_ + (size_t)wr(i0 - 2 + hx) + (size_t)n * (j0 + y);
        hkind = 1;
    } else if (tid < nWR + nWC + nPR) {
        const int t3 = tid - nWR - nWC, row = t3 / TX, xx = t3 - row * TX;
        hy = row == 0 ? 0 : TY + 1;
        hx = xx + 1;
        hoff = base_ + (size_t)(i0 + xx) + (size_t)n * wr(j0 - 1 + hy);
        hkind = 2;
    } else if (tid < nWR + nWC + nPR + nPC) {
        const int t4 = tid - nWR - nWC - nPR, c2 = t4 / TY, y = t4 - c2 * TY;
        hx = c2 == 0 ? 0 : TX + 1;
        hy = y + 1;
        hoff = base_ + (size_t)wr(i0 - 1 + hx) + (size_t)n * (j0 + y);
        hkind = 2;
    }
    // Software pipeline: the loads of plane kk + 1 (w at kk + 3; r, q, diag,
    // p_old at kk + 2; this thread's halo cell of plane kk + 1) are issued
    // before the LDS stores and barrier of plane kk, so their latency overlaps
    // its work.  Every load is unconditional and in bounds (threads without a
    // halo cell read their own), so no branch forces the loads to drain early.
    // the p halo reads r, diag, q, p_old; a w-halo thread points its other
    // three loads at its w cell, a thread without a halo cell all four at its
    // own r cell (cache hits, no extra HBM traffic)
    const T* hsrc = hkind == 1 ? w : rin;
    const T* hdsrc = hkind == 2 ? diag : hsrc;
    const T* hqsrc = hkind == 2 ? qold : hsrc;
    const T* hosrc = hkind == 2 ? pold : hsrc;
    const size_t hq = hkind == 0 ? col[0] : hoff;       // plane offset added per plane
#pragma unroll
    for (int e = 0; e < RPT; ++e) {
        const size_t Q1 = col[e] + nn * wr(k0 + 1);
        wq4[e] = w[col[e] + nn * wr(k0 + 2)];
        rn1[e] = rin[Q1];
        dn1[e] = diag[Q1];
        if (UPD) {
            qn1[e] = qold[Q1];
            on1[e] = pold[Q1];
        }
    }
    T ha = hsrc[nn * (size_t)k0 + hq], hd = hdsrc[nn * (size_t)k0 + hq];
    T hqv = UPD ? hqsrc[nn * (size_t)k0 + hq] : T(0), ho = UPD ? hosrc[nn * (size_t)k0 + hq] : T(0);
    double acc[CG_COLS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int kk = k0; kk < k1; ++kk) {
        const size_t pl = nn * (size_t)kk;
        T wq4c[RPT], dn[RPT], pp[RPT], on[RPT], rp[RPT], zp[RPT], ip[RPT];
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            wq4c[e] = wq4[e];
            dn[e] = dn1[e];
            on[e] = UPD ? on1[e] : T(0);
            rp[e] = resf(rn1[e], UPD ? qn1[e] : T(0));
            ip[e] = jinv(dn1[e]);
            zp[e] = rp[e] * ip[e];
            pp[e] = dirf(zp[e], on[e]);
        }
        T hpc = T(0);
        if (hkind == 2) hpc = dirf(resf(ha, hqv) * jinv(hd), ho);
        const T hwc = ha;
        {
            const size_t Hf = nn * (size_t)wr(kk + 1) + hq;
#pragma unroll
            for (int e = 0; e < RPT; ++e) {
                const size_t Qf = col[e] + nn * wr(kk + 2);
                wq4[e] = w[col[e] + nn * wr(kk + 3)];
                rn1[e] = rin[Qf];
                dn1[e] = diag[Qf];
                if (UPD) {
                    qn1[e] = qold[Qf];
                    on1[e] = pold[Qf];
                }
                if (XE) {
                    const size_t Qx = col[e] + nn * (size_t)(kk + 1 < k1 ? kk + 1 : kk);
                    xn1[e] = stream_ld(x + Qx);
                    o2n1[e] = stream_ld(pold2 + Qx);
                }
            }
            ha = hsrc[Hf];
            hd = hdsrc[Hf];
            if (UPD) {
                hqv = hqsrc[Hf];
                ho = hosrc[Hf];
            }
        }
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            ws[ty + e * NTY + 2][tx + 2] = wq2[e];
            ps[ty + e * NTY + 1][tx + 1] = pc[e];
        }
        if (hkind == 1) ws[hy][hx] = hwc;
        else if (hkind == 2) ps[hy][hx] = hpc;
        lds_barrier();
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            const int y = ty + e * NTY;
            const T kxp = (T(9) * (ws[y + 2][tx + 2] + ws[y + 2][tx + 3]) -
                           (ws[y + 2][tx + 1] + ws[y + 2][tx + 4])) * T(0.0625);
            const T kxm = (T(9) * (ws[y + 2][tx + 1] + ws[y + 2][tx + 2]) -
                           (ws[y + 2][tx] + ws[y + 2][tx + 3])) * T(0.0625);
            const T kyp = (T(9) * (ws[y + 2][tx + 2] + ws[y + 3][tx + 2]) -
                           (ws[y + 1][tx + 2] + ws[y + 4][tx + 2])) * T(0.0625);
            const T kym = (T(9) * (ws[y + 1][tx + 2] + ws[y + 2][tx + 2]) -
                           (ws[y][tx + 2] + ws[y + 3][tx + 2])) * T(0.0625);
            const T kzp = (T(9) * (wq2[e] + wq3[e]) - (wq1[e] + wq4c[e])) * T(0.0625);
            const T kzm = (T(9) * (wq1[e] + wq2[e]) - (wq0[e] + wq3[e])) * T(0.0625);
            const T c0 = pc[e];
            const T lap = kxp * (c0 - ps[y + 1][tx + 2]) + kxm * (c0 - ps[y + 1][tx]) +
                          kyp * (c0 - ps[y + 2][tx + 1]) + kym * (c0 - ps[y][tx + 1]) +
                          kzp * (c0 - pp[e]) + kzm * (c0 - pm[e]);
            const T sumK = kxp + kxm + kyp + kym + kzp + kzm;
            const T qv = (dc[e] - sumK * inv_h2) * c0 + lap * inv_h2;
            stream_st(q + (col[e] + pl), qv);
            stream_st(pnew + (col[e] + pl), c0);
            if (UPD) stream_st(rout + (col[e] + pl), rc[e]);
            if (XE) stream_st(x + (col[e] + pl), xu.two(xc[e], o2c[e], oc[e]));
            cg_accumulate(acc, c0, qv, rc[e], zc[e], ic[e]);
        }
        lds_barrier();
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            wq0[e] = wq1[e];
            wq1[e] = wq2[e];
            wq2[e] = wq3[e];
            wq3[e] = wq4c[e];
            pm[e] = pc[e];
            pc[e] = pp[e];
            rc[e] = rp[e];
            zc[e] = zp[e];
            ic[e] = ip[e];
            dc[e] = dn[e];
            if (UPD) oc[e] = on[e];
            if (XE) {
                xc[e] = xn1[e];
                o2c[e] = o2n1[e];
            }
        }
    }
    block_partials<CG_COLS, 0u, true>(acc, part_out);
}

// Row form for n = 64 V H: a block of kRowWaves wavefronts owns kRowWaves / H
// consecutive full x-rows, H wavefronts per row (wavefront v: row j0 + v / H,
// lanes 64 (v % H) .. 64 (v % H) + 63 of the row; lane l of the row: cells
// x = V l .. V l + V - 1, one vector load per field) and marches along z over
// cz planes.  A whole periodic row lives in the block, so no x halo is read:
// with H = 1 the x neighbours come from the lane's own cells and one lane
// rotation, with H = 2 (FP64: 2 cells per lane, whose registers fit where 4
// would not) from the row's LDS copy that the y neighbours use anyway.  y
// neighbours come from LDS rows (halo 2 for w, 1 for p): with H = 1 loaded by
// wavefronts 0-5 (one halo row each), with H = 2 the p halo by wavefronts 0-3
// (one half row each) and the w halo by 4-7 (both halves of one row each).  z
// neighbours come from per-lane register queues, the lower z face coefficient
// carried over from the plane below.  Prefetches past the chunk's last needed
// plane are clamped to planes already read.  NT: r, q and p_old of the main
// rows load non-temporally (see Launch::nt).
template <typename T, int V, int H, int XM, bool NT>
__global__ void __launch_bounds__(64 * kRowWaves) k_pcg_spmv_rows(
    Phys ph, DevState* st, int k, const T* __restrict__ rin, T* __restrict__ rout,
    const T* __restrict__ diag, const T* __restrict__ w, const T* __restrict__ pold,
    const T* __restrict__ pold2, T* __restrict__ pnew, const T* __restrict__ qold,
    T* __restrict__ q, T* __restrict__ x, const double* part_in, unsigned nb_in, double* part_out,
    int fresh, int maxit, int xzero) {
    constexpr bool UPD = XM > 0, XE = XM == 2;
    using VT = T __attribute__((ext_vector_type(V)));
    static_assert(H == 1 ? kRowWaves >= 6 : H == 2 && kRowWaves == 8,
                  "y halo loads: wavefronts 0-5 (one per row) or 0-7 (two per row)");
    MEMBER(ph)
    const int n = ph.n, cz = ph.cz;   // n == 64 V
    constexpr int TY = kRowWaves / H, RW = 64 * H;   // rows per block, lanes per row
    const int lane = threadIdx.x, wv = threadIdx.y;
    const int r = wv / H, gl = (wv % H) * 64 + lane;   // row in the block, lane in the row
    const int j0 = bp_.y * TY;
    const int k0 = bz_ * cz;
    const int k1 = k0 + cz < n ? k0 + cz : n;
    const size_t nn = (size_t)n * n;
    // rows of the current plane, two sets alternating with the plane's parity:
    // a set is written again only two planes later, after every wavefront has
    // passed the barrier of the plane in between (so one barrier per plane)
    __shared__ VT wlb[2][TY + 4][RW];   // w of rows j0 - 2 .. j0 + TY + 1
    __shared__ VT plb[2][TY + 2][RW];   // p of rows j0 - 1 .. j0 + TY
    auto wr = [n](int a) { return a < 0 ? a + n : (a >= n ? a - n : a); };
    auto ld = [](const T* f, size_t o) { return *reinterpret_cast<const VT*>(f + o); };
    // outputs and x stream past the caches (stream_st), keeping L2 for the
    // halo rows and planes still to be read
    auto st_v = [](T* f, size_t o, VT v) { stream_st(reinterpret_cast<VT*>(f + o), v); };
    auto ld_x = [](const T* f, size_t o) { return stream_ld(reinterpret_cast<const VT*>(f + o)); };
    const size_t col = base_ + (size_t)n * (j0 + r) + (size_t)V * gl;
    auto ldu = [&](const T* f, size_t o) { return UPD ? ld(f, o) : VT(T(0)); };
    // the main rows' r, q, p_old of the planes ahead (read once per iteration)
    auto ldm = [&](const T* f, size_t o) { return NT ? ld_x(f, o) : ld(f, o); };
    auto ldmu = [&](const T* f, size_t o) { return UPD ? ldm(f, o) : VT(T(0)); };
    // this wavefront's y halo loads (h1..h4 from hsrc..hqsrc at hc1..hc4).
    // H = 1: w rows j0-2, j0-1, j0+TY, j0+TY+1 (waves 0-3), p rows j0-1,
    // j0+TY (waves 4-5, from r, q, diag and p_old); waves 6.. read their own
    // w row so that every load is unconditional; waves other than 4-5 point all
    // four loads at the same w row (cache hits).  H = 2: p halves of rows j0-1
    // and j0+TY (waves 0-3), both w halves (h1, h2) of rows j0-2, j0-1,
    // j0+TY, j0+TY+1 (waves 4-7; h3, h4 repeat h1).
    const bool phalo = H == 1 ? wv == 4 || wv == 5 : wv < 4;
    int hrow, hhalf = lane;
    if (H == 1) {
        hrow = wv < 2 ? j0 - 2 + wv : wv < 4 ? j0 + TY - 2 + wv : wv == 4 ? j0 - 1 : wv == 5 ? j0 + TY : j0 + wv;
    } else if (phalo) {
        hrow = wv < 2 ? j0 - 1 : j0 + TY;
        hhalf = (wv % 2) * 64 + lane;
    } else {
        hrow = wv < 6 ? j0 - 6 + wv : j0 + TY - 6 + wv;
    }
    const size_t hc1 = base_ + (size_t)n * wr(hrow) + (size_t)V * hhalf;
    const size_t hc2 = H == 2 && !phalo ? hc1 + (size_t)V * 64 : hc1;
    const size_t hc3 = hc1, hc4 = hc1;
    const T* hsrc = phalo ? rin : w;
    const T* hdsrc = phalo ? diag : w;
    const T* hosrc = phalo ? pold : w;
    const T* hqsrc = phalo ? qold : w;
    auto plane = [&](int kk) { return nn * (size_t)wr(kk); };
    // The first planes' loads go out before the launch's serial head (the
    // stop test, the reduction of the previous iteration's partials, alpha
    // and beta), which they do not depend on, so that their latency overlaps
    // it; the head's barriers order LDS only and leave them in flight.
    const VT wmm = ld(w, col + plane(k0 - 2));
    VT wm1 = ld(w, col + plane(k0 - 1)), w0 = ld(w, col + plane(k0)), wp1 = ld(w, col + plane(k0 + 1));
    VT wp2n = ld(w, col + plane(k0 + 2));
    const size_t Qm = col + plane(k0 - 1), Q0 = col + plane(k0), Q1 = col + plane(k0 + 1);
    const VT rm_in = ld(rin, Qm), qm_in = ldu(qold, Qm), dm_in = ld(diag, Qm), om_in = ldu(pold, Qm);
    VT oc = ldu(pold, Q0);   // p_old of the current plane (x update)
    VT dc = ld(diag, Q0);
    const VT r0_in = ld(rin, Q0), q0_in = ldu(qold, Q0);
    // XE: x and p_{k-2} of the current plane and one plane ahead
    VT xc = XE ? ld_x(x, Q0) : VT(T(0)), xn1 = xc;
    VT o2c = XE ? ld_x(pold2, Q0) : VT(T(0)), o2n1 = o2c;
    VT rnx = ld(rin, Q1), qnx = ldu(qold, Q1), dnx = ld(diag, Q1), onx = ldu(pold, Q1);
    VT h1 = ld(hsrc, hc1 + plane(k0)), h2 = ld(hdsrc, hc2 + plane(k0));
    VT h3 = ldu(hosrc, hc3 + plane(k0)), h4 = ldu(hqsrc, hc4 + plane(k0));
    if (k > (st + mem_)->pcg.it_stop) return;   // see k_pcg_spmv
    const CgHead h = cg_head(ph, (st + mem_)->pcg, MEMBER_FIRST(), mem_, k, part_in, nb_in, fresh,
                             maxit);
    const T alpha = (T)h.alpha, beta = (T)h.beta;
    const T inv_h2 = (T)ph.inv_h2;
    const CgX<T> xu = cg_x<T, XM>((st + mem_)->pcg, k, h.alpha, xzero);
    if (h.stop) {
        if ((UPD || xzero) && !h.skip) {
            for (int kk = k0; kk < k1; ++kk) {
                const size_t Q = col + nn * (size_t)kk;
                st_v(x, Q, XE    ? xu.two(ld(x, Q), ld(pold2, Q), ld(pold, Q))
                           : UPD ? xu.one(ld(x, Q), ld(pold, Q))
                                 : VT(T(0)));
            }
        }
        return;
    }
    // r_k and p_k of a cell from its r_{k-1}, q_{k-1}, diag, p_{k-1}
    auto resf = [&](VT ro, VT qo) -> VT { return UPD ? ro - alpha * qo : ro; };
    auto dirf = [&](VT z, VT po) -> VT { return UPD ? z + beta * po : z; };
    auto jv = [](VT d) {
        VT o;
#pragma unroll
        for (int i = 0; i < V; ++i) o[i] = jinv(d[i]);
        return o;
    };
    VT pm = dirf(resf(rm_in, qm_in) * jv(dm_in), om_in);
    VT rc = resf(r0_in, q0_in);
    VT ic = jv(dc), zc = rc * ic;
    VT pc = dirf(zc, oc);
    VT kzm = (T(9) * (wm1 + w0) - (wmm + wp1)) * T(0.0625);
    auto from_left = [&](T v) { return __shfl(v, (lane + 63) & 63, 64); };
    auto from_right = [&](T v) { return __shfl(v, (lane + 1) & 63, 64); };
    double acc[CG_COLS] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int kk = k0; kk < k1; ++kk) {
        const VT wp2 = wp2n;
        const VT rp = resf(rnx, qnx);
        const VT ip = jv(dnx), zp = rp * ip;
        const VT pp = dirf(zp, onx);
        const VT dn = dnx, on = onx;
        const VT hw = h1, hw2 = h2;
        VT hp = VT(T(0));
        if (phalo) hp = dirf(resf(h1, h4) * jv(h2), h3);
        {
            const int kw = kk + 3 < k1 + 1 ? kk + 3 : k1 + 1;   // last w plane needed: k1 + 1
            const int kp = kk + 2 < k1 ? kk + 2 : k1;           // last p plane needed: k1
            const int kh = kk + 1 < k1 - 1 ? kk + 1 : k1 - 1;   // last halo plane: k1 - 1
            const size_t Qp = col + plane(kp), Qh = plane(kh);
            wp2n = ld(w, col + plane(kw));
            rnx = ldm(rin, Qp);
            qnx = ldmu(qold, Qp);
            dnx = ld(diag, Qp);
            onx = ldmu(pold, Qp);
            h1 = ld(hsrc, hc1 + Qh);
            h2 = ld(hdsrc, hc2 + Qh);
            h3 = ldu(hosrc, hc3 + Qh);
            h4 = ldu(hqsrc, hc4 + Qh);
            if (XE) {
                const size_t Qx = col + nn * (size_t)(kk + 1 < k1 ? kk + 1 : kk);
                xn1 = ld_x(x, Qx);
                o2n1 = ld_x(pold2, Qx);
            }
        }
        VT(&wl)[TY + 4][RW] = wlb[kk & 1];
        VT(&pl)[TY + 2][RW] = plb[kk & 1];
        wl[r + 2][gl] = w0;
        pl[r + 1][gl] = pc;
        if (H == 1) {
            if (wv < 2) wl[wv][lane] = hw;
            else if (wv < 4) wl[TY + wv][lane] = hw;
            else if (wv == 4) pl[0][lane] = hp;
            else if (wv == 5) pl[TY + 1][lane] = hp;
        } else if (phalo) {
            pl[wv < 2 ? 0 : TY + 1][hhalf] = hp;
        } else {
            const int slot = wv < 6 ? wv - 4 : TY + wv - 4;
            wl[slot][lane] = hw;
            wl[slot][64 + lane] = hw2;
        }
        lds_barrier();
        const VT ym2 = wl[r][gl], ym1 = wl[r + 1][gl], yp1 = wl[r + 3][gl], yp2 = wl[r + 4][gl];
        const VT pym = pl[r][gl], pyp = pl[r + 2][gl];
        // H = 2: the x neighbours' cells (periodic row of RW lanes)
        VT wL = VT(T(0)), wR = VT(T(0)), pL = VT(T(0)), pR = VT(T(0));
        if (H == 2) {
            const int gm = (gl + RW - 1) % RW, gp = (gl + 1) % RW;
            wL = wl[r + 2][gm];
            wR = wl[r + 2][gp];
            pL = pl[r + 1][gm];
            pR = pl[r + 1][gp];
        }
        // w at x - 2 .. x + V + 1 and p at x - 1 .. x + V of this lane's cells
        T wx[V + 4], px[V + 2];
        if (H == 1) {
            wx[0] = from_left(w0[V - 2]);
            wx[1] = from_left(w0[V - 1]);
            wx[V + 2] = from_right(w0[0]);
            wx[V + 3] = from_right(w0[1]);
            px[0] = from_left(pc[V - 1]);
            px[V + 1] = from_right(pc[0]);
        } else {
            wx[0] = wL[V - 2];
            wx[1] = wL[V - 1];
            wx[V + 2] = wR[0];
            wx[V + 3] = wR[1];
            px[0] = pL[V - 1];
            px[V + 1] = pR[0];
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            wx[i + 2] = w0[i];
            px[i + 1] = pc[i];
        }
        T kf[V + 1];   // x face coefficients, face f between cells f - 1 and f
#pragma unroll
        for (int f = 0; f <= V; ++f)
            kf[f] = (T(9) * (wx[f + 1] + wx[f + 2]) - (wx[f] + wx[f + 3])) * T(0.0625);
        const VT kzp = (T(9) * (w0 + wp1) - (wm1 + wp2)) * T(0.0625);
        VT qo;
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const T kxp = kf[i + 1], kxm = kf[i];
            const T kyp = (T(9) * (w0[i] + yp1[i]) - (ym1[i] + yp2[i])) * T(0.0625);
            const T kym = (T(9) * (ym1[i] + w0[i]) - (ym2[i] + yp1[i])) * T(0.0625);
            const T c0 = pc[i];
            const T lap = kxp * (c0 - px[i + 2]) + kxm * (c0 - px[i]) + kyp * (c0 - pyp[i]) +
                          kym * (c0 - pym[i]) + kzp[i] * (c0 - pp[i]) + kzm[i] * (c0 - pm[i]);
            const T sumK = kxp + kxm + kyp + kym + kzp[i] + kzm[i];
            const T qv = (dc[i] - sumK * inv_h2) * c0 + lap * inv_h2;
            qo[i] = qv;
            cg_accumulate(acc, c0, qv, rc[i], zc[i], ic[i]);
        }
        const size_t pl0 = nn * (size_t)kk;
        st_v(q, col + pl0, qo);
        st_v(pnew, col + pl0, pc);
        if (UPD) st_v(rout, col + pl0, rc);
        if (XE) {
            st_v(x, col + pl0, xu.two(xc, o2c, oc));
            xc = xn1;
            o2c = o2n1;
        }
        if (UPD) oc = on;
        wm1 = w0;
        w0 = wp1;
        wp1 = wp2;
        kzm = kzp;
        pm = pc;
        pc = pp;
        rc = rp;
        zc = zp;
        ic = ip;
        dc = dn;
    }
    block_partials<CG_COLS, 0u, true>(acc, part_out);
}

// ---- CG preconditioned by a Chebyshev polynomial (stand-alone solve) ----
// A non-learned rival of the learned guess: z = p(D^-1 M) D^-1 r with the
// degree-1 p whose residual polynomial 1 - lambda p(lambda) is the degree-2
// Chebyshev polynomial of [a, 2 - a], a = min psi/dt / diag (the Gershgorin
// interval of D^-1 M): p(lambda) = c0 + c1 lambda,
//   mu = (b + a)/(b - a), T2 = 2 mu^2 - 1, c0 = 8 mu / ((b - a) T2),
//   c1 = -8 / ((b - a)^2 T2),  b = 2 - a.
// Two launches per iteration k: k_cheb_res forms r_k = r_{k-1} - alpha q_{k-1}
// and x_k, then z_k (a stencil over t = r_k / diag); k_cheb_dir tests r_k,
// forms p_k = z_k + beta p_{k-1} and q_k = M p_k.  r and p alternate between
// two buffers (the stencils read the previous iterate at the neighbours);
// partial sums alternate between two column sets by k & 1.  M v is taken in
// its diagonal form diag v - (1/h^2) sum_f K_f v_nb.

// Largest -psi/dt / diag over the cells (the interval's lower end a).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cheb_theta(Phys ph, const T* __restrict__ psidt,
                                                       const T* __restrict__ diag, double* part) {
    MEMBER(ph)
    double v[1] = {-__builtin_inf()};
    FOR_CELLS(ph)
    const double t = -(double)psidt[P] / (double)diag[P];
    v[0] = t > v[0] ? t : v[0];
    END_CELLS
    block_partials<1, 1u>(v, part);
}

template <typename T>
__device__ inline T m_diag_form(const T* __restrict__ diag, const T* __restrict__ w, const CellIdx& c,
                                T inv_h2, T vP, const T (&nb)[6]) {
    T s = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) s += i4(w, c, d, 0) * nb[2 * d] + i4(w, c, d, -1) * nb[2 * d + 1];
    return diag[c.self()] * vP - s * inv_h2;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_cheb_res(Phys ph, DevState* st, int k,
                                                     const T* __restrict__ rin, T* __restrict__ rout,
                                                     const T* __restrict__ q, const T* __restrict__ p,
                                                     const T* __restrict__ diag, const T* __restrict__ w,
                                                     T* __restrict__ x, T* __restrict__ z,
                                                     const double* part_theta, unsigned nb_theta,
                                                     const double* part_prev, double* part_out) {
    MEMBER(ph)
    PcgState& g = (st + mem_)->pcg;
    if (k > g.it_stop) return;
    double c0, c1, alpha = 0.0;
    if (k == 0) {
        double t[1];
        reduce_member<1, 1u>(part_theta, nb_theta, ph.batch, mem_, t);
        const double a = -t[0], b = 2.0 - a, mu = (b + a) / (b - a), t2 = 2.0 * mu * mu - 1.0;
        c0 = 8.0 * mu / ((b - a) * t2);
        c1 = -8.0 / ((b - a) * (b - a) * t2);
        if (MEMBER_FIRST()) {
            g.cheb[0] = c0;
            g.cheb[1] = c1;
        }
    } else {
        c0 = g.cheb[0];
        c1 = g.cheb[1];
        double t[kChebSet];
        reduce_member<kChebSet, 0u>(part_prev, num_blocks(), ph.batch, mem_, t);
        alpha = t[kChebRes] / t[kChebDir];
    }
    const T al = (T)alpha, inv_h2 = (T)ph.inv_h2;
    double v[2] = {0.0, 0.0};
    FOR_CELLS(ph)
    auto res = [&](size_t Q) -> T { return k == 0 ? rin[Q] : rin[Q] - al * q[Q]; };
    auto tv = [&](size_t Q) -> T { return res(Q) / diag[Q]; };
    const T rP = res(P), tP = rP / diag[P];
    const T nb[6] = {tv(c.sh(0, 1)), tv(c.sh(0, -1)), tv(c.sh(1, 1)), tv(c.sh(1, -1)),
                     tv(c.sh(2, 1)), tv(c.sh(2, -1))};
    const T Mt = m_diag_form(diag, w, c, inv_h2, tP, nb);
    const T zP = (T)c0 * tP + (T)c1 * Mt / diag[P];
    if (k > 0) {
        x[P] += al * p[P];
        rout[P] = rP;
    }
    z[P] = zP;
    v[0] += (double)rP * (double)zP;
    v[1] += (double)rP * (double)rP;
    END_CELLS
    block_partials<2, 0u>(v, part_out + kChebRes * (size_t)num_blocks());
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_cheb_dir(Phys ph, DevState* st, int k,
                                                     const T* __restrict__ z, const T* __restrict__ pin,
                                                     T* __restrict__ pout, T* __restrict__ q,
                                                     const T* __restrict__ diag, const T* __restrict__ w,
                                                     const double* part_u, unsigned nb_u,
                                                     const double* part_prev, double* part_cur,
                                                     int maxit) {
    MEMBER(ph)
    PcgState& g = (st + mem_)->pcg;
    if (k > g.it_stop) return;
    double t[kChebSet];
    reduce_member<kChebSet, 0u>(part_cur, num_blocks(), ph.batch, mem_, t);
    double bb;
    if (k == 0) {
        double u[3];
        reduce_member<3, 0u>(part_u, nb_u, ph.batch, mem_, u);
        bb = u[2];
    } else {
        bb = g.bb;
    }
    const double rr = t[kChebRes + 1];
    const bool conv = rr <= g.tol2 * bb;
    const bool stop = conv || k >= maxit;
    if (MEMBER_FIRST()) {
        if (k == 0) g.bb = bb;
        g.rr = rr;
        g.iters = k;
        if (stop) {
            g.it_stop = k;
            g.converged = conv ? 1 : 0;
        }
    }
    if (stop) return;
    double beta = 0.0;
    if (k > 0) {
        double tp[kChebSet];
        reduce_member<kChebSet, 0u>(part_prev, num_blocks(), ph.batch, mem_, tp);
        beta = t[kChebRes] / tp[kChebRes];
    }
    const T be = (T)beta, inv_h2 = (T)ph.inv_h2;
    double v[1] = {0.0};
    FOR_CELLS(ph)
    auto dir = [&](size_t Q) -> T { return k == 0 ? z[Q] : z[Q] + be * pin[Q]; };
    const T pP = dir(P);
    const T nb[6] = {dir(c.sh(0, 1)), dir(c.sh(0, -1)), dir(c.sh(1, 1)), dir(c.sh(1, -1)),
                     dir(c.sh(2, 1)), dir(c.sh(2, -1))};
    const T qP = m_diag_form(diag, w, c, inv_h2, pP, nb);
    pout[P] = pP;
    q[P] = qP;
    v[0] += (double)pP * (double)qP;
    END_CELLS
    block_partials<1, 0u>(v, part_cur + kChebDir * (size_t)num_blocks());
}

// psi/dt of a captured pressure system from its diagonal and w:
// psi/dt = diag - (1/h^2) sum_f I4(w)_f (one grid of n^3 FP64 values).
__global__ void __launch_bounds__(kBlock) k_psidt_of(int n, double inv_h2,
                                                     const double* __restrict__ diag,
                                                     const double* __restrict__ w,
                                                     double* __restrict__ out) {
    const size_t N = (size_t)n * n * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (size_t)gridDim.x * blockDim.x) {
        const CellIdx c(n, (int)(i % n), (int)((i / n) % n), (int)(i / ((size_t)n * n)), 0);
        double sumK = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) sumK += i4(w, c, d, 0) + i4(w, c, d, -1);
        out[i] = diag[i] - sumK * inv_h2;
    }
}

// ---- Fourier closure: the energy predictor (FP64 runs only; the sweep's tiled form is TiledEnergySweep) ----
// The internal energy c_v T of the gas, discretised like the momentum
// predictor (backward Euler, I4 convection with the old fluxes split into the
// diagonal (9/16) div(phi) and the rest, compact Laplacian for the heat flux
// q = -kappa grad T), with the compression work -p^n div u^n:
//   a_T T_P + N(T)_P = s_T,
//   a_T = c_v (rho*/dt + (9/16) div phi) + 6 kappa / h^2,
//   N(T) = c_v [div(phi I4(T)) - (9/16) div(phi) T_P] - (kappa / h^2) sum_nb T_nb,
//   s_T = c_v rho^n T^n / dt - p^n div u^n,
// solved by Jacobi sweeps from T^n (the momentum predictor's count).
template <typename T>
__device__ inline double div_phi_at(const T* __restrict__ phi, const CellIdx& c, size_t N, double inv_V) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) s += (double)phi[d * N + c.self()] - (double)phi[d * N + c.sh(d, -1)];
    return s * inv_V;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_energy_setup(Phys ph, const DevState* st,
                                                         const T* __restrict__ rn,
                                                         const T* __restrict__ rs,
                                                         const T* __restrict__ phi,
                                                         const T* __restrict__ divu,
                                                         const T* __restrict__ pn,
                                                         double* __restrict__ aT,
                                                         double* __restrict__ sT) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const double dt = (st + mem_)->dt, rref = (st + mem_)->rho_ref, pref = (st + mem_)->p_ref;
    const double diag_k = 6.0 * ph.kappa * ph.inv_h2;
    FOR_CELLS(ph)
    const double dphi = div_phi_at(phi, c, N, ph.inv_V);
    aT[P] = ph.cv * ((rref + (double)rs[P]) / dt + 0.5625 * dphi) + diag_k;
    sT[P] = ph.cv * (rref + (double)rn[P]) * ph.tn[P] / dt - (pref + (double)pn[P]) * (double)divu[P];
    END_CELLS
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_energy_sweep(Phys ph, const DevState* st,
                                                         const double* __restrict__ tin,
                                                         double* __restrict__ tout,
                                                         const T* __restrict__ phi,
                                                         const double* __restrict__ aT,
                                                         const double* __restrict__ sT) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    FOR_CELLS(ph)
    double conv = 0.0, nb = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        conv += (double)phi[d * N + P] * i4(tin, c, d, 0) -
                (double)phi[d * N + c.sh(d, -1)] * i4(tin, c, d, -1);
        nb += tin[c.sh(d, 1)] + tin[c.sh(d, -1)];
    }
    const double dphi = div_phi_at(phi, c, N, ph.inv_V);
    const double off = ph.cv * (conv * ph.inv_V - 0.5625 * dphi * tin[P]) - ph.kappa * ph.inv_h2 * nb;
    tout[P] = (sT[P] - off) / aT[P];
    END_CELLS
}

// ---- the momentum predictor solved to a tolerance (BiCGStab) ----
// A y = a_P y + N(y) for each velocity component, N the predictor's
// off-diagonal part (I4 convection with the predictor's face fluxes F, less
// its (9/16) div F diagonal; the compact viscous Laplacian without its centre):
//   N(y)_P = (1/V) sum_f F_f^out I4(y)_f - (9/16) div(F) y_P - (mu/h^2) sum_nb y_nb.
// b = s - grad p^n (Gauss-I4 gradient of the p^n field), the three components
// stacked into one system; BiCGStab (van der Vorst) right-preconditioned by
// K = diag(a_P), from x = u^n, to ||r|| <= mom_tol ||b||.  Per iteration i,
// five launches: k_bicg_dir tests r_{i-1} and forms p = r + beta (p - omega v)
// and y = K^-1 p on the cell; k_bicg_apply takes v = A y on the stencil;
// k_bicg_half forms s = r - alpha v and z = K^-1 s; k_bicg_apply again takes
// t = A z; k_bicg_update forms x += alpha y + omega z and r = s - omega t.
// The pointwise launches let the stencil ones read one stored field.
template <typename T>
__device__ inline double mom_op(const T* __restrict__ F, const T* __restrict__ aP,
                                const T* __restrict__ y, const CellIdx& c, size_t N, double inv_V,
                                double mu_h2) {
    const size_t P = c.self();
    const double yP = (double)y[P];
    double conv = 0.0, dF = 0.0, nb = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double fp = (double)F[d * N + P], fm = (double)F[d * N + c.sh(d, -1)];
        const double ym2 = (double)y[c.sh(d, -2)], ym1 = (double)y[c.sh(d, -1)],
                     yp1 = (double)y[c.sh(d, 1)], yp2 = (double)y[c.sh(d, 2)];
        conv += fp * ((9.0 * (yP + yp1) - (ym1 + yp2)) * 0.0625) -
                fm * ((9.0 * (ym1 + yP) - (ym2 + yp1)) * 0.0625);
        dF += fp - fm;
        nb += yp1 + ym1;
    }
    return (double)aP[P] * yP + conv * inv_V - 0.5625 * dF * inv_V * yP - mu_h2 * nb;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_init(Phys ph, DevState* st, const T* __restrict__ x,
                                                      const T* __restrict__ F, const T* __restrict__ aP,
                                                      const T* __restrict__ src, const T* __restrict__ pn,
                                                      T* __restrict__ r, T* __restrict__ rh,
                                                      double* part) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const double mu_h2 = ph.mu * ph.inv_h2;
    double v[3] = {0.0, 0.0, 0.0};   // (rh, r) = (r, r), (r, r), (b, b)
    FOR_CELLS(ph)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double b = (double)src[m * N + P] - (double)((i4(pn, c, m, 0) - i4(pn, c, m, -1)) * (T)ph.inv_h);
        const double ax = mom_op(F, aP, x + m * N, c, N, ph.inv_V, mu_h2);
        const double rr = b - ax;
        r[m * N + P] = (T)rr;
        rh[m * N + P] = (T)rr;
        v[0] += rr * rr;
        v[2] += b * b;
    }
    v[1] = v[0];
    END_CELLS
    block_partials<3, 0u>(v, part);
    if (MEMBER_FIRST()) {
        BicgState& g = (st + mem_)->bicg;
        g.it_stop = kIterInf;
        g.iters = 0;
        g.converged = 0;
    }
}

// Test r_{i-1}; p = r + beta (p - omega v), y = p / a_P (on the cell).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_dir(Phys ph, DevState* st, int i, double tol2, int maxit,
                                                     const T* __restrict__ r, T* __restrict__ p,
                                                     const T* __restrict__ vv, T* __restrict__ y,
                                                     const T* __restrict__ aP, const double* part_res) {
    MEMBER(ph)
    BicgState& g = (st + mem_)->bicg;
    if (i - 1 > g.it_stop) return;
    const size_t N = ncell(ph);
    double t[3];
    reduce_member<3, 0u>(part_res, num_blocks(), ph.batch, mem_, t);
    const double rho = t[0], rr = t[1], bb = i == 1 ? t[2] : g.bb;
    const bool conv = rr <= tol2 * bb;
    const bool stop = conv || i - 1 >= maxit;
    if (MEMBER_FIRST()) {
        if (i == 1) g.bb = bb;
        g.rr = rr;
        g.rho = rho;
        if (stop) {
            g.it_stop = i - 1;
            g.iters = i - 1;
            g.converged = conv ? 1 : 0;
            if (!conv) (st + mem_)->flags |= 1024;   // the cap reached first
        }
    }
    if (stop) return;
    const double beta = i == 1 ? 0.0 : (rho / g.rho_old) * (g.alpha / g.omega);
    const double om = i == 1 ? 0.0 : g.omega;
    FOR_CELLS(ph)
    const double ia = 1.0 / (double)aP[P];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const size_t o = m * N + P;
        const double pv = i == 1 ? (double)r[o] : (double)r[o] + beta * ((double)p[o] - om * (double)vv[o]);
        p[o] = (T)pv;
        y[o] = (T)(pv * ia);
    }
    END_CELLS
}

// out = A y for the three components; partials (w, out) and, with w2, (out, out).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_apply(Phys ph, DevState* st, int i, int after_half,
                                                       const T* __restrict__ y, T* __restrict__ out,
                                                       const T* __restrict__ F, const T* __restrict__ aP,
                                                       const T* __restrict__ w, double* part) {
    MEMBER(ph)
    const BicgState& g = (st + mem_)->bicg;
    if (i - 1 >= g.it_stop) return;
    const size_t N = ncell(ph);
    const double mu_h2 = ph.mu * ph.inv_h2;
    double v[2] = {0.0, 0.0};
    FOR_CELLS(ph)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double a = mom_op(F, aP, y + m * N, c, N, ph.inv_V, mu_h2);
        out[m * N + P] = (T)a;
        v[0] += (double)w[m * N + P] * a;
        v[1] += a * a;
    }
    END_CELLS
    if (after_half) {
        block_partials<2, 0u>(v, part);
    } else {
        double v1[1] = {v[0]};
        block_partials<1, 0u>(v1, part);
    }
}

// alpha = rho / (rh, v); s = r - alpha v, z = s / a_P (on the cell).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_half(Phys ph, DevState* st, int i,
                                                      const T* __restrict__ r, const T* __restrict__ vv,
                                                      T* __restrict__ s, T* __restrict__ z,
                                                      const T* __restrict__ aP, const double* part_v,
                                                      unsigned nb_v) {
    MEMBER(ph)
    BicgState& g = (st + mem_)->bicg;
    if (i - 1 >= g.it_stop) return;
    const size_t N = ncell(ph);
    double rv[1];
    reduce_member<1, 0u>(part_v, nb_v, ph.batch, mem_, rv);
    const double alpha = g.rho / rv[0];
    if (MEMBER_FIRST()) g.alpha = alpha;
    FOR_CELLS(ph)
    const double ia = 1.0 / (double)aP[P];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const size_t o = m * N + P;
        const double sv = (double)r[o] - alpha * (double)vv[o];
        s[o] = (T)sv;
        z[o] = (T)(sv * ia);
    }
    END_CELLS
}

// omega = (t, s) / (t, t); x += alpha y + omega z; r = s - omega t.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_update(Phys ph, DevState* st, int i, T* __restrict__ x,
                                                        const T* __restrict__ y, const T* __restrict__ z,
                                                        const T* __restrict__ s, const T* __restrict__ tt,
                                                        T* __restrict__ r, const T* __restrict__ rh,
                                                        const double* part_ts, unsigned nb_ts,
                                                        double* part_res) {
    MEMBER(ph)
    BicgState& g = (st + mem_)->bicg;
    if (i - 1 >= g.it_stop) return;
    const size_t N = ncell(ph);
    double ts[2];
    reduce_member<2, 0u>(part_ts, nb_ts, ph.batch, mem_, ts);
    const double omega = ts[1] > 0.0 ? ts[0] / ts[1] : 0.0;
    const double alpha = g.alpha;
    if (MEMBER_FIRST()) {
        g.omega = omega;
        g.rho_old = g.rho;
    }
    double v[2] = {0.0, 0.0};
    FOR_CELLS(ph)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const size_t o = m * N + P;
        x[o] = (T)((double)x[o] + alpha * (double)y[o] + omega * (double)z[o]);
        const double rn = (double)s[o] - omega * (double)tt[o];
        r[o] = (T)rn;
        v[0] += (double)rh[o] * rn;
        v[1] += rn * rn;
    }
    END_CELLS
    block_partials<2, 0u>(v, part_res);
}

// y = M x for the stand-alone operator entry point (psi/dt given as a field).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_helm_apply(Phys ph, const T* __restrict__ psidt,
                                                       const T* __restrict__ w, const T* __restrict__ x,
                                                       T* __restrict__ y) {
    MEMBER(ph)
    const T inv_h2 = (T)ph.inv_h2;
    FOR_CELLS(ph)
    const T xP = x[P];
    T s = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s += i4(w, c, d, 0) * (xP - x[c.sh(d, 1)]);
        s += i4(w, c, d, -1) * (xP - x[c.sh(d, -1)]);
    }
    y[P] = psidt[P] * xP + s * inv_h2;
    END_CELLS
}

// diag(M) = psi/dt + sum_f K_f / h^2, and r = b - M x with partial sums
// b.b, r.(r/diag), r.r (CG start from an arbitrary x).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_helm_start(Phys ph, DevState* st,
                                                       const T* __restrict__ psidt,
                                                       const T* __restrict__ w, const T* __restrict__ b,
                                                       const T* __restrict__ x, T* __restrict__ r,
                                                       T* __restrict__ diag, double* part_u) {
    MEMBER(ph)
    const T inv_h2 = (T)ph.inv_h2;
    double v[3] = {0.0, 0.0, 0.0};
    FOR_CELLS(ph)
    const T xP = x[P];
    T s = T(0), sumK = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T kp = i4(w, c, d, 0), km = i4(w, c, d, -1);
        s += kp * (xP - x[c.sh(d, 1)]) + km * (xP - x[c.sh(d, -1)]);
        sumK += kp + km;
    }
    const T dg = psidt[P] + sumK * inv_h2;
    const T rr = b[P] - (psidt[P] * xP + s * inv_h2);
    r[P] = rr;
    diag[P] = dg;
    v[0] += (double)rr * ((double)rr / (double)dg);
    v[1] += (double)rr * (double)rr;
    v[2] += (double)b[P] * (double)b[P];
    END_CELLS
    block_partials<3, 0u>(v, part_u);
    if (MEMBER_FIRST()) {
        (st + mem_)->pcg.it_stop = kIterInf;
        (st + mem_)->pcg.converged = 0;
        (st + mem_)->pcg.iters = 0;
    }
}

// ---------------------------------------------------------------- learned guess
// Partial sums for the network's input scaling: sum (b/diag)^2, sum p0, sum p0^2.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_net_stats(Phys ph, const T* __restrict__ b,
                                                      const T* __restrict__ diag,
                                                      const T* __restrict__ p0, double* part) {
    MEMBER(ph)
    double v[3] = {0.0, 0.0, 0.0};
    FOR_CELLS(ph)
    const double z = (double)b[P] / (double)diag[P];
    const double p = (double)p0[P];
    v[0] += z * z;
    v[1] += p;
    v[2] += p * p;
    END_CELLS
    block_partials<3, 0u>(v, part);
}

// Network inputs: channel 0 = (b/diag)/s1, channel 1 = (p0 - <p0>)/s2 with s1, s2
// their r.m.s. (the Jacobi-scaled continuity defect and the pressure of the
// current density iterate, each normalised); BF16 [cell][4] and/or FP32
// [cell][2]; with psol the training target psol/s1.  s1, s2 go to (st + mem_)->red[6..7].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_net_input(Phys ph, DevState* st, const double* part,
                                                      unsigned nb, const T* __restrict__ b,
                                                      const T* __restrict__ diag,
                                                      const T* __restrict__ p0,
                                                      uint16_t* __restrict__ x4, float* __restrict__ x2,
                                                      const T* __restrict__ psol,
                                                      float* __restrict__ tgt) {
    MEMBER(ph)
    double t[3];
    reduce_member<3, 0u>(part, nb, ph.batch, mem_, t);
    const double N = (double)ph.N;
    const double s1 = sqrt(t[0] / N);
    const double mean = t[1] / N;
    const double var = t[2] / N - mean * mean;
    const double s2 = var > 0.0 ? sqrt(var) : 0.0;
    const double i1 = s1 > 0.0 ? 1.0 / s1 : 0.0, i2 = s2 > 0.0 ? 1.0 / s2 : 0.0;
    if (st && MEMBER_FIRST()) {
        (st + mem_)->red[6] = s1;
        (st + mem_)->red[7] = s2;
    }
    FOR_CELLS(ph)
    const float c0 = (float)((double)b[P] / (double)diag[P] * i1);
    const float c1 = (float)(((double)p0[P] - mean) * i2);
    if (x4) {
        x4[4 * P + 0] = f2bf(c0);
        x4[4 * P + 1] = f2bf(c1);
        x4[4 * P + 2] = 0;
        x4[4 * P + 3] = 0;
    }
    if (x2) {
        x2[2 * P + 0] = c0;
        x2[2 * P + 1] = c1;
    }
    if (tgt) tgt[P] = (float)((double)psol[P] * i1);
    END_CELLS
}

// The guess g and M g (difference form, FP64 arithmetic), stored in the CG
// scratch vectors, with partial sums g.b and g.(M g): g = s1 y for the
// network's output y, or g = gd (the previous step's solution) when gd is set.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_guess_start(Phys ph, const DevState* st,
                                                        const float* __restrict__ y,
                                                        const T* __restrict__ gd,
                                                        const T* __restrict__ w,
                                                        const T* __restrict__ diag,
                                                        const T* __restrict__ b,
                                                        const double* __restrict__ b64,
                                                        T* __restrict__ gout, T* __restrict__ mg,
                                                        double* part) {
    MEMBER(ph)
    const double s1 = (st + mem_)->red[6], inv_h2 = ph.inv_h2;
    double v[2] = {0.0, 0.0};
    FOR_CELLS(ph)
    T wv[13];
    float yv[7];
    T gv[7];
    gather13(w, c, wv);
    if (gd) gather7(gd, c, gv);
    else gather7(y, c, yv);
    const T dgP = diag[P];
    const double bP = b64 ? b64[P] : (double)b[P];
    loads_issued();
    auto g = [&](int t) { return gd ? (double)gv[t] : s1 * (double)yv[t]; };
    const double gP = g(0);
    double lap = 0.0, sumK = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double kp = i4gr<double>(wv, d, 0), km = i4gr<double>(wv, d, -1);
        lap += kp * (gP - g(2 + 2 * d)) + km * (gP - g(1 + 2 * d));
        sumK += kp + km;
    }
    const double Mg = ((double)dgP - sumK * inv_h2) * gP + lap * inv_h2;
    gout[P] = (T)gP;
    mg[P] = (T)Mg;
    v[0] += gP * bP;
    v[1] += gP * Mg;
    END_CELLS
    block_partials<2, 0u>(v, part);
}

// Start CG from x0 = alpha g with the energy-optimal alpha = g.b / g.(M g) (the
// first CG step along g, so that a poor guess is shrunk rather than followed):
// r = b - alpha M g, b kept in bsave for a fallback.  FP64 storage: x = x0.
// FP32 storage (x64 non-null): x64 = x0 and the inner correction x = 0.
// Partial sums r.(r/diag), ||r0||^2, ||b||^2; alpha goes to (st + mem_)->red[5].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_guess_apply(Phys ph, DevState* st, const double* part_g,
                                                        unsigned nb, const T* __restrict__ g,
                                                        const T* __restrict__ mg,
                                                        const T* __restrict__ diag, T* __restrict__ r,
                                                        T* __restrict__ x, double* __restrict__ x64,
                                                        const double* __restrict__ b64,
                                                        T* __restrict__ bsave, double* part_u) {
    MEMBER(ph)
    double t[2];
    reduce_member<2, 0u>(part_g, nb, ph.batch, mem_, t);
    const double alpha = t[1] > 0.0 ? t[0] / t[1] : 0.0;
    if (MEMBER_FIRST()) {
        (st + mem_)->red[5] = alpha;
        (st + mem_)->pcg.it_stop = kIterInf;
        (st + mem_)->pcg.converged = 0;
        (st + mem_)->pcg.iters = 0;
    }
    double v[3] = {0.0, 0.0, 0.0};
    FOR_CELLS(ph)
    const double bP = b64 ? b64[P] : (double)r[P];
    const double x0 = alpha * (double)g[P];
    const double r0 = bP - alpha * (double)mg[P];
    bsave[P] = r[P];
    const T rT = (T)r0;
    r[P] = rT;
    if (x64) {
        x64[P] = x0;
        x[P] = T(0);
    } else {
        x[P] = (T)x0;
    }
    v[0] += (double)rT * ((double)rT / (double)diag[P]);
    v[1] += r0 * r0;
    v[2] += bP * bP;
    END_CELLS
    block_partials<3, 0u>(v, part_u);
}

// Fallback to the zero guess where the guess does not lower the residual
// (red[1] = ||b - M x0||^2 not below red[2] = ||b||^2, totals left by
// finalize_sums): r = b, x = 0 (and x64 = 0), partials as corr_rhs, flag 8.
// The decision is per member, so all blocks of a member agree.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_guess_revert(Phys ph, DevState* st, T* __restrict__ r,
                                                         T* __restrict__ x, double* __restrict__ x64,
                                                         const double* __restrict__ b64,
                                                         const T* __restrict__ bsave,
                                                         const T* __restrict__ diag, double* part_u) {
    MEMBER(ph)
    if ((st + mem_)->red[1] < (st + mem_)->red[2]) return;
    if (MEMBER_FIRST()) (st + mem_)->flags |= 8;
    double v[3] = {0.0, 0.0, 0.0};
    FOR_CELLS(ph)
    const T bT = bsave[P];
    r[P] = bT;
    x[P] = T(0);
    if (x64) x64[P] = 0.0;
    const double bd = (double)bT, bb = b64 ? b64[P] : bd;
    v[0] += bd * (bd / (double)diag[P]);
    v[1] += bb * bb;
    v[2] += bb * bb;
    END_CELLS
    block_partials<3, 0u>(v, part_u);
}

// ---------------------------------------------------------------- correction
// p = p0 + p'; corrected face fluxes phi = phiH - K A snGrad(p) on own faces.
template <typename T>
__device__ inline void corr_flux_cell(const T (&wv)[13], T p0P, T xP, const T (&p0n)[3],
                                      const T (&xn)[3], const T (&hP)[3], T A, T inv_h, T& pP,
                                      T (&fk)[3]) {
    pP = p0P + xP;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T pQ = p0n[d] + xn[d];
        fk[d] = hP[d] - i4g(wv, d, 0) * A * (pQ - pP) * inv_h;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_corr_flux(Phys ph, const T* __restrict__ p0,
                                                      const T* __restrict__ x, const T* __restrict__ w,
                                                      const T* __restrict__ phiH, T* __restrict__ phik,
                                                      T* __restrict__ pt, double* snap_x) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T A = (T)ph.A, inv_h = (T)ph.inv_h;
    FOR_CELLS(ph)
    T wv[13], p0n[3], xn[3], hP[3];
    gather13(w, c, wv);
    const T p0P = p0[P], xP = x[P];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const size_t Q = c.sh(d, 1);
        p0n[d] = p0[Q];
        xn[d] = x[Q];
        hP[d] = phiH[d * N + P];
    }
    loads_issued();
    T pP, fk[3];
    corr_flux_cell(wv, p0P, xP, p0n, xn, hP, A, inv_h, pP, fk);
    pt[P] = pP;
#pragma unroll
    for (int d = 0; d < 3; ++d) phik[d * N + P] = fk[d];
    if (snap_x) snap_x[P] = (double)xP;
    END_CELLS
}

// Conservative density rho_k = rho^n - dt div(phi) and velocity
// u = HbyA - grad(p)/a_P.  On the last corrector, partial sums for the mass
// budget and the divergence checks (sum r, sum |u|^2, max(-rho)).
template <typename T>
__device__ inline void corr_update_cell(const T (&pv)[13], const T (&fp)[3], const T (&fm)[3],
                                        const T (&hb)[3], T rnP, T a, T dt, T inv_V, T inv_h,
                                        T& r, T (&um)[3]) {
    T dphi = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) dphi += fp[d] - fm[d];
    r = rnP - dt * dphi * inv_V;
#pragma unroll
    for (int m = 0; m < 3; ++m) um[m] = hb[m] - dgauss13(pv, m, inv_h) / a;
}

// BDF2's conservative density: rho_k = (c1 rho^n - c2 rho^{n-1} - dt div phi_k) / c0.
template <typename T>
__device__ inline T corr_rho_bdf2(const T (&fp)[3], const T (&fm)[3], T rnP, double rm1P, T dt,
                                  double inv_V, const double* bc) {
    double dphi = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) dphi += (double)fp[d] - (double)fm[d];
    return (T)((bc[1] * (double)rnP - bc[2] * rm1P - (double)dt * dphi * inv_V) / bc[0]);
}

template <typename T, bool LAST>
__global__ void __launch_bounds__(kBlock) k_corr_update(Phys ph, const DevState* st,
                                                        const T* __restrict__ rn,
                                                        const T* __restrict__ phik,
                                                        const T* __restrict__ hbya,
                                                        const T* __restrict__ pt,
                                                        const T* __restrict__ aP, T* __restrict__ rk,
                                                        T* __restrict__ u, double* partials) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T dt = (T)(st + mem_)->dt;
    const T inv_V = (T)ph.inv_V, inv_h = (T)ph.inv_h;
    double v[3] = {0.0, 0.0, -__builtin_inf()};
    FOR_CELLS(ph)
    T fp[3], fm[3], hb[3], pv[13];
    gather13(pt, c, pv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        fp[d] = phik[d * N + P];
        fm[d] = phik[d * N + c.sh(d, -1)];
        hb[d] = hbya[d * N + P];
    }
    const T rnP = rn[P], a = aP[P];
    loads_issued();
    T r, um[3];
    corr_update_cell(pv, fp, fm, hb, rnP, a, dt, inv_V, inv_h, r, um);
    if (ph.bdf2) r = corr_rho_bdf2(fp, fm, rnP, ph.rm1[P], dt, ph.inv_V, (st + mem_)->bdf);
    rk[P] = r;
    double usq = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        u[m * N + P] = um[m];
        usq += (double)um[m] * (double)um[m];
    }
    if (LAST) {
        v[0] += (double)r;
        v[1] += usq;
        double nrho = -((st + mem_)->rho_ref + (double)r);
        v[2] = nrho > v[2] ? nrho : v[2];
    }
    END_CELLS
    if (LAST) block_partials<3, 4u>(v, partials);
}

// ---------------------------------------------------------------- dust
// Particle-velocity correction source a = Du/Dt = (u^{n+1} - u^n)/dt + (u^{n+1}.grad)u^{n+1}.
// BDF2's a = (c0 u^{n+1} - c1 u^n + c2 u^{n-1}) / dt + (u.grad)u, u^{n-1} at
// um1 (components N apart).
template <typename T>
__device__ inline void dudt_bdf2_cell(const T (&uv)[3][13], const T (&u0)[3], const double* um1,
                                      size_t N, size_t P, T dt, T inv_h, const double* bc,
                                      T (&out)[3]) {
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const T conv = uv[0][0] * dgauss13(uv[m], 0, inv_h) + uv[1][0] * dgauss13(uv[m], 1, inv_h) +
                       uv[2][0] * dgauss13(uv[m], 2, inv_h);
        out[m] = (T)((bc[0] * (double)uv[m][0] - bc[1] * (double)u0[m] + bc[2] * um1[m * N + P]) /
                     (double)dt) + conv;
    }
}

template <typename T>
__device__ inline void dudt_cell(const T (&uv)[3][13], const T (&u0)[3], T dt, T inv_h,
                                 T (&out)[3]) {
    const T ux = uv[0][0], uy = uv[1][0], uz = uv[2][0];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const T conv = ux * dgauss13(uv[m], 0, inv_h) + uy * dgauss13(uv[m], 1, inv_h) +
                       uz * dgauss13(uv[m], 2, inv_h);
        out[m] = (uv[m][0] - u0[m]) / dt + conv;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dudt(Phys ph, const DevState* st,
                                                 const T* __restrict__ un, const T* __restrict__ u1,
                                                 T* __restrict__ acc) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T dt = (T)(st + mem_)->dt, inv_h = (T)ph.inv_h;
    FOR_CELLS(ph)
    T uv[3][13], u0[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        gather13(u1 + m * N, c, uv[m]);
        u0[m] = un[m * N + P];
    }
    loads_issued();
    T out[3];
    dudt_cell(uv, u0, dt, inv_h, out);
    if (ph.bdf2) dudt_bdf2_cell(uv, u0, ph.um1, N, P, dt, inv_h, (st + mem_)->bdf, out);
#pragma unroll
    for (int m = 0; m < 3; ++m) acc[m * N + P] = out[m];
    END_CELLS
}

// Particle mass flux per unit mass ratio on own faces,
// G_d = phi_d - tau I4(rho^{n+1}) (I4(a_d) - g_d) A  (u_p = u + tau (g - Du/Dt)
// at the face), and the starting mass ratio Y = rho_j^n / rho^n.
template <typename T>
__device__ inline void dust_flux_cell(const T (&rv)[13], const T (&al)[3][5], const T (&fv)[3],
                                      T rj, T rnP, T t, T rref, T A, const double (&gr)[3],
                                      T (&g)[3], T& y) {
#pragma unroll
    for (int d = 0; d < 3; ++d)
        g[d] = fv[d] - t * (rref + i4g(rv, d, 0)) * (i4l<T>(al[d], 0) - (T)gr[d]) * A;
    y = rj / (rref + rnP);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dust_flux(Phys ph, const DevState* st, int cls, const T* __restrict__ phi,
                                                      const T* __restrict__ r1, const T* __restrict__ acc,
                                                      T* __restrict__ G, const T* __restrict__ rhoj,
                                                      const T* __restrict__ rn, T* __restrict__ Y) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T A = (T)ph.A, t = (T)(st + mem_)->tau[cls], rref = (T)(st + mem_)->rho_ref;
    FOR_CELLS(ph)
    T rv[13], al[3][5], fv[3];
    gather13(r1, c, rv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        gather_line(acc + d * N, c, d, al[d]);
        fv[d] = phi[d * N + P];
    }
    const T rj = rhoj[P], rnP = rn[P];
    loads_issued();
    T g[3], y;
    dust_flux_cell(rv, al, fv, rj, rnP, t, rref, A, ph.g, g, y);
#pragma unroll
    for (int d = 0; d < 3; ++d) G[d * N + P] = g[d];
    Y[P] = y;
    END_CELLS
}

// One Jacobi sweep of the implicit mass-ratio equation
//   rho^{n+1} Y / dt + (1/V) sum_f G_f^out I4(Y)_f = rho_j^n / dt,
// diagonal rho^{n+1}/dt + (9/16) div G (returned in diag).
template <typename T>
__device__ inline T dust_sweep_cell(const T (&yv)[13], const T (&gpv)[3], const T (&gmv)[3], T rj,
                                    T r1P, T dt, T inv_V, T rref, T& diag) {
    T conv = T(0), dG = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T gp = gpv[d], gm = gmv[d];
        conv += gp * i4g(yv, d, 0) - gm * i4g(yv, d, -1);
        dG += gp - gm;
    }
    conv *= inv_V;
    dG *= inv_V;
    const T off = conv - T(0.5625) * dG * yv[0];
    diag = (rref + r1P) / dt + T(0.5625) * dG;
    return (rj / dt - off) / diag;
}

// BDF2's sweep: diagonal c0 rho^{n+1}/dt + (9/16) div G, right side
// (c1 rho_j - c2 rho_j^{n-1})/dt.
template <typename T>
__device__ inline T dust_sweep_bdf2_cell(const T (&yv)[13], const T (&gpv)[3], const T (&gmv)[3],
                                         T rj, double rjm1P, T r1P, T dt, T inv_V, double rref,
                                         const double* bc, T& diag) {
    T conv = T(0), dG = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        conv += gpv[d] * i4g(yv, d, 0) - gmv[d] * i4g(yv, d, -1);
        dG += gpv[d] - gmv[d];
    }
    conv *= inv_V;
    dG *= inv_V;
    const T off = conv - T(0.5625) * dG * yv[0];
    diag = (T)(bc[0] * (rref + (double)r1P) / (double)dt) + T(0.5625) * dG;
    return ((T)((bc[1] * (double)rj - bc[2] * rjm1P) / (double)dt) - off) / diag;
}

// CHECK (a class's first sweep; the diagonal and G are the same in every
// sweep): partials of max(-diagonal), so that a diagonal <= 0 anywhere is
// flagged, and of the dust's Courant rate sum_f |G_f| / (2 rho^{n+1} V).
template <typename T, bool CHECK>
__global__ void __launch_bounds__(kBlock) k_dust_sweep(Phys ph, const DevState* st,
                                                       const T* __restrict__ Yin, T* __restrict__ Yout,
                                                       const T* __restrict__ G, const T* __restrict__ rhoj,
                                                       const T* __restrict__ r1, double* part) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T dt = (T)(st + mem_)->dt, inv_V = (T)ph.inv_V;
    double v[2] = {-__builtin_inf(), 0.0};
    const double rref = (st + mem_)->rho_ref;
    FOR_CELLS(ph)
    T yv[13], gpv[3], gmv[3];
    gather13(Yin, c, yv);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        gpv[d] = G[d * N + P];
        gmv[d] = G[d * N + c.sh(d, -1)];
    }
    const T rj = rhoj[P], r1P = r1[P];
    loads_issued();
    T dg;
    if (ph.bdf2) {
        Yout[P] = dust_sweep_bdf2_cell(yv, gpv, gmv, rj, ph.rjm1[P], r1P, dt, inv_V, rref,
                                       (st + mem_)->bdf, dg);
    } else {
        Yout[P] = dust_sweep_cell(yv, gpv, gmv, rj, r1P, dt, inv_V, (T)(st + mem_)->rho_ref, dg);
    }
    if (CHECK) {
        v[0] = fmax(v[0], -(double)dg);
        v[1] = fmax(v[1], courant_rate(gpv, gmv, r1P, rref, ph.V));
    }
    END_CELLS
    if (CHECK) block_partials<2, 3u>(v, part);
}

// Face dust mass fluxes F = G I4(Y), overwriting G on own faces.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dust_faceflux(Phys ph, const T* __restrict__ Y,
                                                          T* __restrict__ G) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    FOR_CELLS(ph)
#pragma unroll
    for (int d = 0; d < 3; ++d) G[d * N + P] *= i4(Y, c, d, 0);
    END_CELLS
}

// Conservative finish rho_j^{n+1} = rho_j^n - dt div(F); partial sums of
// rho_j^{n+1} (mass; non-finite if any value is) and max(-rho_j^{n+1}).
// fdo (two-way coupling): the class's own-face fluxes are added to the
// mixture's dust flux F_d of the next step (written by the first class).
// BDF2's conservative finish: (c1 rho_j - c2 rho_j^{n-1} - dt div F) / c0.
template <typename T>
__device__ inline T dust_finish_bdf2(T rj, double rjm1P, T dt, T dF, T inv_V, const double* bc) {
    return (T)((bc[1] * (double)rj - bc[2] * rjm1P - (double)(dt * dF * inv_V)) / bc[0]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dust_finish(Phys ph, const DevState* st,
                                                        const T* __restrict__ rhoj,
                                                        const T* __restrict__ F, T* __restrict__ rhoj1,
                                                        double* partials, T* __restrict__ fdo,
                                                        int first) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T dt = (T)(st + mem_)->dt, inv_V = (T)ph.inv_V;
    double v[2] = {0.0, -__builtin_inf()};
    FOR_CELLS(ph)
    T dF = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) dF += F[d * N + P] - F[d * N + c.sh(d, -1)];
    if (fdo)
#pragma unroll
        for (int d = 0; d < 3; ++d) fdo[d * N + P] = (first ? T(0) : fdo[d * N + P]) + F[d * N + P];
    const T out = ph.bdf2 ? dust_finish_bdf2(rhoj[P], ph.rjm1[P], dt, dF, inv_V, (st + mem_)->bdf)
                          : rhoj[P] - dt * dF * inv_V;
    rhoj1[P] = out;
    v[0] += (double)out;
    v[1] = fmax(v[1], -(double)out);
    END_CELLS
    block_partials<2, 2u>(v, partials);
}

// ---------------------------------------------------------------- statistics
// Partial sums of rho|u|^2/2, |curl u|^2/2 (Gauss-I4), |u|^2 and r.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_stats_gas(Phys ph, const DevState* st,
                                                      const T* __restrict__ r,
                                                      const T* __restrict__ u, double* partials) {
    MEMBER(ph)
    const size_t N = ncell(ph);
    const T inv_h = (T)ph.inv_h;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    FOR_CELLS(ph)
    const T* ux = u;
    const T* uy = u + N;
    const T* uz = u + 2 * N;
    const double wx = (double)(dgauss(uz, c, 1, inv_h) - dgauss(uy, c, 2, inv_h));
    const double wy = (double)(dgauss(ux, c, 2, inv_h) - dgauss(uz, c, 0, inv_h));
    const double wz = (double)(dgauss(uy, c, 0, inv_h) - dgauss(ux, c, 1, inv_h));
    const double q = (double)ux[P] * ux[P] + (double)uy[P] * uy[P] + (double)uz[P] * uz[P];
    v[0] += 0.5 * ((st + mem_)->rho_ref + (double)r[P]) * q;
    v[1] += 0.5 * (wx * wx + wy * wy + wz * wz);
    v[2] += q;
    v[3] += (double)r[P];
    END_CELLS
    block_partials<4, 0u>(v, partials);
}

// Partial sums of (a x + b)^2 and of x, with per-member (a, b) = st[m].aff when
// st is given, else the arguments.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sum_affine_sq(Phys ph, const DevState* st,
                                                          const T* __restrict__ x, double a0,
                                                          double b0, double* partials) {
    MEMBER(ph)
    const double a = st ? (st + mem_)->aff[0] : a0, b = st ? (st + mem_)->aff[1] : b0;
    double v[2] = {0.0, 0.0};
    FOR_CELLS(ph)
    const double y = a * (double)x[P] + b;
    v[0] += y * y;
    v[1] += (double)x[P];
    END_CELLS
    block_partials<2, 0u>(v, partials);
}

// One block per member: totals of nv partial columns (sums) of member
// blockIdx.x into st[member].red[off .. off + nv).
__global__ void __launch_bounds__(kBlock) k_finalize_sums(const double* part, unsigned nbt,
                                                          int batch, int nv, DevState* st, int off,
                                                          int honor_skip) {
    const int m = blockIdx.x;
    if (honor_skip && st[m].pcg.skip) return;   // a skipped refinement round wrote no partials
    for (int c = 0; c < nv; ++c) {
        double t[1];
        reduce_member<1, 0u>(part + (size_t)c * nbt, nbt, batch, m, t);
        if (flat_tid() == 0) st[m].red[off + c] = t[0];
    }
}

// Total of nb partials into dst[0] (one block).
__global__ void __launch_bounds__(kBlock) k_sum_partials(const double* part, unsigned nb,
                                                         double* dst) {
    double t[1];
    reduce_partials<1, 0u>(part, nb, t);
    if (flat_tid() == 0) dst[0] = t[0];
}

// One block per member at the end of a step: mass budget, divergence flags
// and the dust class masses from the partials of the last corrector and of
// the dust finish, and the dust flags: 64 some rho_j < 0, 128 a non-finite
// rho_j (the sum is then non-finite), 256 the implicit diagonal <= 0 in some
// cell (from the first sweep's maxima of -diagonal), 512 the dust's Courant
// number (the first sweep's maxima of its rate, times dt) at or above
// kDustCourantMax, beyond which the transport update amplifies some Fourier
// mode of a uniform drift.
__global__ void __launch_bounds__(kBlock) k_step_finish(Phys ph, DevState* st,
                                                        const double* part_mass, unsigned nb_mass,
                                                        const double* part_dust, int ncls,
                                                        unsigned nb_dust, const double* part_diag,
                                                        unsigned nb_diag, size_t cls_stride) {
    const int m = blockIdx.x;
    DevState* sm = st + m;
    double v[3];
    reduce_member<3, 4u>(part_mass, nb_mass, ph.batch, m, v);
    if (flat_tid() == 0) {
        sm->mass_gas = (sm->rho_ref * (double)ph.N + v[0]) * ph.V;
        sm->usq = v[1];
        sm->rho_min = -v[2];
        if (!isfinite(v[0]) || !isfinite(v[1])) sm->flags |= 2;
        if (!(-v[2] > 0.0)) sm->flags |= 4;
    }
    if (flat_tid() == 0) sm->courant_dust = 0.0;
    for (int c = 0; c < ncls; ++c) {
        // columns nb_dust apart: sum rho_j, max(-rho_j); nb_diag apart:
        // max(-diagonal), max Courant rate
        double mm[2], dg[2];
        reduce_member<2, 2u>(part_dust + (size_t)(2 * c) * cls_stride, nb_dust, ph.batch, m, mm);
        reduce_member<2, 3u>(part_diag + (size_t)(2 * c) * cls_stride, nb_diag, ph.batch, m, dg);
        if (flat_tid() == 0) {
            sm->mass_p[c] = mm[0] * ph.V;
            if (!isfinite(mm[0])) sm->flags |= 128;
            else if (mm[1] > 0.0) sm->flags |= 64;
            if (!(dg[0] < 0.0)) sm->flags |= 256;
            const double cd = dg[1] * sm->dt;
            if (cd > sm->courant_dust) sm->courant_dust = cd;
            if (!(cd < kDustCourantMax)) sm->flags |= 512;
        }
    }
}

// Accept the step of every member: t += dt, dt_prev = dt, and fold the step
// record into the accumulators (one thread per member).
__global__ void k_commit(DevState* st, int batch) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= batch) return;
    DevState& d = st[m];
    d.t += d.dt;
    d.dt_prev = d.dt;
    d.flags_acc |= d.flags;
    d.steps_acc += 1;
    for (int c = 0; c < kMaxCorr; ++c) {
        if (d.it_first[c] > d.it_first_max[c]) d.it_first_max[c] = d.it_first[c];
        if (d.it_later[c] > d.it_later_max[c]) d.it_later_max[c] = d.it_later[c];
    }
}

// Clear the accumulators of every member.
__global__ void k_clear_acc(DevState* st, int batch) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= batch) return;
    DevState& d = st[m];
    d.flags_acc = 0;
    d.steps_acc = 0;
    for (int c = 0; c < kMaxCorr; ++c) {
        d.it_first_max[c] = 0;
        d.it_later_max[c] = 0;
    }
}

// Per-member affine coefficients for k_sum_affine_sq from the totals in red[]:
// mode 0: (1, -red[3]/N) (deviation from the mean of r); mode 1: (0, 0) (plain
// sums); mode 2: (1/mean, -1) with mean = red[5]/N (relative deviation).
__global__ void k_set_affine(DevState* st, int batch, int mode, double N) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= batch) return;
    double a = 0.0, b = 0.0;
    if (mode == 0) {
        a = 1.0;
        b = -st[m].red[3] / N;
    } else if (mode == 2) {
        const double mean = st[m].red[5] / N;
        a = mean != 0.0 ? 1.0 / mean : 0.0;
        b = mean != 0.0 ? -1.0 : 0.0;
    }
    st[m].aff[0] = a;
    st[m].aff[1] = b;
}

// Record a solve of corrector `corr` in every member's step record.
// add: the solve just finished counts -- its iterations are added to the
// step's total and kept as the first solve's (round <= 1: the FP64 solve or
// the first FP32 round) or as the largest later round's.  fin (1: residual
// from the last CG check, 2: from red[0] = ||r64||^2 after refinement):
// the final relative residual against the original ||b|| and the refinement
// rounds (round) are stored, and flag 1 is raised unless the residual meets
// the requested tolerance.
__global__ void k_record_solve(DevState* st, int batch, int corr, int round, int add, int fin) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= batch) return;
    DevState& d = st[m];
    if (add) {
        const int it = d.pcg.iters;
        d.it_corr[corr] += it;
        if (round <= 1) d.it_first[corr] = it;
        else if (it > d.it_later[corr]) d.it_later[corr] = it;
    }
    if (!fin) return;
    const double rr = fin == 2 ? d.red[0] : d.pcg.rr;
    d.rel_corr[corr] = d.pcg.bb > 0.0 ? sqrt(rr / d.pcg.bb) : 0.0;
    d.rounds_corr[corr] = round;
    if (!(rr <= d.pcg.tol_final * d.pcg.bb)) d.flags |= 1;
}

// Tolerance of the next FP32 refinement round of every member from red[0] =
// ||r64||^2 and the original ||b||^2 (pcg.bb): reduce the current residual
// to half the requested one, but by no less than the factor tau_min (and at
// least by 1/2).  A member already within p_tol gets skip = 1: the round's
// solve stops at k = 0 without touching x, and its refinement and the totals
// of its partials return at once (x64, xf and red[0] keep the values of the
// last round that ran).  Rounds beyond convergence occur in captured steps,
// whose round count is fixed.
__global__ void k_set_tol_refine(DevState* st, int batch, double tau_min) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= batch) return;
    DevState& d = st[m];
    const double rr = d.red[0], bb = d.pcg.bb;
    d.pcg.skip = 0;
    if (rr <= d.pcg.tol_final * bb || !(bb > 0.0)) {
        // done: the round's solve and refinement return at once
        d.pcg.tol2 = 1.0;
        d.pcg.skip = 1;
        return;
    }
    double tau = 0.5 * sqrt(d.pcg.tol_final * bb / rr);
    tau = tau < tau_min ? tau_min : (tau > 0.5 ? 0.5 : tau);
    d.pcg.tol2 = tau * tau * (rr / bb);
}

// Set the CG tolerance (squared, relative to the reference ||b||) of every member.
__global__ void k_set_tol(DevState* st, int batch, double tol2) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= batch) return;
    st[m].pcg.tol2 = tol2;
    st[m].pcg.skip = 0;
}

// Clear the step flags and the step record of every member (start of a step).
__global__ void k_clear_flags(DevState* st, int batch) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= batch) return;
    st[m].flags = 0;
    for (int c = 0; c < kMaxCorr; ++c) {
        st[m].it_corr[c] = 0;
        st[m].rel_corr[c] = 0.0;
        st[m].rounds_corr[c] = 0;
        st[m].it_first[c] = 0;
        st[m].it_later[c] = 0;
    }
}

// ------------------------------------------------------------------------
// launch wrappers
// ------------------------------------------------------------------------
Launch make_launch_shaped(int n, int batch, int bx, int cz) {
    Launch L;
    const int by = kBlock / bx;
    const int gx = (n + bx - 1) / bx, gy = (n + by - 1) / by;
    cz = cz < 1 ? 1 : (cz > n ? n : cz);
    const int nz = (n + cz - 1) / cz;
    L.block = dim3(bx, by, 1);
    L.grid = dim3(gx, gy, nz * batch);
    L.nblocks = L.grid.x * L.grid.y * L.grid.z;
    L.cz = cz;
    L.nz = nz;
    return L;
}

// ---------------------------------------------------------------- tiled
// Generic z-march over 64 x 8 column tiles (n a multiple of 64) for
// the field kernels whose cells gather 13-point crosses, for the reason of
// k_mom_sweep_tiled: each of the K::NS stencil fields is read once per cell
// from HBM; its x-y neighbours on the current plane come from a halo-2 LDS
// tile, its z neighbours from a five-plane register queue.  With K::FACES the
// three components of a face field and the low-side neighbour each needs
// (x - 1, y - 1, z - 1) come from LDS and a two-plane queue.  K supplies the
// cell's own point values (K::load, issued a plane ahead) and the arithmetic
// (K::cell: the cell function of the gathered kernel, fed the same gathered
// arrays, lines and 7-point crosses being subsets of the 13-point one).  A
// halo value is loaded together with its owner tile's queue head of the same
// plane (four planes ahead, then held in a three-plane register queue), so
// that the two reads of a line fall together in L2.  Loads past the chunk's
// last needed plane are clamped to planes already read.  The functors read
// their point values with streaming loads (stream_ld) and write their outputs
// with streaming stores (stream_st), as do the other z-marches.
template <typename T, class K>
__global__ void __launch_bounds__(kTX * kTY) k_tiled(Phys ph, DevState* st, K kern) {
    MEMBER(ph)
    constexpr int NS = K::NS;
    constexpr bool FACES = K::FACES;
    constexpr int NRA = K::NR > 0 ? K::NR : 1;
    const size_t N = ncell(ph);
    K k = kern;
    k.member(ph, st + mem_);
    if (MEMBER_FIRST()) k.lead(st + mem_);   // state a launch records even when it skips
    if (k.skip(st + mem_)) return;           // whole block, before any barrier
    const int n = ph.n, cz = ph.cz;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = tx + kTX * ty;
    const int i0 = bp_.x * kTX, j0 = bp_.y * kTY;
    const int k0 = bz_ * cz;
    const int k1 = k0 + cz < n ? k0 + cz : n;
    const size_t nn = (size_t)n * n;
    constexpr int kHalo = 4 * kTX + 4 * kTY;    // halo cells of one stencil tile
    constexpr int kJobs = NS * kHalo + (FACES ? kTY + kTX : 0);
    constexpr int kPer = (kJobs + kTX * kTY - 1) / (kTX * kTY);
    constexpr int kUW = kTX + 4, kUS = (kTY + 4) * kUW;
    constexpr int kFX = NS * kUS;
    constexpr int kFY = kFX + (FACES ? kTY * (kTX + 1) : 0);
    constexpr int kDum = kFY + (FACES ? (kTY + 1) * kTX : 0);
    // one LDS array: the stencil tiles, face x at x = i0 - 1 .. i0 + 63, face
    // y at y = j0 - 1 .. j0 + 7, a scratch slot per thread for idle halo jobs
    __shared__ T lds[kDum + kTX * kTY];
    auto U = [&](int f, int y, int x) -> T& { return lds[f * kUS + y * kUW + x]; };
    auto FX = [&](int y, int x) -> T& { return lds[kFX + y * (kTX + 1) + x]; };
    auto FY = [&](int y, int x) -> T& { return lds[kFY + y * kTX + x]; };
    auto wr = [n](int a) { return a < 0 ? a + n : (a >= n ? a - n : a); };
    auto clampk = [](int a, int hi) { return a < hi ? a : hi; };
    const size_t col = base_ + (size_t)(i0 + tx) + (size_t)n * (j0 + ty);
    typedef const T __attribute__((address_space(1)))* gptr;   // global memory
    gptr hsrc[kPer];
    size_t hoff[kPer];
    int hdst[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int jb = tid + q * kTX * kTY;
        hsrc[q] = (gptr)k.sf[0];
        hoff[q] = col;
        hdst[q] = kDum + tid;
        if (jb < NS * kHalo) {
            const int f = jb / kHalo, h = jb - f * kHalo;
#pragma unroll
            for (int g = 0; g < NS; ++g)    // a select, not a dynamic index into k.sf
                if (g == f) hsrc[q] = (gptr)k.sf[g];
            if (h < 4 * kTX) {                  // rows j0-2, j0-1, j0+8, j0+9
                const int row = h / kTX, x = h - row * kTX;
                const int yy = row < 2 ? row : kTY + row;
                hoff[q] = base_ + (size_t)(i0 + x) + (size_t)n * wr(j0 - 2 + yy);
                hdst[q] = f * kUS + yy * kUW + x + 2;
            } else {                            // columns i0-2, i0-1, i0+64, i0+65
                const int t = h - 4 * kTX, c4 = t / kTY, y = t - c4 * kTY;
                const int xx = c4 < 2 ? c4 : kTX + c4;
                hoff[q] = base_ + (size_t)wr(i0 - 2 + xx) + (size_t)n * (j0 + y);
                hdst[q] = f * kUS + (y + 2) * kUW + xx;
            }
        } else if (FACES && jb < NS * kHalo + kTY) {   // face x at x = i0 - 1
            const int y = jb - NS * kHalo;
            hsrc[q] = (gptr)k.face;
            hoff[q] = base_ + (size_t)wr(i0 - 1) + (size_t)n * (j0 + y);
            hdst[q] = kFX + y * (kTX + 1);
        } else if (FACES && jb < kJobs) {               // face y at y = j0 - 1
            const int x = jb - NS * kHalo - kTY;
            hsrc[q] = (gptr)(k.face + N);
            hoff[q] = base_ + (size_t)(i0 + x) + (size_t)n * wr(j0 - 1);
            hdst[q] = kFY + x;
        }
    }
    // halo values of planes kk .. kk + 2 (hq[.][0] goes to LDS at plane kk)
    T q5[NS][5], fzq[2] = {T(0), T(0)}, cfx = T(0), cfy = T(0), hq[kPer][3];
#pragma unroll
    for (int f = 0; f < NS; ++f)
#pragma unroll
        for (int t = 0; t < 5; ++t) q5[f][t] = k.sf[f][col + nn * wr(k0 - 2 + t)];
    if (FACES) {
        fzq[0] = k.face[2 * N + col + nn * wr(k0 - 1)];
        fzq[1] = k.face[2 * N + col + nn * k0];
        cfx = k.face[col + nn * k0];
        cfy = k.face[N + col + nn * k0];
    }
    typename K::Pts cur = k.load(col + nn * k0), nxt;
#pragma unroll
    for (int q = 0; q < kPer; ++q)
#pragma unroll
        for (int t = 0; t < 3; ++t)
            hq[q][t] = hsrc[q][nn * (size_t)wr(clampk(k0 + t, k1 - 1)) + hoff[q]];
    T nq[NS], nfz = T(0), nfx = T(0), nfy = T(0), nh[kPer];
    // queue heads at plane kq, halo values at kh, own values at kv
    auto prefetch = [&](int kq, int kh, int kv) {
        const size_t p5 = nn * (size_t)wr(kq), phh = nn * (size_t)wr(kh), pv = nn * (size_t)wr(kv);
#pragma unroll
        for (int f = 0; f < NS; ++f) nq[f] = k.sf[f][col + p5];
        if (FACES) {
            nfz = k.face[2 * N + col + pv];
            nfx = k.face[col + pv];
            nfy = k.face[N + col + pv];
        }
        nxt = k.load(col + pv);
#pragma unroll
        for (int q = 0; q < kPer; ++q) nh[q] = hsrc[q][phh + hoff[q]];
    };
    // last planes the chunk needs: queue heads k1 + 1, halo and own values k1 - 1
    prefetch(clampk(k0 + 3, k1 + 1), clampk(k0 + 3, k1 - 1), clampk(k0 + 1, k1 - 1));
    double acc[NRA];
    k.init(acc);
    for (int kk = k0; kk < k1; ++kk) {
        const size_t P = col + nn * (size_t)kk;
#pragma unroll
        for (int f = 0; f < NS; ++f) U(f, ty + 2, tx + 2) = q5[f][2];
        if (FACES) {
            FX(ty, tx + 1) = cfx;
            FY(ty + 1, tx) = cfy;
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) lds[hdst[q]] = hq[q][0];
        lds_barrier();
        T v[NS][13], fp[3], fm[3];
#pragma unroll
        for (int f = 0; f < NS; ++f) {
            v[f][0] = q5[f][2];
            v[f][1] = U(f, ty + 2, tx);
            v[f][2] = U(f, ty + 2, tx + 1);
            v[f][3] = U(f, ty + 2, tx + 3);
            v[f][4] = U(f, ty + 2, tx + 4);
            v[f][5] = U(f, ty, tx + 2);
            v[f][6] = U(f, ty + 1, tx + 2);
            v[f][7] = U(f, ty + 3, tx + 2);
            v[f][8] = U(f, ty + 4, tx + 2);
            v[f][9] = q5[f][0];
            v[f][10] = q5[f][1];
            v[f][11] = q5[f][3];
            v[f][12] = q5[f][4];
        }
        if (FACES) {
            fp[0] = FX(ty, tx + 1);
            fm[0] = FX(ty, tx);
            fp[1] = FY(ty + 1, tx);
            fm[1] = FY(ty, tx);
            fp[2] = fzq[1];
            fm[2] = fzq[0];
        }
        lds_barrier();
        k.cell(P, v, fp, fm, cur, acc);
        // advance the queues with the values loaded a plane ago, then load the
        // queue heads at kk + 4 and the values of plane kk + 2
#pragma unroll
        for (int f = 0; f < NS; ++f) {
#pragma unroll
            for (int t = 0; t < 4; ++t) q5[f][t] = q5[f][t + 1];
            q5[f][4] = nq[f];
        }
        if (FACES) {
            fzq[0] = fzq[1];
            fzq[1] = nfz;
            cfx = nfx;
            cfy = nfy;
        }
        cur = nxt;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            hq[q][0] = hq[q][1];
            hq[q][1] = hq[q][2];
            hq[q][2] = nh[q];
        }
        prefetch(clampk(kk + 4, k1 + 1), clampk(kk + 4, k1 - 1), clampk(kk + 2, k1 - 1));
    }
    if constexpr (K::NR > 0) block_partials<K::NR, K::MASK>(acc, k.part);
    if (MEMBER_FIRST()) k.first(st + mem_);
}

// The 13-point cross v of a field: the line of five cells along d (as
// gather_line) and the 7-point cross (as gather7).
template <typename T>
__device__ inline void cross_line(const T (&v)[13], int d, T (&o)[5]) {
    o[0] = v[1 + 4 * d];
    o[1] = v[2 + 4 * d];
    o[2] = v[0];
    o[3] = v[3 + 4 * d];
    o[4] = v[4 + 4 * d];
}
template <typename T, typename R>
__device__ inline void cross7(const T (&v)[13], R (&o)[7]) {
    o[0] = (R)v[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        o[1 + 2 * d] = (R)v[2 + 4 * d];
        o[2 + 2 * d] = (R)v[3 + 4 * d];
    }
}

// Cell functors of k_tiled.  Members: NS stencil fields sf, FACES and the face
// field, NR partial sums (block_partials mask MASK) into part, the member's
// constants (member), the point values (Pts, load), the arithmetic (cell),
// and what the member's first thread does at the end (first).
template <typename T>
struct TiledBase {
    static constexpr bool FACES = false;
    static constexpr int NR = 0;
    static constexpr unsigned MASK = 0u;
    const T* face = nullptr;
    double* part = nullptr;
    size_t NT = 0;
    __device__ void init(double* acc) const { acc[0] = 0.0; }
    __device__ void first(DevState*) const {}
    // true: the member has nothing to do in this launch (a solve already stopped)
    __device__ bool skip(const DevState*) const { return false; }
    // the member's first thread, before the skip test
    __device__ void lead(DevState*) const {}
};

template <typename T>
struct TiledMomSource : TiledBase<T> {
    static constexpr int NS = 1;          // div u
    const T* sf[1];
    const T *rn, *un;
    T* src;
    T dt, m3, inv_h, rref;
    // BDF2: the coefficients and the state at t^{n-1}
    const double *bc, *rm1, *um1;
    struct Pts { T rn, u[3]; };
    __device__ void member(const Phys& ph, const DevState* d) {
        this->NT = ph.NT;
        dt = (T)d->dt;
        m3 = (T)(ph.mu / 3.0);
        inv_h = (T)ph.inv_h;
        rref = (T)d->rho_ref;
        bc = ph.bdf2 ? d->bdf : nullptr;
        rm1 = ph.rm1;
        um1 = ph.um1;
    }
    __device__ Pts load(size_t P) const {
        return {stream_ld(rn + P),
                {stream_ld(un + P), stream_ld(un + this->NT + P),
                 stream_ld(un + 2 * this->NT + P)}};
    }
    __device__ void cell(size_t P, const T (&v)[1][13], const T (&)[3], const T (&)[3],
                         const Pts& p, double*) const {
        T out[3];
        const T rho = rref + p.rn;
        mom_source_cell(v[0], p.u, rho, dt, m3, inv_h, out);
        if (bc) {   // as k_mom_source
            const double rm = (double)rref + rm1[P];
#pragma unroll
            for (int m = 0; m < 3; ++m)
                out[m] = (T)((bc[1] * (double)rho * (double)p.u[m] - bc[2] * rm * um1[m * this->NT + P]) /
                             (double)dt + (double)m3 * (double)dgauss13(v[0], m, inv_h));
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) stream_st(src + (m * this->NT + P), out[m]);
    }
};

template <typename T>
struct TiledCorrFlux : TiledBase<T> {
    static constexpr int NS = 3;          // w, p0, x
    const T* sf[3];
    const T* phiH;
    T *phik, *pt;
    double* snap_x;
    T A, inv_h;
    struct Pts { T h[3]; };
    __device__ void member(const Phys& ph, const DevState*) {
        this->NT = ph.NT;
        A = (T)ph.A;
        inv_h = (T)ph.inv_h;
    }
    __device__ Pts load(size_t P) const {
        return {{stream_ld(phiH + P), stream_ld(phiH + this->NT + P),
                 stream_ld(phiH + 2 * this->NT + P)}};
    }
    __device__ void cell(size_t P, const T (&v)[3][13], const T (&)[3], const T (&)[3],
                         const Pts& p, double*) const {
        T p0n[3], xn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            p0n[d] = v[1][3 + 4 * d];   // +1 along d
            xn[d] = v[2][3 + 4 * d];
        }
        T pP, fk[3];
        corr_flux_cell(v[0], v[1][0], v[2][0], p0n, xn, p.h, A, inv_h, pP, fk);
        stream_st(pt + P, pP);
#pragma unroll
        for (int d = 0; d < 3; ++d) stream_st(phik + (d * this->NT + P), fk[d]);
        if (snap_x) snap_x[P] = (double)v[2][0];
    }
};

template <typename T, bool LAST>
struct TiledCorrUpdate : TiledBase<T> {
    static constexpr int NS = 1;          // p
    static constexpr bool FACES = true;   // phi_k
    static constexpr int NR = LAST ? 3 : 0;
    static constexpr unsigned MASK = 4u;  // column 2 is a maximum
    const T* sf[1];
    const T *rn, *hbya, *aP;
    T *rk, *u;
    T dt, inv_V, inv_h;
    double rref;
    const double *bc, *rm1;   // BDF2: the coefficients and rho at t^{n-1}
    double inv_Vd;
    struct Pts { T hb[3], rn, a; };
    __device__ void member(const Phys& ph, const DevState* d) {
        this->NT = ph.NT;
        dt = (T)d->dt;
        inv_V = (T)ph.inv_V;
        inv_h = (T)ph.inv_h;
        rref = d->rho_ref;
        bc = ph.bdf2 ? d->bdf : nullptr;
        rm1 = ph.rm1;
        inv_Vd = ph.inv_V;
    }
    __device__ void init(double* acc) const {
        acc[0] = 0.0;
        if (LAST) {
            acc[1] = 0.0;
            acc[2] = -__builtin_inf();
        }
    }
    __device__ Pts load(size_t P) const {
        return {{stream_ld(hbya + P), stream_ld(hbya + this->NT + P),
                 stream_ld(hbya + 2 * this->NT + P)},
                stream_ld(rn + P), stream_ld(aP + P)};
    }
    __device__ void cell(size_t P, const T (&v)[1][13], const T (&fp)[3], const T (&fm)[3],
                         const Pts& p, double* acc) const {
        T r, um[3];
        corr_update_cell(v[0], fp, fm, p.hb, p.rn, p.a, dt, inv_V, inv_h, r, um);
        if (bc) r = corr_rho_bdf2(fp, fm, p.rn, rm1[P], dt, inv_Vd, bc);
        stream_st(rk + P, r);
        double usq = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            stream_st(u + (m * this->NT + P), um[m]);
            usq += (double)um[m] * (double)um[m];
        }
        if (LAST) {
            acc[0] += (double)r;
            acc[1] += usq;
            const double nrho = -(rref + (double)r);
            acc[2] = nrho > acc[2] ? nrho : acc[2];
        }
    }
};

template <typename T>
struct TiledRefineFromZero : TiledBase<T> {
    static constexpr int NS = 2;          // w, d
    static constexpr int NR = 3;
    const T* sf[2];
    const double* b64;
    const T* diag;
    double* x64n;
    T *xf, *r32;
    bool store_x;
    double inv_h2;
    struct Pts { double b; T dg; };
    __device__ void member(const Phys& ph, const DevState*) { inv_h2 = ph.inv_h2; }
    __device__ void init(double* acc) const { acc[0] = acc[1] = acc[2] = 0.0; }
    __device__ Pts load(size_t P) const { return {stream_ld(b64 + P), stream_ld(diag + P)}; }
    __device__ void cell(size_t P, const T (&v)[2][13], const T (&)[3], const T (&)[3],
                         const Pts& p, double* acc) const {
        const double xv[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        T dv[7];
        cross7(v[1], dv);
        double xP, r;
        refine_cell(v[0], xv, dv, p.b, p.dg, inv_h2, xP, r);
        if (store_x) {
            stream_st(x64n + P, xP);
            stream_st(xf + P, (T)xP);
        }
        const T rT = (T)r;
        stream_st(r32 + P, rT);
        acc[0] += (double)rT * ((double)rT / (double)p.dg);
        acc[1] += r * r;
        acc[2] += r * r;
    }
    __device__ void first(DevState* d) const {
        d->pcg.it_stop = kIterInf;
        d->pcg.converged = 0;
        d->pcg.iters = 0;
    }
};

template <typename T>
struct TiledDudt : TiledBase<T> {
    static constexpr int NS = 3;          // u^{n+1}
    const T* sf[3];
    const T* un;
    T* acc_out;
    T dt, inv_h;
    const double *bc, *um1;   // BDF2: the coefficients and u at t^{n-1}
    struct Pts { T u0[3]; };
    __device__ void member(const Phys& ph, const DevState* d) {
        this->NT = ph.NT;
        dt = (T)d->dt;
        inv_h = (T)ph.inv_h;
        bc = ph.bdf2 ? d->bdf : nullptr;
        um1 = ph.um1;
    }
    __device__ Pts load(size_t P) const {
        return {{stream_ld(un + P), stream_ld(un + this->NT + P), stream_ld(un + 2 * this->NT + P)}};
    }
    __device__ void cell(size_t P, const T (&v)[3][13], const T (&)[3], const T (&)[3],
                         const Pts& p, double*) const {
        T out[3];
        if (bc) dudt_bdf2_cell(v, p.u0, um1, this->NT, P, dt, inv_h, bc, out);
        else dudt_cell(v, p.u0, dt, inv_h, out);
#pragma unroll
        for (int m = 0; m < 3; ++m) stream_st(acc_out + (m * this->NT + P), out[m]);
    }
};

template <typename T>
struct TiledDustFlux : TiledBase<T> {
    static constexpr int NS = 4;          // rho^{n+1}, a_x, a_y, a_z
    const T* sf[4];
    const T *phi, *rhoj, *rn;
    T *G, *Y;
    T A, t, rref;
    double gr[3];
    int cls;
    struct Pts { T f[3], rj, rn; };
    __device__ void member(const Phys& ph, const DevState* d) {
        this->NT = ph.NT;
        A = (T)ph.A;
        t = (T)d->tau[cls];
        rref = (T)d->rho_ref;
        gr[0] = ph.g[0];
        gr[1] = ph.g[1];
        gr[2] = ph.g[2];
    }
    __device__ Pts load(size_t P) const {
        return {{stream_ld(phi + P), stream_ld(phi + this->NT + P),
                 stream_ld(phi + 2 * this->NT + P)},
                stream_ld(rhoj + P), stream_ld(rn + P)};
    }
    __device__ void cell(size_t P, const T (&v)[4][13], const T (&)[3], const T (&)[3],
                         const Pts& p, double*) const {
        T al[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d) cross_line(v[1 + d], d, al[d]);
        T g[3], y;
        dust_flux_cell(v[0], al, p.f, p.rj, p.rn, t, rref, A, gr, g, y);
#pragma unroll
        for (int d = 0; d < 3; ++d) stream_st(G + (d * this->NT + P), g[d]);
        stream_st(Y + P, y);
    }
};

template <typename T, bool CHECK>
struct TiledDustSweep : TiledBase<T> {
    static constexpr int NS = 1;          // Y_in
    static constexpr bool FACES = true;   // G
    static constexpr int NR = CHECK ? 2 : 0;   // max(-diagonal), Courant rate, as k_dust_sweep
    static constexpr unsigned MASK = 3u;
    const T* sf[1];
    const T *rhoj, *r1;
    T* Yout;
    T dt, inv_V, rref;
    double Vc;
    const double *bc, *rjm1;   // BDF2: the coefficients and the class's rho_j at t^{n-1}
    double rrefd;
    struct Pts { T rj, r1; };
    __device__ void member(const Phys& ph, const DevState* d) {
        dt = (T)d->dt;
        inv_V = (T)ph.inv_V;
        rref = (T)d->rho_ref;
        Vc = ph.V;
        bc = ph.bdf2 ? d->bdf : nullptr;
        rjm1 = ph.rjm1;
        rrefd = d->rho_ref;
    }
    __device__ Pts load(size_t P) const { return {stream_ld(rhoj + P), stream_ld(r1 + P)}; }
    __device__ void init(double* acc) const {
        acc[0] = -__builtin_inf();
        if (CHECK) acc[1] = 0.0;
    }
    __device__ void cell(size_t P, const T (&v)[1][13], const T (&fp)[3], const T (&fm)[3],
                         const Pts& p, double* acc) const {
        T dg;
        stream_st(Yout + P, bc ? dust_sweep_bdf2_cell(v[0], fp, fm, p.rj, rjm1[P], p.r1, dt, inv_V,
                                                      rrefd, bc, dg)
                               : dust_sweep_cell(v[0], fp, fm, p.rj, p.r1, dt, inv_V, rref, dg));
        if (CHECK) {
            acc[0] = fmax(acc[0], -(double)dg);
            acc[1] = fmax(acc[1], courant_rate(fp, fm, p.r1, (double)rref, Vc));
        }
    }
};

// The face dust fluxes and the conservative finish in one pass: F_f =
// G_f I4(Y)_f on the cell's own faces and, from the low-side G and the same
// four Y cells, on its lower faces (the values k_dust_faceflux would store
// in the neighbours), then rho_j^{n+1} = rho_j^n - dt div(F) and the partial
// mass sum, as k_dust_finish.  F itself is not stored.
template <typename T>
struct TiledDustFinish : TiledBase<T> {
    static constexpr int NS = 1;          // Y
    static constexpr bool FACES = true;   // G
    static constexpr int NR = 2;          // sum rho_j, max(-rho_j), as k_dust_finish
    static constexpr unsigned MASK = 2u;
    const T* sf[1];
    const T* rhoj;
    T* rhoj1;
    T* fdo;        // two-way coupling: the dust flux F_d of the next step (as k_dust_finish)
    int first_cls;
    T dt, inv_V;
    const double *bc, *rjm1;   // BDF2: the coefficients and the class's rho_j at t^{n-1}
    struct Pts { T rj; };
    __device__ void member(const Phys& ph, const DevState* d) {
        this->NT = ph.NT;
        dt = (T)d->dt;
        inv_V = (T)ph.inv_V;
        bc = ph.bdf2 ? d->bdf : nullptr;
        rjm1 = ph.rjm1;
    }
    __device__ Pts load(size_t P) const { return {stream_ld(rhoj + P)}; }
    __device__ void init(double* acc) const {
        acc[0] = 0.0;
        acc[1] = -__builtin_inf();
    }
    __device__ void cell(size_t P, const T (&v)[1][13], const T (&fp)[3], const T (&fm)[3],
                         const Pts& p, double* acc) const {
        T dF = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) dF += fp[d] * i4g(v[0], d, 0) - fm[d] * i4g(v[0], d, -1);
        if (fdo)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                T* q = fdo + (d * this->NT + P);
                *q = (first_cls ? T(0) : *q) + fp[d] * i4g(v[0], d, 0);
            }
        const T out = bc ? dust_finish_bdf2(p.rj, rjm1[P], dt, dF, inv_V, bc) : p.rj - dt * dF * inv_V;
        stream_st(rhoj1 + P, out);
        acc[0] += (double)out;
        acc[1] = fmax(acc[1], -(double)out);
    }
};

// The corrector's flux correction and update in one pass: p = p0 + p' on the
// 13-point cross, the corrected fluxes phi = phiH - K A snGrad(p) on the
// cell's own faces (stored) and on its lower faces (from the low-side phiH
// and the same w and p cells: bitwise the values the neighbours store), then
// the update of rho_k and u as k_corr_update.  p itself is not stored.  LAST
// (the step's last corrector): the mass-budget partials and, as a fourth
// column, the Courant maxima of the new state, bitwise what k_cfl computes
// from it at the start of the next step.
template <typename T, bool LAST>
struct TiledCorrFluxUpdate : TiledBase<T> {
    static constexpr int NS = 3;          // w, p0, p'
    static constexpr bool FACES = true;   // phiH
    static constexpr int NR = LAST ? 4 : 0;
    static constexpr unsigned MASK = 4u | 8u;
    const T* sf[3];
    const T *rn, *hbya, *aP;
    T *phik, *rk, *u;
    double* snap_x;
    T A, inv_h, dt, inv_V;
    double rref, V;
    const double *bc, *rm1;   // BDF2: the coefficients and rho at t^{n-1}
    double inv_Vd;
    struct Pts { T hb[3], rn, a; };
    __device__ void member(const Phys& ph, const DevState* d) {
        this->NT = ph.NT;
        A = (T)ph.A;
        inv_h = (T)ph.inv_h;
        dt = (T)d->dt;
        inv_V = (T)ph.inv_V;
        rref = d->rho_ref;
        V = ph.V;
        bc = ph.bdf2 ? d->bdf : nullptr;
        rm1 = ph.rm1;
        inv_Vd = ph.inv_V;
    }
    __device__ void init(double* acc) const {
        acc[0] = 0.0;
        if (LAST) {
            acc[1] = 0.0;
            acc[2] = -__builtin_inf();
            acc[3] = 0.0;
        }
    }
    __device__ Pts load(size_t P) const {
        return {{stream_ld(hbya + P), stream_ld(hbya + this->NT + P),
                 stream_ld(hbya + 2 * this->NT + P)},
                stream_ld(rn + P), stream_ld(aP + P)};
    }
    __device__ void cell(size_t P, const T (&v)[3][13], const T (&hp)[3], const T (&hm)[3],
                         const Pts& p, double* acc) const {
        T pv[13];
#pragma unroll
        for (int t = 0; t < 13; ++t) pv[t] = v[1][t] + v[2][t];
        const T pP = pv[0];
        T fp[3], fm[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            fp[d] = hp[d] - i4g(v[0], d, 0) * A * (pv[3 + 4 * d] - pP) * inv_h;
            fm[d] = hm[d] - i4g(v[0], d, -1) * A * (pP - pv[2 + 4 * d]) * inv_h;
            stream_st(phik + (d * this->NT + P), fp[d]);
        }
        if (snap_x) snap_x[P] = (double)v[2][0];
        T r, um[3];
        corr_update_cell(pv, fp, fm, p.hb, p.rn, p.a, dt, inv_V, inv_h, r, um);
        if (bc) r = corr_rho_bdf2(fp, fm, p.rn, rm1[P], dt, inv_Vd, bc);
        stream_st(rk + P, r);
        double usq = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            stream_st(u + (m * this->NT + P), um[m]);
            usq += (double)um[m] * (double)um[m];
        }
        if (LAST) {
            acc[0] += (double)r;
            acc[1] += usq;
            const double nrho = -(rref + (double)r);
            acc[2] = nrho > acc[2] ? nrho : acc[2];
            const double sg = courant_rate(fp, fm, r, rref, V);
            acc[3] = sg > acc[3] ? sg : acc[3];
        }
    }
};

// The Chebyshev-preconditioned CG's two launches, as k_cheb_res and
// k_cheb_dir (the head of each, from the partial sums of the previous launch
// of nb blocks, runs in member(); its state writes in lead()).
template <typename T>
struct TiledChebRes : TiledBase<T> {
    static constexpr int NS = 4;          // r_{k-1}, q_{k-1}, diag, w
    static constexpr int NR = 2;          // (r, z), (r, r)
    const T* sf[4];
    const T* p;
    T *rout, *x, *z;
    const DevState* st0;                  // member 0's state
    const double *part_theta, *part_prev;
    unsigned nb_theta, nb;
    int k;
    double c0, c1, alpha;
    T inv_h2;
    bool stopped;
    struct Pts { T p, x; };
    __device__ void member(const Phys& ph, const DevState* d) {
        const int mem = (int)(d - st0);
        inv_h2 = (T)ph.inv_h2;
        stopped = k > d->pcg.it_stop;
        alpha = 0.0;
        if (k == 0) {
            double t[1];
            reduce_member<1, 1u>(part_theta, nb_theta, ph.batch, mem, t);
            const double a = -t[0], b = 2.0 - a, mu = (b + a) / (b - a), t2 = 2.0 * mu * mu - 1.0;
            c0 = 8.0 * mu / ((b - a) * t2);
            c1 = -8.0 / ((b - a) * (b - a) * t2);
        } else {
            c0 = d->pcg.cheb[0];
            c1 = d->pcg.cheb[1];
            double t[kChebSet];
            reduce_member<kChebSet, 0u>(part_prev, nb, ph.batch, mem, t);
            alpha = t[kChebRes] / t[kChebDir];
        }
    }
    __device__ void lead(DevState* d) const {
        if (k == 0) {
            d->pcg.cheb[0] = c0;
            d->pcg.cheb[1] = c1;
        }
    }
    __device__ bool skip(const DevState*) const { return stopped; }
    __device__ void init(double* acc) const { acc[0] = acc[1] = 0.0; }
    __device__ Pts load(size_t P) const { return {p[P], x[P]}; }
    __device__ void cell(size_t P, const T (&v)[4][13], const T (&)[3], const T (&)[3],
                         const Pts& pt, double* acc) const {
        const T al = (T)alpha;
        auto res = [&](int i) -> T { return k == 0 ? v[0][i] : v[0][i] - al * v[1][i]; };
        auto tv = [&](int d, int sgn) -> T {
            const int i = 1 + 4 * d + (sgn < 0 ? 1 : 2);   // g13 index of the +-1 neighbour
            return res(i) / v[2][i];
        };
        const T rP = res(0), tP = rP / v[2][0];
        T s = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) s += i4g(v[3], d, 0) * tv(d, 1) + i4g(v[3], d, -1) * tv(d, -1);
        const T Mt = v[2][0] * tP - s * inv_h2;
        const T zP = (T)c0 * tP + (T)c1 * Mt / v[2][0];
        if (k > 0) {
            x[P] = pt.x + al * pt.p;
            rout[P] = rP;
        }
        z[P] = zP;
        acc[0] += (double)rP * (double)zP;
        acc[1] += (double)rP * (double)rP;
    }
};

template <typename T>
struct TiledChebDir : TiledBase<T> {
    static constexpr int NS = 3;          // z_k, p_{k-1}, w
    static constexpr int NR = 1;          // (p, q)
    const T* sf[3];
    const T* diag;
    T *pout, *q;
    const DevState* st0;
    const double *part_u, *part_prev, *part_cur;
    unsigned nb_u, nb;
    int k, maxit;
    double beta, bb, rr;
    T inv_h2;
    bool stopped, stop, conv;
    struct Pts { T dg; };
    __device__ void member(const Phys& ph, const DevState* d) {
        const int mem = (int)(d - st0);
        inv_h2 = (T)ph.inv_h2;
        stopped = k > d->pcg.it_stop;
        double t[kChebSet];
        reduce_member<kChebSet, 0u>(part_cur, nb, ph.batch, mem, t);
        if (k == 0) {
            double u[3];
            reduce_member<3, 0u>(part_u, nb_u, ph.batch, mem, u);
            bb = u[2];
        } else {
            bb = d->pcg.bb;
        }
        rr = t[kChebRes + 1];
        conv = rr <= d->pcg.tol2 * bb;
        stop = conv || k >= maxit;
        beta = 0.0;
        if (k > 0 && !stop) {
            double tp[kChebSet];
            reduce_member<kChebSet, 0u>(part_prev, nb, ph.batch, mem, tp);
            beta = t[kChebRes] / tp[kChebRes];
        }
    }
    __device__ void lead(DevState* d) const {
        if (stopped) return;
        if (k == 0) d->pcg.bb = bb;
        d->pcg.rr = rr;
        d->pcg.iters = k;
        if (stop) {
            d->pcg.it_stop = k;
            d->pcg.converged = conv ? 1 : 0;
        }
    }
    __device__ bool skip(const DevState*) const { return stopped || stop; }
    __device__ Pts load(size_t P) const { return {diag[P]}; }
    __device__ void cell(size_t P, const T (&v)[3][13], const T (&)[3], const T (&)[3],
                         const Pts& pt, double* acc) const {
        const T be = (T)beta;
        auto dir = [&](int i) -> T { return k == 0 ? v[0][i] : v[0][i] + be * v[1][i]; };
        const T pP = dir(0);
        T s = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d)
            s += i4g(v[2], d, 0) * dir(1 + 4 * d + 2) + i4g(v[2], d, -1) * dir(1 + 4 * d + 1);
        const T qP = pt.dg * pP - s * inv_h2;
        pout[P] = pP;
        q[P] = qP;
        acc[0] += (double)pP * (double)qP;
    }
};

// The momentum operator of the BiCGStab predictor, as k_bicg_apply: out = A y
// for the three components, partials (w, out) and with NR = 2 (out, out);
// nothing to do once the member's solve has stopped before iteration it.
template <typename T, int NR_>
struct TiledBicgApply : TiledBase<T> {
    static constexpr int NS = 3;          // y
    static constexpr bool FACES = true;   // F, the predictor's face fluxes
    static constexpr int NR = NR_;
    const T* sf[3];
    const T *aP, *w;
    T* out;
    int it;
    double inv_V, mu_h2;
    struct Pts { T a, w[3]; };
    __device__ void member(const Phys& ph, const DevState*) {
        this->NT = ph.NT;
        inv_V = ph.inv_V;
        mu_h2 = ph.mu * ph.inv_h2;
    }
    __device__ bool skip(const DevState* d) const { return it - 1 >= d->bicg.it_stop; }
    __device__ void init(double* acc) const {
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] = 0.0;
    }
    __device__ Pts load(size_t P) const {
        return {stream_ld(aP + P),
                {stream_ld(w + P), stream_ld(w + this->NT + P), stream_ld(w + 2 * this->NT + P)}};
    }
    __device__ void cell(size_t P, const T (&v)[3][13], const T (&fp)[3], const T (&fm)[3],
                         const Pts& p, double* acc) const {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const double yP = (double)v[m][0];
            double conv = 0.0, dF = 0.0, nb = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double f1 = (double)fp[d], f0 = (double)fm[d];
                const double ym2 = (double)g13(v[m], d, -2), ym1 = (double)g13(v[m], d, -1),
                             yp1 = (double)g13(v[m], d, 1), yp2 = (double)g13(v[m], d, 2);
                conv += f1 * ((9.0 * (yP + yp1) - (ym1 + yp2)) * 0.0625) -
                        f0 * ((9.0 * (ym1 + yP) - (ym2 + yp1)) * 0.0625);
                dF += f1 - f0;
                nb += yp1 + ym1;
            }
            const double a = (double)p.a * yP + conv * inv_V - 0.5625 * dF * inv_V * yP - mu_h2 * nb;
            stream_st(out + (m * this->NT + P), (T)a);
            acc[0] += (double)p.w[m] * a;
            if (NR == 2) acc[NR - 1] += a * a;
        }
    }
};

// One Jacobi sweep of the Fourier closure's energy predictor, as
// k_energy_sweep (FP64 fields; T = double).
template <typename T>
struct TiledEnergySweep : TiledBase<T> {
    static constexpr int NS = 1;          // T^in
    static constexpr bool FACES = true;   // phi^n
    const T* sf[1];
    const double *aT, *sT;
    double* tout;
    double cv, kh2, inv_V;
    struct Pts { double a, s; };
    __device__ void member(const Phys& ph, const DevState*) {
        cv = ph.cv;
        kh2 = ph.kappa * ph.inv_h2;
        inv_V = ph.inv_V;
    }
    __device__ Pts load(size_t P) const { return {stream_ld(aT + P), stream_ld(sT + P)}; }
    __device__ void cell(size_t P, const T (&v)[1][13], const T (&fp)[3], const T (&fm)[3],
                         const Pts& p, double*) const {
        double conv = 0.0, nb = 0.0, dphi = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            conv += (double)fp[d] * i4g(v[0], d, 0) - (double)fm[d] * i4g(v[0], d, -1);
            nb += g13(v[0], d, 1) + g13(v[0], d, -1);
            dphi += (double)fp[d] - (double)fm[d];
        }
        const double off = cv * (conv * inv_V - 0.5625 * (dphi * inv_V) * v[0][0]) - kh2 * nb;
        stream_st(tout + P, (p.s - off) / p.a);
    }
};

// The predictor: dt from the Courant partials (every block reduces them, as
// k_predict), then predict_cell; the member's first thread stores dt.
template <typename T>
struct TiledPredict : TiledBase<T> {
    static constexpr int NS = 3;          // u^n
    static constexpr bool FACES = true;   // phi^n
    const T* sf[3];
    const DevState* st0;                  // member 0's state
    const double* part_cfl;
    unsigned nb_cfl;
    double dt_fixed, cfl, growth, dt_max;
    const T* rn;
    T *rs, *aP, *divu, *pn;
    double dtd, sigma, pref, gamma;
    T dt, inv_V, inv_h, diag_visc, rref;
    // variants: the ideal gas at T^n (Fourier), the BDF2 coefficients
    const double *tn, *rm1;
    double R, bc[3];
    bool fourier, bdf2;
    struct Pts { T rn; };
    __device__ void member(const Phys& ph, const DevState* d) {
        double sg[1];
        reduce_member<1, 1u>(part_cfl, nb_cfl, ph.batch, (int)(d - st0), sg);
        sigma = sg[0];
        dtd = predict_dt(sigma, d->dt_prev, dt_fixed, cfl, growth, dt_max);
        dt = (T)dtd;
        inv_V = (T)ph.inv_V;
        inv_h = (T)ph.inv_h;
        diag_visc = (T)(6.0 * ph.mu * ph.inv_h2);
        rref = (T)d->rho_ref;
        pref = d->p_ref;
        gamma = ph.gamma;
        fourier = ph.fourier;
        bdf2 = ph.bdf2;
        tn = ph.tn;
        rm1 = ph.rm1;
        R = ph.R;
        bc[0] = bc[1] = 1.0;
        bc[2] = 0.0;
        if (bdf2) bdf2_coef(dtd, d->dt_prev, bc);
    }
    __device__ Pts load(size_t P) const { return {stream_ld(rn + P)}; }
    __device__ void cell(size_t P, const T (&v)[3][13], const T (&fp)[3], const T (&fm)[3],
                         const Pts& p, double*) const {
        T ul[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d) cross_line(v[d], d, ul[d]);
        T r, a, dv, pp;
        predict_cell(fp, fm, ul, p.rn, dt, inv_V, inv_h, diag_visc, rref, pref, gamma, r, a, dv, pp);
        if (fourier) pp = (T)(((double)rref + (double)p.rn) * R * tn[P] - pref);
        if (bdf2) {   // as k_predict
            double dphi = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) dphi += (double)fp[d] - (double)fm[d];
            dphi *= (double)inv_V;
            const double rr = (bc[1] * (double)p.rn - bc[2] * rm1[P] - dtd * dphi) / bc[0];
            r = (T)rr;
            a = (T)(bc[0] * ((double)rref + rr) / dtd + 0.5625 * dphi + (double)diag_visc);
        }
        stream_st(rs + P, r);
        stream_st(aP + P, a);
        stream_st(divu + P, dv);
        stream_st(pn + P, pp);
    }
    __device__ void first(DevState* d) const {
        if (!(dtd > 0.0) || !isfinite(dtd)) d->flags |= 16;  // bad dt
        d->sigma = sigma;
        d->dt = dtd;
#pragma unroll
        for (int q = 0; q < 3; ++q) d->bdf[q] = bc[q];
    }
};

// Launch of k_tiled over the tiled launch TL; returns its block count (the
// number of partials a reducing functor writes).
template <typename T, class K>
static unsigned tiled_launch(const Launch& TL, hipStream_t s, const Phys& ph, const DevState* st,
                             const K& k) {
    Phys pt = ph;
    pt.cz = TL.cz;
    pt.nz = TL.nz;
    hipLaunchKernelGGL((k_tiled<T, K>), TL.grid, TL.block, 0, s, pt, const_cast<DevState*>(st), k);
    return TL.nblocks;
}

Launch make_launch(int n, int batch) {
    const int bx = n >= 64 ? 64 : 32;
    const int gx = (n + bx - 1) / bx, gy = (n + kBlock / bx - 1) / (kBlock / bx);
    // about kTargetBlocks blocks per member: the partials of a reduction stay
    // small enough for every block of the consuming kernel to total them
    int nz = kTargetBlocks / (gx * gy);
    nz = nz < 1 ? 1 : (nz > n ? n : nz);
    return make_launch_shaped(n, batch, bx, (n + nz - 1) / nz);
}

Launch make_tiled_launch(int n, int batch, int cz_tile) {
    Launch L{};
    if (n < 64 || n % kTX != 0 || n % kTY != 0) return L;   // nblocks = 0: not available
    const int gx = n / kTX, gy = n / kTY;
    int nz = kTiledBlocks / (gx * gy);
    nz = nz < 1 ? 1 : nz;
    int cz = (n + nz - 1) / nz;
    if (cz < 8) cz = 8;
    if (cz_tile > 0) cz = cz_tile < n ? cz_tile : n;
    nz = (n + cz - 1) / cz;
    L.block = dim3(kTX, kTY, 1);
    L.grid = dim3(gx, gy, nz * batch);
    L.nblocks = L.grid.x * L.grid.y * L.grid.z;
    L.cz = cz;
    L.nz = nz;
    return L;
}

Launch make_spmv_launch(int n, int batch, int elem_bytes, int cz_tile) {
    Launch L{};
    const int rh = row_waves(n, elem_bytes);
    if (rh) {   // full-row form
        const int gy = n / (kRowWaves / rh);
        int nz = kRowBlocks / gy;
        nz = nz < 1 ? 1 : nz;
        const int cz = (n + nz - 1) / nz;
        nz = (n + cz - 1) / cz;
        L.block = dim3(64, kRowWaves, 1);
        L.grid = dim3(1, gy, nz * batch);
        L.nblocks = L.grid.x * L.grid.y * L.grid.z;
        L.cz = cz;
        L.nz = nz;
        L.v = n / (64 * rh);
        L.h = rh;
        const double field = (double)elem_bytes * n * n * n * batch;
        L.nt = 9.0 * field > kMallBytes && 2.0 * field <= 0.6 * kMallBytes;
        return L;
    }
    const int TY = kTY * spmv_rows(elem_bytes);
    const bool wide = n >= 64 && n % kTX == 0 && n % TY == 0;
    if (!wide && n % kSmallTX != 0) return L;   // nblocks = 0: not available
    const int tx = wide ? kTX : kSmallTX, ty = wide ? TY : kSmallTX;
    const int gx = n / tx, gy = n / ty;
    int nz = kTiledBlocks / (gx * gy);
    nz = nz < 1 ? 1 : nz;
    int cz = (n + nz - 1) / nz;
    if (cz < 8) cz = 8;   // 4 or 2 planes: slower at 32^3-48^3 (z halo, launch of more blocks)
    if (cz_tile > 0) cz = cz_tile < n ? cz_tile : n;
    nz = (n + cz - 1) / cz;
    L.block = wide ? dim3(kTX, kTY, 1) : dim3(kSmallTX, kSmallTX, 1);
    L.grid = dim3(gx, gy, nz * batch);
    L.nblocks = L.grid.x * L.grid.y * L.grid.z;
    L.cz = cz;
    L.nz = nz;
    return L;
}

static dim3 lin_grid(size_t count) {
    size_t b = (count + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

#define LAUNCH(kern, L, s, ...) hipLaunchKernelGGL(kern, L.grid, L.block, 0, s, __VA_ARGS__)

void psidt_of(hipStream_t s, int n, const double* diag, const double* w, double* out) {
    const double h = 2.0 * M_PI / n;
    const size_t N = (size_t)n * n * n;
    hipLaunchKernelGGL(k_psidt_of, lin_grid(N), dim3(kBlock), 0, s, n, 1.0 / (h * h), diag, w, out);
}

template <typename T>
void Ops<T>::cast_in(hipStream_t s, const double* src, T* dst, size_t count, double shift) {
    hipLaunchKernelGGL(k_cast_in<T>, lin_grid(count), dim3(kBlock), 0, s, src, dst, count, shift);
}
template <typename T>
void Ops<T>::cast_out(hipStream_t s, const T* src, double* dst, size_t count, double shift) {
    hipLaunchKernelGGL(k_cast_out<T>, lin_grid(count), dim3(kBlock), 0, s, src, dst, count, shift);
}
template <typename T>
void Ops<T>::pressure_out(hipStream_t s, const Phys& ph, double rho_ref, double p_ref, const T* r,
                          double* dst, const double* temp) {
    hipLaunchKernelGGL(k_pressure_out<T>, lin_grid(ph.N), dim3(kBlock), 0, s, ph.gamma, rho_ref,
                       p_ref, r, dst, ph.N, temp, ph.R);
}
template <typename T>
void Ops<T>::init_phi(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                      const T* r, const T* u, T* phi) {
    LAUNCH(k_init_phi<T>, L, s, ph, st, r, u, phi);
}
template <typename T>
void Ops<T>::cfl(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st, const T* r,
                 const T* phi, double* part) {
    LAUNCH(k_cfl<T>, L, s, ph, st, r, phi, part);
}
template <typename T>
void Ops<T>::predict(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                     DevState* st, const double* part_cfl, unsigned nb_cfl, double dt_fixed,
                     double cfl, double growth, double dt_max, const T* rn, const T* un,
                     const T* phi, T* rs, T* aP, T* divu, T* pn) {
    if (TL.nblocks) {
        TiledPredict<T> k{};
        for (int d = 0; d < 3; ++d) k.sf[d] = un + d * ph.NT;
        k.face = phi;
        k.st0 = st;
        k.part_cfl = part_cfl;
        k.nb_cfl = nb_cfl;
        k.dt_fixed = dt_fixed;
        k.cfl = cfl;
        k.growth = growth;
        k.dt_max = dt_max;
        k.rn = rn;
        k.rs = rs;
        k.aP = aP;
        k.divu = divu;
        k.pn = pn;
        tiled_launch<T>(TL, s, ph, st, k);
        return;
    }
    LAUNCH(k_predict<T>, L, s, ph, st, part_cfl, nb_cfl, dt_fixed, cfl, growth, dt_max, rn, un,
           phi, rs, aP, divu, pn);
}
template <typename T>
void Ops<T>::mom_source(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                        const DevState* st, const T* rn, const T* un, const T* divu, T* src) {
    if (TL.nblocks) {
        TiledMomSource<T> k{};
        k.sf[0] = divu;
        k.rn = rn;
        k.un = un;
        k.src = src;
        tiled_launch<T>(TL, s, ph, st, k);
        return;
    }
    LAUNCH(k_mom_source<T>, L, s, ph, st, rn, un, divu, src);
}
template <typename T>
void Ops<T>::mom_sweep(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                       const DevState* st, const T* uin, T* uout, const T* phi, const T* aP,
                       const T* src, const T* pn) {
    if (TL.nblocks) {
        Phys pt = ph;
        pt.cz = TL.cz;
        pt.nz = TL.nz;
        LAUNCH((k_mom_sweep_tiled<T, false>), TL, s, pt, st, uin, uout, phi, aP, src, pn,
               (const T*)nullptr, (T*)nullptr, (T*)nullptr);
    } else {
        LAUNCH((k_mom_sweep<T, false>), L, s, ph, st, uin, uout, phi, aP, src, pn,
               (const T*)nullptr, (T*)nullptr, (T*)nullptr);
    }
}
template <typename T>
void Ops<T>::hbya(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                  const DevState* st, const T* uin, T* hb, const T* phi, const T* aP,
                  const T* src, const T* rk, T* w, T* p0) {
    if (TL.nblocks) {
        Phys pt = ph;
        pt.cz = TL.cz;
        pt.nz = TL.nz;
        LAUNCH((k_mom_sweep_tiled<T, true>), TL, s, pt, st, uin, hb, phi, aP, src,
               (const T*)nullptr, rk, w, p0);
    } else {
        LAUNCH((k_mom_sweep<T, true>), L, s, ph, st, uin, hb, phi, aP, src, (const T*)nullptr, rk,
               w, p0);
    }
}
template <typename T>
unsigned Ops<T>::corr_rhs(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                          DevState* st, const T* rn, const T* rk, const T* w, const T* hb,
                          const T* p0, T* phiH, T* r, T* diag, double* part_u, double* snap_b,
                          double* snap_diag, double* snap_p0, double* b64) {
    if (TL.nblocks) {
        Phys pt = ph;
        pt.cz = TL.cz;
        pt.nz = TL.nz;
        LAUNCH(k_corr_rhs_tiled<T>, TL, s, pt, st, rn, rk, w, hb, p0, phiH, r, diag, part_u, snap_b,
               snap_diag, snap_p0, b64);
        return TL.nblocks;
    }
    LAUNCH(k_corr_rhs<T>, L, s, ph, st, rn, rk, w, hb, p0, phiH, r, diag, part_u, snap_b,
           snap_diag, snap_p0, b64);
    return L.nblocks;
}
template <typename T>
unsigned Ops<T>::refine(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                        DevState* st, const double* x64, const T* d, double* x64n, T* xf,
                        const double* b64, const T* w, const T* diag, T* r32, double* part_u,
                        bool from_zero, bool store_x) {
    if (from_zero && TL.nblocks) {
        TiledRefineFromZero<T> k{};
        k.store_x = store_x;
        k.sf[0] = w;
        k.sf[1] = d;
        k.part = part_u;
        k.b64 = b64;
        k.diag = diag;
        k.x64n = x64n;
        k.xf = xf;
        k.r32 = r32;
        return tiled_launch<T>(TL, s, ph, st, k);
    }
    if (from_zero)
        LAUNCH((k_refine<T, true>), L, s, ph, st, x64, d, x64n, xf, b64, w, diag, r32, part_u,
               store_x ? 1 : 0);
    else
        LAUNCH((k_refine<T, false>), L, s, ph, st, x64, d, x64n, xf, b64, w, diag, r32, part_u, 1);
    return L.nblocks;
}
template <typename T, int XM>
static void spmv_launch(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                        DevState* st, int k, const CgArgs<T>& a) {
#define SPMV_ARGS st, k, a.rin, a.rout, a.diag, a.w, a.pold, a.pold2, a.pnew, a.qold, a.q, a.x, \
                  a.part_in, a.nb_in, a.part_out, a.fresh, a.maxit, a.xzero
    if (TL.nblocks && TL.v) {
        Phys pt = ph;
        pt.cz = TL.cz;
        pt.nz = TL.nz;
        if (TL.nt) {
            if (TL.v == 2 && TL.h == 1) LAUNCH((k_pcg_spmv_rows<T, 2, 1, XM, true>), TL, s, pt, SPMV_ARGS);
            else if (TL.v == 2) LAUNCH((k_pcg_spmv_rows<T, 2, 2, XM, true>), TL, s, pt, SPMV_ARGS);
            else if constexpr (sizeof(T) == 4)
                LAUNCH((k_pcg_spmv_rows<T, 4, 1, XM, true>), TL, s, pt, SPMV_ARGS);
        } else {
            if (TL.v == 2 && TL.h == 1) LAUNCH((k_pcg_spmv_rows<T, 2, 1, XM, false>), TL, s, pt, SPMV_ARGS);
            else if (TL.v == 2) LAUNCH((k_pcg_spmv_rows<T, 2, 2, XM, false>), TL, s, pt, SPMV_ARGS);
            else if constexpr (sizeof(T) == 4)
                LAUNCH((k_pcg_spmv_rows<T, 4, 1, XM, false>), TL, s, pt, SPMV_ARGS);
        }
        return;
    }
    if (TL.nblocks) {
        Phys pt = ph;
        pt.cz = TL.cz;
        pt.nz = TL.nz;
        if (TL.block.x == kSmallTX)
            LAUNCH((k_pcg_spmv_tiled<T, 1, XM, kSmallTX, kSmallTX>), TL, s, pt, SPMV_ARGS);
        else
            LAUNCH((k_pcg_spmv_tiled<T, spmv_rows(sizeof(T)), XM, kTX, kTY>), TL, s, pt, SPMV_ARGS);
    } else {
        LAUNCH((k_pcg_spmv<T, XM>), L, s, ph, SPMV_ARGS);
    }
#undef SPMV_ARGS
}
template <typename T>
void Ops<T>::pcg_iter(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                      DevState* st, int k, const CgArgs<T>& a) {
    if (k == 0)
        spmv_launch<T, 0>(L, TL, s, ph, st, k, a);
    else if (k & 1)
        spmv_launch<T, 1>(L, TL, s, ph, st, k, a);
    else
        spmv_launch<T, 2>(L, TL, s, ph, st, k, a);
}
template <typename T>
void Ops<T>::helm_apply(const Launch& L, hipStream_t s, const Phys& ph, const T* psidt, const T* w,
                        const T* x, T* y) {
    LAUNCH(k_helm_apply<T>, L, s, ph, psidt, w, x, y);
}
template <typename T>
void Ops<T>::bicg_init(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, const T* x,
                       const T* F, const T* aP, const T* src, const T* pn, T* r, T* rh, double* part) {
    LAUNCH(k_bicg_init<T>, L, s, ph, st, x, F, aP, src, pn, r, rh, part);
}
template <typename T>
void Ops<T>::bicg_iter(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                       DevState* st, int i, double tol2, int maxit, T* x, T* r, const T* rh,
                       T* const w[6], const T* F, const T* aP, double* part_res, double* part_v,
                       double* part_ts) {
    T *p = w[0], *v = w[1], *y = w[2], *sv = w[3], *z = w[4], *tv = w[5];
    // the stencil applications tiled where available (their partials then come
    // from TL.nblocks blocks)
    auto apply = [&](const T* yin, T* out, const T* wv, double* part, bool two) -> unsigned {
        if (TL.nblocks) {
            auto run = [&](auto k) {
                for (int m = 0; m < 3; ++m) k.sf[m] = yin + (size_t)m * ph.NT;
                k.face = F;
                k.aP = aP;
                k.w = wv;
                k.out = out;
                k.it = i;
                k.part = part;
                return tiled_launch<T>(TL, s, ph, st, k);
            };
            return two ? run(TiledBicgApply<T, 2>{}) : run(TiledBicgApply<T, 1>{});
        }
        LAUNCH(k_bicg_apply<T>, L, s, ph, st, i, two ? 1 : 0, yin, out, F, aP, wv, part);
        return L.nblocks;
    };
    LAUNCH(k_bicg_dir<T>, L, s, ph, st, i, tol2, maxit, r, p, v, y, aP, part_res);
    const unsigned nb_v = apply(y, v, rh, part_v, false);
    LAUNCH(k_bicg_half<T>, L, s, ph, st, i, r, v, sv, z, aP, part_v, nb_v);
    const unsigned nb_ts = apply(z, tv, sv, part_ts, true);
    LAUNCH(k_bicg_update<T>, L, s, ph, st, i, x, y, z, sv, tv, r, rh, part_ts, nb_ts, part_res);
}
template <typename T>
void Ops<T>::energy_setup(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                          const T* rn, const T* rs, const T* phi, const T* divu, const T* pn,
                          double* aT, double* sT) {
    LAUNCH(k_energy_setup<T>, L, s, ph, st, rn, rs, phi, divu, pn, aT, sT);
}
template <typename T>
void Ops<T>::energy_sweep(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                          const DevState* st, const double* tin, double* tout, const T* phi,
                          const double* aT, const double* sT) {
    if constexpr (sizeof(T) == sizeof(double)) {
        if (TL.nblocks) {
            TiledEnergySweep<T> k{};
            k.sf[0] = tin;
            k.face = phi;
            k.aT = aT;
            k.sT = sT;
            k.tout = tout;
            tiled_launch<T>(TL, s, ph, st, k);
            return;
        }
    }
    LAUNCH(k_energy_sweep<T>, L, s, ph, st, tin, tout, phi, aT, sT);
}
void fill_value(hipStream_t s, double* dst, size_t count, double v) {
    hipLaunchKernelGGL(k_fill, lin_grid(count), dim3(kBlock), 0, s, dst, count, v);
}
template <typename T>
void Ops<T>::cheb_theta(const Launch& L, hipStream_t s, const Phys& ph, const T* psidt, const T* diag,
                        double* part) {
    LAUNCH(k_cheb_theta<T>, L, s, ph, psidt, diag, part);
}
template <typename T>
void Ops<T>::cheb_res(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph, DevState* st,
                      int k, const T* rin, T* rout, const T* q, const T* p, const T* diag, const T* w,
                      T* x, T* z, const double* part_theta, unsigned nb_theta,
                      const double* part_prev, double* part_out) {
    if (TL.nblocks) {
        TiledChebRes<T> kr{};
        kr.sf[0] = rin;
        kr.sf[1] = k == 0 ? rin : q;   // q_{k-1} is not read at k = 0
        kr.sf[2] = diag;
        kr.sf[3] = w;
        kr.p = p;
        kr.rout = rout;
        kr.x = x;
        kr.z = z;
        kr.st0 = st;
        kr.part_theta = part_theta;
        kr.nb_theta = nb_theta;
        kr.part_prev = part_prev;
        kr.nb = TL.nblocks;
        kr.k = k;
        kr.part = part_out + kChebRes * (size_t)TL.nblocks;
        tiled_launch<T>(TL, s, ph, st, kr);
        return;
    }
    LAUNCH(k_cheb_res<T>, L, s, ph, st, k, rin, rout, q, p, diag, w, x, z, part_theta, nb_theta,
           part_prev, part_out);
}
template <typename T>
void Ops<T>::cheb_dir(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph, DevState* st,
                      int k, const T* z, const T* pin, T* pout, T* q, const T* diag, const T* w,
                      const double* part_u, unsigned nb_u, const double* part_prev,
                      double* part_cur, int maxit) {
    if (TL.nblocks) {
        TiledChebDir<T> kd{};
        kd.sf[0] = z;
        kd.sf[1] = k == 0 ? z : pin;   // p_{k-1} is not read at k = 0
        kd.sf[2] = w;
        kd.diag = diag;
        kd.pout = pout;
        kd.q = q;
        kd.st0 = st;
        kd.part_u = part_u;
        kd.nb_u = nb_u;
        kd.part_prev = part_prev;
        kd.part_cur = part_cur;
        kd.nb = TL.nblocks;
        kd.k = k;
        kd.maxit = maxit;
        kd.part = part_cur + kChebDir * (size_t)TL.nblocks;
        tiled_launch<T>(TL, s, ph, st, kd);
        return;
    }
    LAUNCH(k_cheb_dir<T>, L, s, ph, st, k, z, pin, pout, q, diag, w, part_u, nb_u, part_prev, part_cur,
           maxit);
}
template <typename T>
void Ops<T>::helm_start(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                        const T* psidt, const T* w, const T* b, const T* x, T* r, T* diag,
                        double* part_u) {
    LAUNCH(k_helm_start<T>, L, s, ph, st, psidt, w, b, x, r, diag, part_u);
}
template <typename T>
void Ops<T>::corr_flux(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                       const DevState* st, const T* p0, const T* x, const T* w, const T* phiH,
                       T* phik, T* pt, double* snap_x) {
    if (TL.nblocks) {
        TiledCorrFlux<T> k{};
        k.sf[0] = w;
        k.sf[1] = p0;
        k.sf[2] = x;
        k.phiH = phiH;
        k.phik = phik;
        k.pt = pt;
        k.snap_x = snap_x;
        tiled_launch<T>(TL, s, ph, st, k);
        return;
    }
    LAUNCH(k_corr_flux<T>, L, s, ph, p0, x, w, phiH, phik, pt, snap_x);
}
template <typename T, bool LAST>
static unsigned corr_update_tiled(const Launch& TL, hipStream_t s, const Phys& ph,
                                  const DevState* st, const T* rn, const T* phik, const T* hb,
                                  const T* pt, const T* aP, T* rk, T* u, double* part_mass) {
    TiledCorrUpdate<T, LAST> k{};
    k.sf[0] = pt;
    k.face = phik;
    k.part = part_mass;
    k.rn = rn;
    k.hbya = hb;
    k.aP = aP;
    k.rk = rk;
    k.u = u;
    return tiled_launch<T>(TL, s, ph, st, k);
}
template <typename T>
unsigned Ops<T>::corr_update(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                             const DevState* st, bool last, const T* rn, const T* phik,
                             const T* hb, const T* pt, const T* aP, T* rk, T* u,
                             double* part_mass) {
    if (TL.nblocks)
        return last ? corr_update_tiled<T, true>(TL, s, ph, st, rn, phik, hb, pt, aP, rk, u, part_mass)
                    : corr_update_tiled<T, false>(TL, s, ph, st, rn, phik, hb, pt, aP, rk, u,
                                                  part_mass);
    if (last)
        LAUNCH((k_corr_update<T, true>), L, s, ph, st, rn, phik, hb, pt, aP, rk, u, part_mass);
    else
        LAUNCH((k_corr_update<T, false>), L, s, ph, st, rn, phik, hb, pt, aP, rk, u, part_mass);
    return L.nblocks;
}
template <typename T>
void Ops<T>::dudt(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                  const DevState* st, const T* un, const T* u1, T* acc) {
    if (TL.nblocks) {
        TiledDudt<T> k{};
        for (int m = 0; m < 3; ++m) k.sf[m] = u1 + (size_t)m * ph.NT;
        k.un = un;
        k.acc_out = acc;
        tiled_launch<T>(TL, s, ph, st, k);
        return;
    }
    LAUNCH(k_dudt<T>, L, s, ph, st, un, u1, acc);
}
template <typename T>
void Ops<T>::dust_flux(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                       const DevState* st, int cls, const T* phi, const T* r1, const T* acc, T* G,
                       const T* rhoj, const T* rn, T* Y) {
    if (TL.nblocks) {
        TiledDustFlux<T> k{};
        k.sf[0] = r1;
        for (int d = 0; d < 3; ++d) k.sf[1 + d] = acc + (size_t)d * ph.NT;
        k.phi = phi;
        k.rhoj = rhoj;
        k.rn = rn;
        k.G = G;
        k.Y = Y;
        k.cls = cls;
        tiled_launch<T>(TL, s, ph, st, k);
        return;
    }
    LAUNCH(k_dust_flux<T>, L, s, ph, st, cls, phi, r1, acc, G, rhoj, rn, Y);
}
template <typename T, bool CHECK>
static unsigned dust_sweep_tiled(const Launch& TL, hipStream_t s, const Phys& ph,
                                 const DevState* st, const T* Yin, T* Yout, const T* G,
                                 const T* rhoj, const T* r1, double* part_diag) {
    TiledDustSweep<T, CHECK> k{};
    k.sf[0] = Yin;
    k.face = G;
    k.rhoj = rhoj;
    k.r1 = r1;
    k.Yout = Yout;
    k.part = part_diag;
    return tiled_launch<T>(TL, s, ph, st, k);
}
template <typename T>
unsigned Ops<T>::dust_sweep(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                            const DevState* st, const T* Yin, T* Yout, const T* G, const T* rhoj,
                            const T* r1, double* part_diag) {
    if (TL.nblocks)
        return part_diag ? dust_sweep_tiled<T, true>(TL, s, ph, st, Yin, Yout, G, rhoj, r1, part_diag)
                         : dust_sweep_tiled<T, false>(TL, s, ph, st, Yin, Yout, G, rhoj, r1, nullptr);
    if (part_diag) LAUNCH((k_dust_sweep<T, true>), L, s, ph, st, Yin, Yout, G, rhoj, r1, part_diag);
    else LAUNCH((k_dust_sweep<T, false>), L, s, ph, st, Yin, Yout, G, rhoj, r1, nullptr);
    return L.nblocks;
}
template <typename T>
void Ops<T>::dust_faceflux(const Launch& L, hipStream_t s, const Phys& ph, const T* Y, T* G) {
    LAUNCH(k_dust_faceflux<T>, L, s, ph, Y, G);
}
template <typename T>
void Ops<T>::dust_finish(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                         const T* rhoj, const T* F, T* rhoj1, double* part, T* fdo, bool first) {
    LAUNCH(k_dust_finish<T>, L, s, ph, st, rhoj, F, rhoj1, part, fdo, first ? 1 : 0);
}
template <typename T>
void Ops<T>::init_fd(const Launch& L, hipStream_t s, const Phys& ph, int ncls, const T* rhoj,
                     const T* u, T* fd) {
    LAUNCH(k_init_fd<T>, L, s, ph, ncls, rhoj, u, fd);
}
template <typename T>
void Ops<T>::mixture(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st, int ncls,
                     const T* rn, const T* un, const T* rhoj, const T* phi, const T* fd, T* fm,
                     T* aP, T* src) {
    LAUNCH(k_mixture<T>, L, s, ph, st, ncls, rn, un, rhoj, phi, fd, fm, aP, src);
}
template <typename T, bool LAST>
static unsigned corr_finish_tiled(const Launch& TL, hipStream_t s, const Phys& ph,
                                  const DevState* st, const T* p0, const T* x, const T* w,
                                  const T* phiH, T* phik, double* snap_x, const T* rn,
                                  const T* hb, const T* aP, T* rk, T* u, double* part_mass) {
    TiledCorrFluxUpdate<T, LAST> k{};
    k.sf[0] = w;
    k.sf[1] = p0;
    k.sf[2] = x;
    k.face = phiH;
    k.part = part_mass;
    k.rn = rn;
    k.hbya = hb;
    k.aP = aP;
    k.phik = phik;
    k.rk = rk;
    k.u = u;
    k.snap_x = snap_x;
    return tiled_launch<T>(TL, s, ph, st, k);
}
template <typename T>
unsigned Ops<T>::corr_finish_fused(const Launch& TL, hipStream_t s, const Phys& ph,
                                   const DevState* st, bool last, const T* p0, const T* x,
                                   const T* w, const T* phiH, T* phik, double* snap_x,
                                   const T* rn, const T* hb, const T* aP, T* rk, T* u,
                                   double* part_mass) {
    return last ? corr_finish_tiled<T, true>(TL, s, ph, st, p0, x, w, phiH, phik, snap_x, rn, hb,
                                             aP, rk, u, part_mass)
                : corr_finish_tiled<T, false>(TL, s, ph, st, p0, x, w, phiH, phik, snap_x, rn, hb,
                                              aP, rk, u, part_mass);
}
template <typename T>
unsigned Ops<T>::dust_finish_fused(const Launch& TL, hipStream_t s, const Phys& ph,
                                   const DevState* st, const T* Y, const T* G, const T* rhoj,
                                   T* rhoj1, double* part, T* fdo, bool first) {
    TiledDustFinish<T> k{};
    k.sf[0] = Y;
    k.face = G;
    k.part = part;
    k.rhoj = rhoj;
    k.rhoj1 = rhoj1;
    k.fdo = fdo;
    k.first_cls = first ? 1 : 0;
    return tiled_launch<T>(TL, s, ph, st, k);
}
template <typename T>
void Ops<T>::stats_gas(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                       const T* r, const T* u, double* part) {
    LAUNCH(k_stats_gas<T>, L, s, ph, st, r, u, part);
}
template <typename T>
void Ops<T>::sum_affine_sq(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                           const T* x, double a, double b, double* part) {
    LAUNCH(k_sum_affine_sq<T>, L, s, ph, st, x, a, b, part);
}

void finalize_sums(hipStream_t s, const double* part, unsigned nbt, int batch, int nv,
                   DevState* st, int off, bool honor_skip) {
    hipLaunchKernelGGL(k_finalize_sums, dim3(batch), dim3(64, 4), 0, s, part, nbt, batch, nv, st,
                       off, honor_skip ? 1 : 0);
}
void sum_partials(hipStream_t s, const double* part, unsigned nb, double* dst) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64, 4), 0, s, part, nb, dst);
}
void step_finish(hipStream_t s, const Phys& ph, DevState* st, const double* part_mass,
                 unsigned nb_mass, const double* part_dust, int ncls, unsigned nb_dust,
                 const double* part_diag, unsigned nb_diag, size_t cls_stride) {
    hipLaunchKernelGGL(k_step_finish, dim3(ph.batch), dim3(64, 4), 0, s, ph, st, part_mass,
                       nb_mass, part_dust, ncls, nb_dust, part_diag, nb_diag, cls_stride);
}
void commit(hipStream_t s, DevState* st, int batch) {
    hipLaunchKernelGGL(k_commit, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch);
}
void clear_acc(hipStream_t s, DevState* st, int batch) {
    hipLaunchKernelGGL(k_clear_acc, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch);
}
void set_tol_refine(hipStream_t s, DevState* st, int batch, double tau_min) {
    hipLaunchKernelGGL(k_set_tol_refine, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch,
                       tau_min);
}
void set_tol(hipStream_t s, DevState* st, int batch, double tol2) {
    hipLaunchKernelGGL(k_set_tol, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch, tol2);
}
void set_affine(hipStream_t s, DevState* st, int batch, int mode, double N) {
    hipLaunchKernelGGL(k_set_affine, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch, mode, N);
}
void record_solve(hipStream_t s, DevState* st, int batch, int corr, int round, int add, int fin) {
    hipLaunchKernelGGL(k_record_solve, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch, corr,
                       round, add, fin);
}
void clear_flags(hipStream_t s, DevState* st, int batch) {
    hipLaunchKernelGGL(k_clear_flags, dim3((batch + 63) / 64), dim3(64), 0, s, st, batch);
}

template <typename T>
void Ops<T>::net_stats(const Launch& L, hipStream_t s, const Phys& ph, const T* b, const T* diag,
                       const T* p0, double* part) {
    LAUNCH(k_net_stats<T>, L, s, ph, b, diag, p0, part);
}
template <typename T>
void Ops<T>::net_input(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                       const double* part, const T* b, const T* diag, const T* p0, uint16_t* x4,
                       float* x2, const T* psol, float* tgt) {
    LAUNCH(k_net_input<T>, L, s, ph, st, part, L.nblocks, b, diag, p0, x4, x2, psol, tgt);
}
template <typename T>
void Ops<T>::guess_start(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                         const float* y, const T* gd, const T* w, const T* diag, const T* b,
                         const double* b64, T* g, T* mg, double* part) {
    LAUNCH(k_guess_start<T>, L, s, ph, st, y, gd, w, diag, b, b64, g, mg, part);
}
template <typename T>
void Ops<T>::guess_apply(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                         const double* part_g, const T* g, const T* mg, const T* diag, T* r, T* x,
                         double* x64, const double* b64, T* bsave, double* part_u) {
    LAUNCH(k_guess_apply<T>, L, s, ph, st, part_g, L.nblocks, g, mg, diag, r, x, x64, b64, bsave,
           part_u);
}
template <typename T>
void Ops<T>::guess_revert(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, T* r,
                          T* x, double* x64, const double* b64, const T* bsave, const T* diag,
                          double* part_u) {
    LAUNCH(k_guess_revert<T>, L, s, ph, st, r, x, x64, b64, bsave, diag, part_u);
}

template struct Ops<double>;
template struct Ops<float>;

}  // namespace pisoc
