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

#define FOR_CELLS(ph)                                                        \
    const int ci_ = blockIdx.x * blockDim.x + threadIdx.x;                   \
    const int cj_ = blockIdx.y * blockDim.y + threadIdx.y;                   \
    for (int zz_ = 0; zz_ < (ph).cz; ++zz_) {                                \
        const int ck_ = blockIdx.z * (ph).cz + zz_;                          \
        if (ci_ >= (ph).n || cj_ >= (ph).n || ck_ >= (ph).n) continue;       \
        const CellIdx c{(ph).n, ci_, cj_, ck_};                              \
        const size_t P = c.self();
#define END_CELLS }

__host__ __device__ static inline size_t ncell(const Phys& ph) { return (size_t)ph.n * ph.n * ph.n; }

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

// p = p_ref + p_dev(r) as FP64
template <typename T>
__global__ void k_pressure_out(Phys ph, const T* __restrict__ r, double* __restrict__ dst,
                               size_t count) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) dst[i] = ph.p_ref + pdev((double)r[i], ph);
}

// Initial face mass fluxes phi_d = I4(rho) I4(u_d) A.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_init_phi(Phys ph, const T* __restrict__ r,
                                                     const T* __restrict__ u, T* __restrict__ phi) {
    const size_t N = ncell(ph);
    const T rref = (T)ph.rho_ref, A = (T)ph.A;
    FOR_CELLS(ph)
#pragma unroll
    for (int d = 0; d < 3; ++d)
        phi[d * N + P] = (rref + i4(r, c, d, 0)) * i4(u + d * N, c, d, 0) * A;
    END_CELLS
}

// ---------------------------------------------------------------- time step
// Convective Courant rate sigma = max_P sum_f |phi_f| / (2 rho_P V) and the
// adaptive dt = min(cfl / sigma, growth * dt_prev, dt_max) (or dt_fixed).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cfl(Phys ph, DevState* st, const T* __restrict__ r,
                                                const T* __restrict__ phi, double* partials,
                                                double dt_fixed, double cfl, double growth,
                                                double dt_prev, double dt_max) {
    const size_t N = ncell(ph);
    double v[1] = {0.0};
    FOR_CELLS(ph)
    double f = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        f += fabs((double)phi[d * N + P]) + fabs((double)phi[d * N + c.sh(d, -1)]);
    double s = f / (2.0 * (ph.rho_ref + (double)r[P]) * ph.V);
    v[0] = s > v[0] ? s : v[0];
    END_CELLS
    if (grid_reduce<1, 1u>(v, partials, &st->counter[0]) && flat_tid() == 0) {
        double sigma = v[0];
        double dt;
        if (dt_fixed > 0.0) {
            dt = dt_fixed;
        } else {
            dt = sigma > 0.0 ? cfl / sigma : __builtin_inf();
            if (growth * dt_prev < dt) dt = growth * dt_prev;
            if (dt_max > 0.0 && dt_max < dt) dt = dt_max;
        }
        if (!(dt > 0.0) || !isfinite(dt)) st->flags |= 16;  // bad dt
        st->sigma = sigma;
        st->dt = dt;
    }
}

// Density predictor rho* = rho^n - dt div(phi^n); momentum diagonal
// a_P = rho*/dt + (9/16) div(phi^n) + 6 mu / h^2; div u^n (Gauss-I4); p(rho^n).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_predict(Phys ph, const DevState* st,
                                                    const T* __restrict__ rn, const T* __restrict__ un,
                                                    const T* __restrict__ phi, T* __restrict__ rs,
                                                    T* __restrict__ aP, T* __restrict__ divu,
                                                    T* __restrict__ pn) {
    const size_t N = ncell(ph);
    const T dt = (T)st->dt;
    const T inv_V = (T)ph.inv_V, inv_h = (T)ph.inv_h;
    const T diag_visc = (T)(6.0 * ph.mu * ph.inv_h2);
    FOR_CELLS(ph)
    T dphi = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) dphi += phi[d * N + P] - phi[d * N + c.sh(d, -1)];
    dphi *= inv_V;
    T r = rn[P] - dt * dphi;
    rs[P] = r;
    aP[P] = ((T)ph.rho_ref + r) / dt + T(0.5625) * dphi + diag_visc;
    T du = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) du += i4(un + d * N, c, d, 0) - i4(un + d * N, c, d, -1);
    divu[P] = du * inv_h;
    pn[P] = pdev(rn[P], ph);
    END_CELLS
}

// Explicit momentum source s = rho^n u^n / dt + (mu/3) grad(div u^n).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_mom_source(Phys ph, const DevState* st,
                                                       const T* __restrict__ rn,
                                                       const T* __restrict__ un,
                                                       const T* __restrict__ divu,
                                                       T* __restrict__ s) {
    const size_t N = ncell(ph);
    const T dt = (T)st->dt;
    const T m3 = (T)(ph.mu / 3.0), inv_h = (T)ph.inv_h;
    FOR_CELLS(ph)
    const T rho = (T)ph.rho_ref + rn[P];
#pragma unroll
    for (int m = 0; m < 3; ++m) s[m * N + P] = rho * un[m * N + P] / dt + m3 * dgauss(divu, c, m, inv_h);
    END_CELLS
}

// One Jacobi sweep of the momentum predictor,
//   u_out = (s - N(u_in) - grad p^n) / a_P        (HBYA = false), or
// the corrector's HbyA = (s - N(u_in)) / a_P     (HBYA = true), which also
// stores w = rho_k / a_P and p_dev(rho_k) of the current density iterate.
// N(u) = (1/V) sum_f phi_f^out I4(u)_f - (9/16) div(phi) u_P - mu sum_nb u_nb / h^2.
template <typename T, bool HBYA>
__global__ void __launch_bounds__(kBlock) k_mom_sweep(Phys ph, const T* __restrict__ uin,
                                                      T* __restrict__ uout, const T* __restrict__ phi,
                                                      const T* __restrict__ aP, const T* __restrict__ s,
                                                      const T* __restrict__ pn, const T* __restrict__ rk,
                                                      T* __restrict__ w, T* __restrict__ p0) {
    const size_t N = ncell(ph);
    const T inv_V = (T)ph.inv_V, inv_h = (T)ph.inv_h;
    const T mu_h2 = (T)(ph.mu * ph.inv_h2);
    FOR_CELLS(ph)
    T fp[3], fm[3];
    T dphi = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        fp[d] = phi[d * N + P];
        fm[d] = phi[d * N + c.sh(d, -1)];
        dphi += fp[d] - fm[d];
    }
    dphi *= inv_V;
    const T a = aP[P];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const T* q = uin + m * N;
        T conv = T(0), nb = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            conv += fp[d] * i4(q, c, d, 0) - fm[d] * i4(q, c, d, -1);
            nb += q[c.sh(d, 1)] + q[c.sh(d, -1)];
        }
        T off = conv * inv_V - T(0.5625) * dphi * q[P] - mu_h2 * nb;
        T rhs = s[m * N + P] - off;
        if (!HBYA) rhs -= dgauss(pn, c, m, inv_h);
        uout[m * N + P] = rhs / a;
    }
    if (HBYA) {
        w[P] = ((T)ph.rho_ref + rk[P]) / a;
        p0[P] = pdev(rk[P], ph);
    }
    END_CELLS
}

// Corrector set-up: predicted fluxes phiH = I4(rho_k) I4(HbyA_d) A on the
// cell's own faces, and the pressure system M p' = b with
//   b = -[(rho_k - rho^n)/dt + div(phiH - K A snGrad p0)],  K = I4(w),
//   diag(M) = psi/dt + sum K / h^2,  psi = rho/(gamma p) = 1/(gamma C rho^(gamma-1)).
// Starts CG from x = 0: r = b, partial sums of b.b and b.(b/diag).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_corr_rhs(
    Phys ph, DevState* st, const T* __restrict__ rn, const T* __restrict__ rk,
    const T* __restrict__ w, const T* __restrict__ hbya, const T* __restrict__ p0,
    T* __restrict__ phiH, T* __restrict__ rvec, T* __restrict__ x, T* __restrict__ diag,
    double* partials, double* snap_b, double* snap_diag, double* snap_p0) {
    const size_t N = ncell(ph);
    const T dt = (T)st->dt;
    const T A = (T)ph.A, inv_V = (T)ph.inv_V, inv_h = (T)ph.inv_h, inv_h2 = (T)ph.inv_h2;
    const T rref = (T)ph.rho_ref;
    double v[2] = {0.0, 0.0};
    FOR_CELLS(ph)
    T divF = T(0), sumK = T(0);
    const T p0P = p0[P];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int s = -1; s <= 0; ++s) {
            const T Kf = i4(w, c, d, s);
            const T ph_f = (rref + i4(rk, c, d, s)) * i4(hbya + d * N, c, d, s) * A;
            const T sn = (s == 0 ? (p0[c.sh(d, 1)] - p0P) : (p0P - p0[c.sh(d, -1)])) * inv_h;
            const T F = ph_f - Kf * A * sn;
            divF += s == 0 ? F : -F;
            sumK += Kf;
            if (s == 0) phiH[d * N + P] = ph_f;
        }
    }
    const T b = -((rk[P] - rn[P]) / dt + divF * inv_V);
    const T rho = rref + rk[P];
    const T psidt = rho / ((T)ph.gamma * ((T)ph.p_ref + p0P)) / dt;
    const T dg = psidt + sumK * inv_h2;
    rvec[P] = b;
    x[P] = T(0);
    diag[P] = dg;
    v[0] += (double)b * (double)b;
    v[1] += (double)b * ((double)b / (double)dg);
    if (snap_b) {
        snap_b[P] = (double)b;
        snap_diag[P] = (double)dg;
        snap_p0[P] = ph.p_ref + (double)p0P;
    }
    END_CELLS
    if (grid_reduce<2, 0u>(v, partials, &st->counter[0]) && flat_tid() == 0) {
        PcgState& g = st->pcg;
        g.bb = v[0];
        g.rr = v[0];
        g.rz = v[1];
        g.iters = 0;
        g.converged = v[0] <= g.tol2 * v[0] ? 1 : 0;
        g.it_stop = g.converged ? 0 : kIterInf;
    }
}

// ---------------------------------------------------------------- CG
// Iteration k, first half: direction p_k = z_k + beta_{k-1} p_{k-1} with
// z = r / diag (recomputed on the stencil, not stored), q = M p_k with the
// face coefficients K = I4(w) formed on the fly, partial sums of p_k.q, and
// alpha_k = r.z / p.q in the last block.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pcg_spmv(Phys ph, DevState* st, int k,
                                                     const T* __restrict__ r, const T* __restrict__ diag,
                                                     const T* __restrict__ w, const T* __restrict__ pold,
                                                     T* __restrict__ pnew, T* __restrict__ q,
                                                     double* partials) {
    if (k >= st->pcg.it_stop) return;
    const T beta = k == 0 ? T(0) : (T)st->pcg.beta;
    const bool first = k == 0;
    const T inv_h2 = (T)ph.inv_h2;
    double v[1] = {0.0};
    FOR_CELLS(ph)
    auto dir = [&](size_t Q) -> T {
        T z = r[Q] / diag[Q];
        return first ? z : z + beta * pold[Q];
    };
    const T pP = dir(P);
    T off = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        off += i4(w, c, d, 0) * dir(c.sh(d, 1));
        off += i4(w, c, d, -1) * dir(c.sh(d, -1));
    }
    const T qP = diag[P] * pP - off * inv_h2;
    pnew[P] = pP;
    q[P] = qP;
    v[0] += (double)pP * (double)qP;
    END_CELLS
    if (grid_reduce<1, 0u>(v, partials, &st->counter[0]) && flat_tid() == 0)
        st->pcg.alpha = st->pcg.rz / v[0];
}

// Iteration k, second half: x += alpha p, r -= alpha q, partial sums of
// r.(r/diag) and r.r; the last block forms beta_k and tests
// ||r||^2 <= tol^2 ||b||^2 (or k + 1 = maxit), which stops later launches.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pcg_update(Phys ph, DevState* st, int k,
                                                       T* __restrict__ r, const T* __restrict__ q,
                                                       const T* __restrict__ diag, T* __restrict__ x,
                                                       const T* __restrict__ p, double* partials) {
    if (k >= st->pcg.it_stop) return;
    const T alpha = (T)st->pcg.alpha;
    double v[2] = {0.0, 0.0};
    FOR_CELLS(ph)
    x[P] += alpha * p[P];
    const T rn = r[P] - alpha * q[P];
    r[P] = rn;
    v[0] += (double)rn * ((double)rn / (double)diag[P]);
    v[1] += (double)rn * (double)rn;
    END_CELLS
    if (grid_reduce<2, 0u>(v, partials, &st->counter[0]) && flat_tid() == 0) {
        PcgState& g = st->pcg;
        g.beta = v[0] / g.rz;
        g.rz = v[0];
        g.rr = v[1];
        g.iters = k + 1;
        if (v[1] <= g.tol2 * g.bb) {
            g.converged = 1;
            g.it_stop = k + 1;
        } else if (k + 1 >= g.maxit) {
            g.it_stop = k + 1;
        }
    }
}

// y = M x for the stand-alone operator entry point (psi/dt given as a field).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_helm_apply(Phys ph, const T* __restrict__ psidt,
                                                       const T* __restrict__ w, const T* __restrict__ x,
                                                       T* __restrict__ y) {
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
                                                       T* __restrict__ diag, double* partials) {
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
    v[0] += (double)b[P] * (double)b[P];
    v[1] += (double)rr * ((double)rr / (double)dg);
    v[2] += (double)rr * (double)rr;
    END_CELLS
    if (grid_reduce<3, 0u>(v, partials, &st->counter[0]) && flat_tid() == 0) {
        PcgState& g = st->pcg;
        g.bb = v[0];
        g.rz = v[1];
        g.rr = v[2];
        g.iters = 0;
        g.converged = v[2] <= g.tol2 * v[0] ? 1 : 0;
        g.it_stop = g.converged ? 0 : kIterInf;
    }
}

// ---------------------------------------------------------------- correction
// p = p0 + p'; corrected face fluxes phi = phiH - K A snGrad(p) on own faces.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_corr_flux(Phys ph, const T* __restrict__ p0,
                                                      const T* __restrict__ x, const T* __restrict__ w,
                                                      const T* __restrict__ phiH, T* __restrict__ phik,
                                                      T* __restrict__ pt, double* snap_x) {
    const size_t N = ncell(ph);
    const T A = (T)ph.A, inv_h = (T)ph.inv_h;
    FOR_CELLS(ph)
    const T pP = p0[P] + x[P];
    pt[P] = pP;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const size_t Q = c.sh(d, 1);
        const T pQ = p0[Q] + x[Q];
        phik[d * N + P] = phiH[d * N + P] - i4(w, c, d, 0) * A * (pQ - pP) * inv_h;
    }
    if (snap_x) snap_x[P] = (double)x[P];
    END_CELLS
}

// Conservative density rho_k = rho^n - dt div(phi) and velocity
// u = HbyA - grad(p)/a_P.  On the last corrector, partial sums for the mass
// budget and the divergence checks (sum r, sum |u|^2, max(-rho)).
template <typename T, bool LAST>
__global__ void __launch_bounds__(kBlock) k_corr_update(Phys ph, DevState* st,
                                                        const T* __restrict__ rn,
                                                        const T* __restrict__ phik,
                                                        const T* __restrict__ hbya,
                                                        const T* __restrict__ pt,
                                                        const T* __restrict__ aP, T* __restrict__ rk,
                                                        T* __restrict__ u, double* partials) {
    const size_t N = ncell(ph);
    const T dt = (T)st->dt;
    const T inv_V = (T)ph.inv_V, inv_h = (T)ph.inv_h;
    double v[3] = {0.0, 0.0, -__builtin_inf()};
    FOR_CELLS(ph)
    T dphi = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) dphi += phik[d * N + P] - phik[d * N + c.sh(d, -1)];
    const T r = rn[P] - dt * dphi * inv_V;
    rk[P] = r;
    const T a = aP[P];
    double usq = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const T um = hbya[m * N + P] - dgauss(pt, c, m, inv_h) / a;
        u[m * N + P] = um;
        usq += (double)um * (double)um;
    }
    if (LAST) {
        v[0] += (double)r;
        v[1] += usq;
        double nrho = -(ph.rho_ref + (double)r);
        v[2] = nrho > v[2] ? nrho : v[2];
    }
    END_CELLS
    if (LAST) {
        if (grid_reduce<3, 4u>(v, partials, &st->counter[0]) && flat_tid() == 0) {
            st->mass_gas = (ph.rho_ref * (double)ncell(ph) + v[0]) * ph.V;
            st->usq = v[1];
            st->rho_min = -v[2];
            if (!isfinite(v[0]) || !isfinite(v[1])) st->flags |= 2;
            if (!(-v[2] > 0.0)) st->flags |= 4;
        }
    }
}

// ---------------------------------------------------------------- dust
// Particle-velocity correction source a = Du/Dt = (u^{n+1} - u^n)/dt + (u^{n+1}.grad)u^{n+1}.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dudt(Phys ph, const DevState* st,
                                                 const T* __restrict__ un, const T* __restrict__ u1,
                                                 T* __restrict__ acc) {
    const size_t N = ncell(ph);
    const T dt = (T)st->dt, inv_h = (T)ph.inv_h;
    FOR_CELLS(ph)
    const T ux = u1[P], uy = u1[N + P], uz = u1[2 * N + P];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const T* q = u1 + m * N;
        const T conv = ux * dgauss(q, c, 0, inv_h) + uy * dgauss(q, c, 1, inv_h) +
                       uz * dgauss(q, c, 2, inv_h);
        acc[m * N + P] = (q[P] - un[m * N + P]) / dt + conv;
    }
    END_CELLS
}

// Particle mass flux per unit mass ratio on own faces,
// G_d = phi_d - tau I4(rho^{n+1}) I4(a_d) A  (u_p = u - tau Du/Dt at the face),
// and the starting mass ratio Y = rho_j^n / rho^n.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dust_flux(Phys ph, double tau, const T* __restrict__ phi,
                                                      const T* __restrict__ r1, const T* __restrict__ acc,
                                                      T* __restrict__ G, const T* __restrict__ rhoj,
                                                      const T* __restrict__ rn, T* __restrict__ Y) {
    const size_t N = ncell(ph);
    const T A = (T)ph.A, t = (T)tau, rref = (T)ph.rho_ref;
    FOR_CELLS(ph)
#pragma unroll
    for (int d = 0; d < 3; ++d)
        G[d * N + P] = phi[d * N + P] - t * (rref + i4(r1, c, d, 0)) * i4(acc + d * N, c, d, 0) * A;
    Y[P] = rhoj[P] / (rref + rn[P]);
    END_CELLS
}

// One Jacobi sweep of the implicit mass-ratio equation
//   rho^{n+1} Y / dt + (1/V) sum_f G_f^out I4(Y)_f = rho_j^n / dt,
// diagonal rho^{n+1}/dt + (9/16) div G.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dust_sweep(Phys ph, const DevState* st,
                                                       const T* __restrict__ Yin, T* __restrict__ Yout,
                                                       const T* __restrict__ G, const T* __restrict__ rhoj,
                                                       const T* __restrict__ r1) {
    const size_t N = ncell(ph);
    const T dt = (T)st->dt, inv_V = (T)ph.inv_V;
    FOR_CELLS(ph)
    T conv = T(0), dG = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T gp = G[d * N + P], gm = G[d * N + c.sh(d, -1)];
        conv += gp * i4(Yin, c, d, 0) - gm * i4(Yin, c, d, -1);
        dG += gp - gm;
    }
    conv *= inv_V;
    dG *= inv_V;
    const T off = conv - T(0.5625) * dG * Yin[P];
    Yout[P] = (rhoj[P] / dt - off) / (((T)ph.rho_ref + r1[P]) / dt + T(0.5625) * dG);
    END_CELLS
}

// Face dust mass fluxes F = G I4(Y), overwriting G on own faces.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dust_faceflux(Phys ph, const T* __restrict__ Y,
                                                          T* __restrict__ G) {
    const size_t N = ncell(ph);
    FOR_CELLS(ph)
#pragma unroll
    for (int d = 0; d < 3; ++d) G[d * N + P] *= i4(Y, c, d, 0);
    END_CELLS
}

// Conservative finish rho_j^{n+1} = rho_j^n - dt div(F); partial mass sum.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dust_finish(Phys ph, DevState* st, int cls,
                                                        const T* __restrict__ rhoj,
                                                        const T* __restrict__ F, T* __restrict__ rhoj1,
                                                        double* partials) {
    const size_t N = ncell(ph);
    const T dt = (T)st->dt, inv_V = (T)ph.inv_V;
    double v[1] = {0.0};
    FOR_CELLS(ph)
    T dF = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) dF += F[d * N + P] - F[d * N + c.sh(d, -1)];
    const T out = rhoj[P] - dt * dF * inv_V;
    rhoj1[P] = out;
    v[0] += (double)out;
    END_CELLS
    if (grid_reduce<1, 0u>(v, partials, &st->counter[0]) && flat_tid() == 0)
        st->mass_p[cls] = v[0] * ph.V;
}

// ---------------------------------------------------------------- statistics
// Sums of rho|u|^2/2, |curl u|^2/2 (Gauss-I4), |u|^2 and r into st->red[0..3].
template <typename T>
__global__ void __launch_bounds__(kBlock) k_stats_gas(Phys ph, DevState* st,
                                                      const T* __restrict__ r,
                                                      const T* __restrict__ u, double* partials) {
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
    v[0] += 0.5 * (ph.rho_ref + (double)r[P]) * q;
    v[1] += 0.5 * (wx * wx + wy * wy + wz * wz);
    v[2] += q;
    v[3] += (double)r[P];
    END_CELLS
    if (grid_reduce<4, 0u>(v, partials, &st->counter[0]) && flat_tid() == 0)
        for (int i = 0; i < 4; ++i) st->red[i] = v[i];
}

// st->red[slot] = sum (a x + b)^2 and st->red[slot+1] = sum x.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sum_affine_sq(Phys ph, DevState* st,
                                                          const T* __restrict__ x, double a,
                                                          double b, int slot, double* partials) {
    double v[2] = {0.0, 0.0};
    FOR_CELLS(ph)
    const double y = a * (double)x[P] + b;
    v[0] += y * y;
    v[1] += (double)x[P];
    END_CELLS
    if (grid_reduce<2, 0u>(v, partials, &st->counter[0]) && flat_tid() == 0) {
        st->red[slot] = v[0];
        st->red[slot + 1] = v[1];
    }
}

// ------------------------------------------------------------------------
// launch wrappers
// ------------------------------------------------------------------------
Launch make_launch(int n, int cz) {
    Launch L;
    const int bx = n >= 64 ? 64 : 32;
    const int by = kBlock / bx;
    L.block = dim3(bx, by, 1);
    L.grid = dim3((n + bx - 1) / bx, (n + by - 1) / by, (n + cz - 1) / cz);
    L.nblocks = L.grid.x * L.grid.y * L.grid.z;
    L.cz = cz;
    return L;
}

static dim3 lin_grid(size_t count) {
    size_t b = (count + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

#define LAUNCH(kern, L, s, ...) hipLaunchKernelGGL(kern, L.grid, L.block, 0, s, __VA_ARGS__)

template <typename T>
void Ops<T>::cast_in(hipStream_t s, const double* src, T* dst, size_t count, double shift) {
    hipLaunchKernelGGL(k_cast_in<T>, lin_grid(count), dim3(kBlock), 0, s, src, dst, count, shift);
}
template <typename T>
void Ops<T>::cast_out(hipStream_t s, const T* src, double* dst, size_t count, double shift) {
    hipLaunchKernelGGL(k_cast_out<T>, lin_grid(count), dim3(kBlock), 0, s, src, dst, count, shift);
}
template <typename T>
void Ops<T>::pressure_out(hipStream_t s, const Phys& ph, const T* r, double* dst) {
    size_t N = ncell(ph);
    hipLaunchKernelGGL(k_pressure_out<T>, lin_grid(N), dim3(kBlock), 0, s, ph, r, dst, N);
}
template <typename T>
void Ops<T>::init_phi(const Launch& L, hipStream_t s, const Phys& ph, const T* r, const T* u, T* phi) {
    LAUNCH(k_init_phi<T>, L, s, ph, r, u, phi);
}
template <typename T>
void Ops<T>::cfl(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, const T* r,
                 const T* phi, double* partials, double dt_fixed, double cfl, double growth,
                 double dt_prev, double dt_max) {
    LAUNCH(k_cfl<T>, L, s, ph, st, r, phi, partials, dt_fixed, cfl, growth, dt_prev, dt_max);
}
template <typename T>
void Ops<T>::predict(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                     const T* rn, const T* un, const T* phi, T* rs, T* aP, T* divu, T* pn) {
    LAUNCH(k_predict<T>, L, s, ph, st, rn, un, phi, rs, aP, divu, pn);
}
template <typename T>
void Ops<T>::mom_source(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                        const T* rn, const T* un, const T* divu, T* src) {
    LAUNCH(k_mom_source<T>, L, s, ph, st, rn, un, divu, src);
}
template <typename T>
void Ops<T>::mom_sweep(const Launch& L, hipStream_t s, const Phys& ph, const T* uin, T* uout,
                       const T* phi, const T* aP, const T* src, const T* pn) {
    LAUNCH((k_mom_sweep<T, false>), L, s, ph, uin, uout, phi, aP, src, pn, (const T*)nullptr,
           (T*)nullptr, (T*)nullptr);
}
template <typename T>
void Ops<T>::hbya(const Launch& L, hipStream_t s, const Phys& ph, const T* uin, T* hb,
                  const T* phi, const T* aP, const T* src, const T* rk, T* w, T* p0) {
    LAUNCH((k_mom_sweep<T, true>), L, s, ph, uin, hb, phi, aP, src, (const T*)nullptr, rk, w, p0);
}
template <typename T>
void Ops<T>::corr_rhs(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, const T* rn,
                      const T* rk, const T* w, const T* hb, const T* p0, T* phiH, T* r, T* x,
                      T* diag, double* partials, double* snap_b, double* snap_diag,
                      double* snap_p0) {
    LAUNCH(k_corr_rhs<T>, L, s, ph, st, rn, rk, w, hb, p0, phiH, r, x, diag, partials, snap_b,
           snap_diag, snap_p0);
}
template <typename T>
void Ops<T>::pcg_spmv(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, int k,
                      const T* r, const T* diag, const T* w, const T* pold, T* pnew, T* q,
                      double* partials) {
    LAUNCH(k_pcg_spmv<T>, L, s, ph, st, k, r, diag, w, pold, pnew, q, partials);
}
template <typename T>
void Ops<T>::pcg_update(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, int k, T* r,
                        const T* q, const T* diag, T* x, const T* p, double* partials) {
    LAUNCH(k_pcg_update<T>, L, s, ph, st, k, r, q, diag, x, p, partials);
}
template <typename T>
void Ops<T>::helm_apply(const Launch& L, hipStream_t s, const Phys& ph, const T* psidt, const T* w,
                        const T* x, T* y) {
    LAUNCH(k_helm_apply<T>, L, s, ph, psidt, w, x, y);
}
template <typename T>
void Ops<T>::helm_start(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                        const T* psidt, const T* w, const T* b, const T* x, T* r, T* diag,
                        double* partials) {
    LAUNCH(k_helm_start<T>, L, s, ph, st, psidt, w, b, x, r, diag, partials);
}
template <typename T>
void Ops<T>::corr_flux(const Launch& L, hipStream_t s, const Phys& ph, const T* p0, const T* x,
                       const T* w, const T* phiH, T* phik, T* pt, double* snap_x) {
    LAUNCH(k_corr_flux<T>, L, s, ph, p0, x, w, phiH, phik, pt, snap_x);
}
template <typename T>
void Ops<T>::corr_update(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, bool last,
                         const T* rn, const T* phik, const T* hb, const T* pt, const T* aP, T* rk,
                         T* u, double* partials) {
    if (last)
        LAUNCH((k_corr_update<T, true>), L, s, ph, st, rn, phik, hb, pt, aP, rk, u, partials);
    else
        LAUNCH((k_corr_update<T, false>), L, s, ph, st, rn, phik, hb, pt, aP, rk, u, partials);
}
template <typename T>
void Ops<T>::dudt(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st, const T* un,
                  const T* u1, T* acc) {
    LAUNCH(k_dudt<T>, L, s, ph, st, un, u1, acc);
}
template <typename T>
void Ops<T>::dust_flux(const Launch& L, hipStream_t s, const Phys& ph, double tau, const T* phi,
                       const T* r1, const T* acc, T* G, const T* rhoj, const T* rn, T* Y) {
    LAUNCH(k_dust_flux<T>, L, s, ph, tau, phi, r1, acc, G, rhoj, rn, Y);
}
template <typename T>
void Ops<T>::dust_sweep(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                        const T* Yin, T* Yout, const T* G, const T* rhoj, const T* r1) {
    LAUNCH(k_dust_sweep<T>, L, s, ph, st, Yin, Yout, G, rhoj, r1);
}
template <typename T>
void Ops<T>::dust_faceflux(const Launch& L, hipStream_t s, const Phys& ph, const T* Y, T* G) {
    LAUNCH(k_dust_faceflux<T>, L, s, ph, Y, G);
}
template <typename T>
void Ops<T>::dust_finish(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, int cls,
                         const T* rhoj, const T* F, T* rhoj1, double* partials) {
    LAUNCH(k_dust_finish<T>, L, s, ph, st, cls, rhoj, F, rhoj1, partials);
}
template <typename T>
void Ops<T>::stats_gas(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, const T* r,
                       const T* u, double* partials) {
    LAUNCH(k_stats_gas<T>, L, s, ph, st, r, u, partials);
}
template <typename T>
void Ops<T>::sum_affine_sq(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                           const T* x, double a, double b, int slot, double* partials) {
    LAUNCH(k_sum_affine_sq<T>, L, s, ph, st, x, a, b, slot, partials);
}

template struct Ops<double>;
template struct Ops<float>;

}  // namespace pisoc
