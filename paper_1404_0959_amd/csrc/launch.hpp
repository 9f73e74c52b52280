// launch.hpp -- host-side launch wrappers of the PISO kernels (one set per
// storage type T), used by the step orchestration in pisoc.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "device.hpp"

namespace pisoc {

struct Launch {
    dim3 grid, block;
    unsigned nblocks;
    int cz;
};

// Blocks of 64x4 (n >= 64) or 32x8 threads over x-y; each thread walks cz cells along z.
Launch make_launch(int n, int cz);

template <typename T>
struct Ops {
    static void cast_in(hipStream_t s, const double* src, T* dst, size_t count, double shift);
    static void cast_out(hipStream_t s, const T* src, double* dst, size_t count, double shift);
    static void pressure_out(hipStream_t s, const Phys& ph, const T* r, double* dst);
    static void init_phi(const Launch& L, hipStream_t s, const Phys& ph, const T* r, const T* u,
                         T* phi);
    static void cfl(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, const T* r,
                    const T* phi, double* partials, double dt_fixed, double cfl, double growth,
                    double dt_prev, double dt_max);
    static void predict(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                        const T* rn, const T* un, const T* phi, T* rs, T* aP, T* divu, T* pn);
    static void mom_source(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                           const T* rn, const T* un, const T* divu, T* src);
    static void mom_sweep(const Launch& L, hipStream_t s, const Phys& ph, const T* uin, T* uout,
                          const T* phi, const T* aP, const T* src, const T* pn);
    static void hbya(const Launch& L, hipStream_t s, const Phys& ph, const T* uin, T* hb,
                     const T* phi, const T* aP, const T* src, const T* rk, T* w, T* p0);
    static void corr_rhs(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                         const T* rn, const T* rk, const T* w, const T* hb, const T* p0, T* phiH,
                         T* r, T* x, T* diag, double* partials, double* snap_b,
                         double* snap_diag, double* snap_p0);
    static void pcg_spmv(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, int k,
                         const T* r, const T* diag, const T* w, const T* pold, T* pnew, T* q,
                         double* partials);
    static void pcg_update(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, int k,
                           T* r, const T* q, const T* diag, T* x, const T* p, double* partials);
    static void helm_apply(const Launch& L, hipStream_t s, const Phys& ph, const T* psidt,
                           const T* w, const T* x, T* y);
    static void helm_start(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                           const T* psidt, const T* w, const T* b, const T* x, T* r, T* diag,
                           double* partials);
    static void corr_flux(const Launch& L, hipStream_t s, const Phys& ph, const T* p0, const T* x,
                          const T* w, const T* phiH, T* phik, T* pt, double* snap_x);
    static void corr_update(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                            bool last, const T* rn, const T* phik, const T* hb, const T* pt,
                            const T* aP, T* rk, T* u, double* partials);
    static void dudt(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                     const T* un, const T* u1, T* acc);
    static void dust_flux(const Launch& L, hipStream_t s, const Phys& ph, double tau,
                          const T* phi, const T* r1, const T* acc, T* G, const T* rhoj,
                          const T* rn, T* Y);
    static void dust_sweep(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                           const T* Yin, T* Yout, const T* G, const T* rhoj, const T* r1);
    static void dust_faceflux(const Launch& L, hipStream_t s, const Phys& ph, const T* Y, T* G);
    static void dust_finish(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, int cls,
                            const T* rhoj, const T* F, T* rhoj1, double* partials);
    static void stats_gas(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                          const T* r, const T* u, double* partials);
    static void sum_affine_sq(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                              const T* x, double a, double b, int slot, double* partials);
};

}  // namespace pisoc
