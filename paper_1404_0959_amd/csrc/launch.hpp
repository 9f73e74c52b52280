// launch.hpp -- host-side launch wrappers of the PISO kernels (one set per
// storage type T), used by the step orchestration in pisoc.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "device.hpp"

namespace pisoc {

struct Launch {
    dim3 grid, block;
    unsigned nblocks;   // all members
    int cz;             // cells per thread along z
    int nz;             // blocks per member along z
    int v = 0;          // CG kernel: cells per lane along x of the full-row form (0: tiles)
    int h = 0;          // and wavefronts per x-row
    bool nt = false;    // and its once-read fields streamed past the caches (make_spmv_launch)
};

constexpr int kTargetBlocks = 2048;
constexpr int kTX = 64, kTY = 8;     // x-y tile of the z-marching kernels
constexpr int kTiledBlocks = 1024;

// Blocks of 64x4 (n >= 64) or 32x8 threads over x-y; each thread walks cz
// consecutive cells along z, with cz chosen for about kTargetBlocks blocks.
Launch make_launch(int n, int batch = 1);

// The same kernels with blocks of bx x (kBlock / bx) threads and cz cells per
// thread along z (bx a power of two in 16..256, 1 <= cz <= n).
Launch make_launch_shaped(int n, int batch, int bx, int cz);

// Launch of the LDS-tiled z-marching kernels (64 x 8 threads per block); nblocks
// is 0 when n is not a multiple of the tile (64 x 8); at n = 64 one tile spans
// x and its x halo wraps onto itself.  Blocks march over at least 8 planes, or
// exactly min(cz_tile, n) when cz_tile > 0 (a tuned choice).
Launch make_tiled_launch(int n, int batch = 1, int cz_tile = 0);

// Launch of the CG kernel for fields of elem_bytes per value.
// * n = 128 and 256: the full-row form, blocks of kRowWaves wavefronts, about
//   kRowBlocks blocks per member (v cells per lane, h wavefronts per row): at
//   256 one wavefront per x-row and 4 cells per lane in FP32, two per x-row and
//   2 cells per lane in FP64 (4 doubles per lane spill registers); at 128 one
//   wavefront per x-row and 2 cells per lane.
// * Other multiples of 64 (and of 8 spmv_rows): tiles of 64 x (8 spmv_rows)
//   cells, 64 x 8 threads each owning spmv_rows rows (v = 0; two rows in FP64
//   halve the tile's y halo; in FP32 two measured no faster).
// * Other multiples of kSmallTX: tiles of kSmallTX x kSmallTX cells, one thread
//   per column (block.x = kSmallTX).
// nblocks is 0 when none is available.  Tiles march over at least 8 planes, or
// exactly min(cz_tile, n) when cz_tile > 0 (a tuned choice; the full-row form
// ignores it).
// nt (full-row form): the fields a CG iteration reads once (r, q, p_old of the
// main rows) are loaded non-temporally, so that w and diag, which every
// iteration of a solve reads again, stay in the memory-side cache (kMallBytes)
// between launches.  Taken when the iteration's nine fields do not fit in that
// cache but w and diag fit in 60 % of it: at 256^3 in FP32 the CG then takes
// 5 % less time; in FP64 (w and diag 268 MB) it took 8 % more.
constexpr double kMallBytes = 256.0 * 1024 * 1024;
constexpr int spmv_rows(int elem_bytes) { return elem_bytes == 8 ? 2 : 1; }
constexpr int kSmallTX = 16;
constexpr int kRowWaves = 8, kRowBlocks = 256;
// Wavefronts per x-row of the full-row CG form for n and elem_bytes (0: none).
constexpr int row_waves(int n, int elem_bytes) {
    return n == 128 ? 1 : n != 256 ? 0 : elem_bytes == 4 ? 1 : 2;
}
Launch make_spmv_launch(int n, int batch, int elem_bytes, int cz_tile = 0);

// dst[0..count) = v (FP64).
void fill_value(hipStream_t s, double* dst, size_t count, double v);

// psi/dt = diag - (1/h^2) sum_f I4(w)_f of a captured pressure system (n^3 FP64).
void psidt_of(hipStream_t s, int n, const double* diag, const double* w, double* out);

// Partial-sum columns written by one CG iteration.
constexpr int kCgCols = 7;
// The momentum predictor's BiCGStab: partial slots from PS_CG for (rh.r, r.r,
// b.b), (rh.v) and (t.s, t.t).
constexpr int kBicgRes = 0, kBicgV = 3, kBicgTs = 4;
// Chebyshev-preconditioned CG: one set of columns per iteration (r.z, r.r,
// p.q), sets alternating by k & 1 from PS_CG, the interval's end after them.
constexpr int kChebRes = 0, kChebDir = 2, kChebSet = 3;

// Partial-sum slots in the workspace (columns of num_blocks doubles each).
enum PartSlot {
    PS_U = 0,      // 3 columns: r.z, r.r, b.b (CG system set-up)
    PS_CG = 3,     // 2 x kCgCols columns: CG iteration k in set k & 1
    PS_MASS = PS_CG + 2 * kCgCols,   // 3 columns: sum r, sum |u|^2, max(-rho)
    PS_CFL = PS_MASS + 3,            // 1 column: Courant maxima (k_cfl); must follow PS_MASS
    PS_STAT = PS_CFL + 1,            // 4 columns: statistics
    // 2 kMaxClasses columns: class c's dust finish writes, from PS_DUST + 2c
    // on, columns of nb partials each: sum rho_j, then max(-rho_j)
    PS_DUST = PS_STAT + 4,
    // 2 kMaxClasses columns: class c's first sweep writes, from PS_DDIAG + 2c
    // on, columns of nb partials each: max(-diagonal) of its implicit
    // equation, then its maximal Courant rate sum_f |G_f| / (2 rho V)
    PS_DDIAG = PS_DUST + 2 * kMaxClasses,
    PS_COLUMNS = PS_DDIAG + 2 * kMaxClasses
};

// Operands of CG iteration k.  Reads r_{k-1}, p_{k-1}, q_{k-1} (rin, pold,
// qold; only rin = r_0 at k = 0), diag and w, and at even k >= 2 p_{k-2}
// (pold2) and x; writes r_k (k >= 1), p_k, q_k and, at even k and at the
// stop, x.  part_in: the partials of iteration k-1 (kCgCols columns),
// at k = 0 those of the set-up kernel (r.z, r.r, b.b), written by nb_in
// blocks; part_out: this iteration's.  fresh: the set-up's b.b is the
// reference ||b||^2 of the solve; xzero: the solve started from x = 0 without
// x being written.
template <typename T>
struct CgArgs {
    const T* rin;
    T* rout;
    const T *diag, *w, *pold, *pold2;
    T* pnew;
    const T* qold;
    T *q, *x;
    const double* part_in;
    unsigned nb_in;
    double* part_out;
    int fresh, maxit, xzero;
};

template <typename T>
struct Ops {
    static void cast_in(hipStream_t s, const double* src, T* dst, size_t count, double shift);
    static void cast_out(hipStream_t s, const T* src, double* dst, size_t count, double shift);
    // one member's pressure p_ref + p_dev(r) (r points at the member's cells)
    // p = C rho^gamma, or rho R T with temp non-null (Fourier closure)
    static void pressure_out(hipStream_t s, const Phys& ph, double rho_ref, double p_ref,
                             const T* r, double* dst, const double* temp = nullptr);
    static void init_phi(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                         const T* r, const T* u, T* phi);
    static void cfl(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                    const T* r, const T* phi, double* part);
    // TL: the tiled z-march when available; nb_cfl: the number of Courant
    // partials in part_cfl (from cfl, or from the previous step's last
    // corrector pass)
    static void predict(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                        DevState* st, const double* part_cfl, unsigned nb_cfl, double dt_fixed,
                        double cfl, double growth, double dt_max, const T* rn, const T* un,
                        const T* phi, T* rs, T* aP, T* divu, T* pn);
    // Field kernels taking TL run as k_tiled z-marches when TL.nblocks > 0;
    // those that write partials return how many (blocks of the launch used).
    static void mom_source(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                           const DevState* st, const T* rn, const T* un, const T* divu, T* src);
    // TL: tiled launch (used when TL.nblocks > 0)
    static void mom_sweep(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                          const DevState* st, const T* uin, T* uout, const T* phi, const T* aP,
                          const T* src, const T* pn);
    static void hbya(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                     const DevState* st, const T* uin, T* hb, const T* phi, const T* aP,
                     const T* src, const T* rk, T* w, T* p0);
    // CG starts from x = 0 without x being written (see pcg_spmv's xzero).
    // TL: the tiled z-march when available.  Returns the number of partials
    // written to part_u (blocks of the launch used).
    static unsigned corr_rhs(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                             DevState* st, const T* rn, const T* rk, const T* w, const T* hb,
                             const T* p0, T* phiH, T* r, T* diag, double* part_u, double* snap_b,
                             double* snap_diag, double* snap_p0, double* b64);
    // from_zero: x64 is zero and not read (first round of a solve from zero);
    // xf: the new x64n rounded to T (not aliasing d); store_x = false (with
    // from_zero): x64n = d exactly, neither x64n nor xf is written
    static unsigned refine(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                           DevState* st, const double* x64, const T* d, double* x64n, T* xf,
                           const double* b64, const T* w, const T* diag, T* r32,
                           double* part_u, bool from_zero, bool store_x);
    // CG iteration k (one kernel); TL: the CG launch of make_spmv_launch
    // (used when TL.nblocks > 0)
    static void pcg_iter(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                         DevState* st, int k, const CgArgs<T>& a);
    static void helm_apply(const Launch& L, hipStream_t s, const Phys& ph, const T* psidt,
                           const T* w, const T* x, T* y);
    // the momentum predictor solved to a tolerance: BiCGStab set-up (x = u^n
    // in place) and iteration i >= 1 (three launches)
    static void bicg_init(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, const T* x,
                          const T* F, const T* aP, const T* src, const T* pn, T* r, T* rh,
                          double* part);
    static void bicg_iter(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                          DevState* st, int i, double tol2, int maxit, T* x, T* r, const T* rh,
                          T* const w[6], const T* F, const T* aP, double* part_res, double* part_v,
                          double* part_ts);
    // Fourier closure: the energy predictor's coefficients and one Jacobi sweep
    static void energy_setup(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                             const T* rn, const T* rs, const T* phi, const T* divu, const T* pn,
                             double* aT, double* sT);
    static void energy_sweep(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                             const DevState* st, const double* tin, double* tout, const T* phi,
                             const double* aT, const double* sT);
    // CG preconditioned by a Chebyshev polynomial (stand-alone solve): the
    // interval's lower end, then per iteration the residual/preconditioner and
    // the direction/operator launches
    static void cheb_theta(const Launch& L, hipStream_t s, const Phys& ph, const T* psidt,
                           const T* diag, double* part);
    static void cheb_res(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                         DevState* st, int k, const T* rin, T* rout, const T* q, const T* p,
                         const T* diag, const T* w, T* x, T* z, const double* part_theta,
                         unsigned nb_theta, const double* part_prev, double* part_out);
    static void cheb_dir(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                         DevState* st, int k, const T* z, const T* pin, T* pout, T* q,
                         const T* diag, const T* w, const double* part_u, unsigned nb_u,
                         const double* part_prev, double* part_cur, int maxit);
    static void helm_start(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                           const T* psidt, const T* w, const T* b, const T* x, T* r, T* diag,
                           double* part_u);
    static void corr_flux(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                          const DevState* st, const T* p0, const T* x, const T* w,
                          const T* phiH, T* phik, T* pt, double* snap_x);
    // corr_flux and corr_update in one tiled pass (TL.nblocks > 0), p not
    // stored; the last corrector writes, from part_mass on, columns of nb
    // partials each: the three of the mass budget, then the Courant maxima of
    // the new state (4 nb <= 4 max_blocks: within PS_MASS and PS_CFL).
    // Returns nb, the launch's block count.
    static unsigned corr_finish_fused(const Launch& TL, hipStream_t s, const Phys& ph,
                                      const DevState* st, bool last, const T* p0, const T* x,
                                      const T* w, const T* phiH, T* phik, double* snap_x,
                                      const T* rn, const T* hb, const T* aP, T* rk, T* u,
                                      double* part_mass);
    static unsigned corr_update(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                                const DevState* st, bool last, const T* rn, const T* phik,
                                const T* hb, const T* pt, const T* aP, T* rk, T* u,
                                double* part_mass);
    static void dudt(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                     const DevState* st, const T* un, const T* u1, T* acc);
    static void dust_flux(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                          const DevState* st, int cls, const T* phi, const T* r1, const T* acc,
                          T* G, const T* rhoj, const T* rn, T* Y);
    // part_diag non-null (the class's first sweep): partials max(-diagonal)
    // of the implicit equation and max of the dust's Courant rate (two
    // columns of the launch's block count); returns the launch's block count
    static unsigned dust_sweep(const Launch& L, const Launch& TL, hipStream_t s, const Phys& ph,
                               const DevState* st, const T* Yin, T* Yout, const T* G,
                               const T* rhoj, const T* r1, double* part_diag);
    static void dust_faceflux(const Launch& L, hipStream_t s, const Phys& ph, const T* Y, T* G);
    // partials: two columns of L.nblocks from part on, sum rho_j and max(-rho_j);
    // fdo (two-way coupling, else null): the class's own-face fluxes go into the
    // next step's dust flux F_d (written by the first class, added by the others)
    static void dust_finish(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                            const T* rhoj, const T* F, T* rhoj1, double* part, T* fdo,
                            bool first);
    // two-way coupling: initial dust mass fluxes fd = I4(sum_j rho_j) I4(u) A
    static void init_fd(const Launch& L, hipStream_t s, const Phys& ph, int ncls,
                        const T* rhoj, const T* u, T* fd);
    // two-way coupling: a_P and the source of the mixture, and its mass flux fm
    static void mixture(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                        int ncls, const T* rn, const T* un, const T* rhoj, const T* phi,
                        const T* fd, T* fm, T* aP, T* src);
    // dust_faceflux and dust_finish in one tiled pass (TL.nblocks > 0), F not
    // stored; returns the number of partials written per column (two columns,
    // as dust_finish)
    static unsigned dust_finish_fused(const Launch& TL, hipStream_t s, const Phys& ph,
                                      const DevState* st, const T* Y, const T* G,
                                      const T* rhoj, T* rhoj1, double* part, T* fdo,
                                      bool first);
    static void stats_gas(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                          const T* r, const T* u, double* part);
    // st non-null: per-member (a, b) = st[m].aff
    static void sum_affine_sq(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                              const T* x, double a, double b, double* part);
    // learned guess
    static void net_stats(const Launch& L, hipStream_t s, const Phys& ph, const T* b,
                          const T* diag, const T* p0, double* part);
    static void net_input(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                          const double* part, const T* b, const T* diag, const T* p0,
                          uint16_t* x4, float* x2, const T* psol, float* tgt);
    // g = s1 y (y: the network's output) or, with gd set, g = gd
    static void guess_start(const Launch& L, hipStream_t s, const Phys& ph, const DevState* st,
                            const float* y, const T* gd, const T* w, const T* diag, const T* b,
                            const double* b64, T* g, T* mg, double* part);
    static void guess_apply(const Launch& L, hipStream_t s, const Phys& ph, DevState* st,
                            const double* part_g, const T* g, const T* mg, const T* diag, T* r,
                            T* x, double* x64, const double* b64, T* bsave, double* part_u);
    // per member, where the guess does not lower ||r|| (totals in st[m].red[1..2])
    static void guess_revert(const Launch& L, hipStream_t s, const Phys& ph, DevState* st, T* r,
                             T* x, double* x64, const double* b64, const T* bsave,
                             const T* diag, double* part_u);
};

// Per member: totals of nv partial columns (written by a launch of nbt blocks
// over `batch` members) into st[m].red[off ..]; honor_skip: not for a member
// whose refinement round was skipped (pcg.skip).
void finalize_sums(hipStream_t s, const double* part, unsigned nbt, int batch, int nv,
                   DevState* st, int off, bool honor_skip = false);
// Total of nb partials (one column) into dst[0].
void sum_partials(hipStream_t s, const double* part, unsigned nb, double* dst);
// Per member: end-of-step mass budget and flags.
// nb_mass: partials of the last corrector update; nb_dust: of the dust finish
// (class c's two columns from part_dust + 2 c cls_stride); nb_diag: of the
// first dust sweep (class c's two columns from part_diag + 2 c cls_stride)
void step_finish(hipStream_t s, const Phys& ph, DevState* st, const double* part_mass,
                 unsigned nb_mass, const double* part_dust, int ncls, unsigned nb_dust,
                 const double* part_diag, unsigned nb_diag, size_t cls_stride);
// Per member: t += dt, dt_prev = dt (the step is accepted); fold the step
// record into the accumulators.
void commit(hipStream_t s, DevState* st, int batch);
// Per member: clear the accumulators.
void clear_acc(hipStream_t s, DevState* st, int batch);
// Per member: tolerance of the next FP32 refinement round (see k_set_tol_refine).
void set_tol_refine(hipStream_t s, DevState* st, int batch, double tau_min);
// Per member: CG tolerance (squared) for the next solve.
void set_tol(hipStream_t s, DevState* st, int batch, double tol2);
// Per member: affine coefficients for sum_affine_sq (see k_set_affine).
void set_affine(hipStream_t s, DevState* st, int batch, int mode, double N);
// Per member: record a solve of corrector corr in the step record (see k_record_solve).
void record_solve(hipStream_t s, DevState* st, int batch, int corr, int round, int add, int fin);
// Per member: clear the step flags.
void clear_flags(hipStream_t s, DevState* st, int batch);

}  // namespace pisoc
