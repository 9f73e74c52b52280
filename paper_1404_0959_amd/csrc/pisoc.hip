// pisoc.hip -- host orchestration of the PISO step and the C ABI (pisoc.h).
//
// The library owns no device memory: every field, the CG vectors, the
// reduction partials and the device-side state live in the caller's
// workspace.  All work is enqueued on the caller's stream.  The host waits on
// the stream only to learn when a pressure solve has converged (one wait per
// batch of CG iterations, whose size is predicted from the previous solve) and
// at the end of each step, to check it before committing it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pisoc.h"
#include "device.hpp"
#include "launch.hpp"
#include "net.hpp"

using namespace pisoc;

namespace {

constexpr size_t kAlign = 256;
constexpr double kTwoPi = 6.283185307179586476925286766559;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of every buffer inside the workspace.
struct Layout {
    size_t state, partials;
    size_t rn, rk, aP, divu, pn, w, p0, r, x, diag, pp0, pp1, q, Y0, Y1;
    size_t u3[3], phin, phik, src, hbya, phiH, acc, G;
    size_t rhop, rhop1;
    size_t snap;   // 4 FP64 fields when capturing
    size_t b64, x64a, x64b;  // FP64 refinement fields (FP32 storage only)
    size_t wpk, nx4, na, nb, ny, bsave;  // learned guess: packed weights, activations
    size_t total;
    unsigned max_blocks;
};


// Kernel classes for the optional per-launch event timing.
enum KCls {
    KC_CFL, KC_PREDICT, KC_MOM_SOURCE, KC_MOM_SWEEP, KC_HBYA, KC_CORR_RHS, KC_PCG_SPMV,
    KC_PCG_UPDATE, KC_CORR_FLUX, KC_CORR_UPDATE, KC_DUDT, KC_DUST_FLUX, KC_DUST_SWEEP,
    KC_DUST_FACEFLUX, KC_DUST_FINISH, KC_REFINE, KC_NET, KC_COUNT
};
const char* const kKernelName[KC_COUNT] = {
    "k_cfl", "k_predict", "k_mom_source", "k_mom_sweep", "k_hbya", "k_corr_rhs",
    "k_pcg_spmv", "k_pcg_update", "k_corr_flux", "k_corr_update", "k_dudt", "k_dust_flux",
    "k_dust_sweep", "k_dust_faceflux", "k_dust_finish", "k_refine", "learned_guess"};

struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int cls; size_t ea, eb; double bytes; int k; };
    std::vector<Rec> pending;
    pisoc_kernel_stat stat[KC_COUNT];

    size_t take() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return (size_t)-1;
            pool.push_back(e);
        }
        return used++;
    }
    void reset() {
        std::memset(stat, 0, sizeof(stat));
        for (int i = 0; i < KC_COUNT; ++i)
            std::snprintf(stat[i].name, sizeof(stat[i].name), "%s", kKernelName[i]);
        pending.clear();
        used = 0;
    }
    // Attribute completed launches; CG launches with k >= it_stop returned at once.
    void resolve(int it_stop) {
        for (const Rec& r : pending) {
            if (r.k >= 0 && r.k >= it_stop) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pool[r.ea], pool[r.eb]) != hipSuccess) continue;
            stat[r.cls].launches += 1;
            stat[r.cls].ms += ms;
            stat[r.cls].bytes += r.bytes;
        }
        pending.clear();
        used = 0;
    }
    ~Prof() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

bool valid_params(const pisoc_params* p, std::string* why) {
    auto fail = [&](const char* m) { if (why) *why = m; return false; };
    if (!p) return fail("params is NULL");
    if (p->n < PISOC_MIN_N || p->n > PISOC_MAX_N) return fail("n out of range");
    if (p->n_classes < 0 || p->n_classes > PISOC_MAX_CLASSES) return fail("n_classes out of range");
    if (!(p->gamma > 1.0) || !(p->C > 0.0) || !(p->mu >= 0.0)) return fail("bad gamma, C or mu");
    if (p->n_corr < 1 || p->n_corr > PISOC_MAX_CORR) return fail("n_corr out of range");
    if (p->n_mom_sweeps < 1 || p->n_dust_sweeps < 1) return fail("sweep counts must be >= 1");
    if (!(p->p_tol > 0.0) || !(p->p_tol < 1.0) || p->p_maxit < 1) return fail("bad p_tol or p_maxit");
    if (!(p->dt_fixed > 0.0) && !(p->cfl > 0.0 && p->dt_growth > 0.0))
        return fail("need dt_fixed > 0 or cfl > 0 and dt_growth > 0");
    for (int c = 0; c < p->n_classes; ++c)
        if (!(p->tau_p[c] >= 0.0)) return fail("tau_p must be >= 0");
    if (p->precision != PISOC_FP64 && p->precision != PISOC_FP32_REFINED)
        return fail("unknown precision");
    if (p->precision == PISOC_FP32_REFINED &&
        (!(p->inner_tol > 0.0) || !(p->inner_tol < 1.0) || p->max_refine < 1))
        return fail("FP32_REFINED needs 0 < inner_tol < 1 and max_refine >= 1");
    if (p->guess != PISOC_GUESS_ZERO && p->guess != PISOC_GUESS_LEARNED) return fail("unknown guess");
    if (p->guess == PISOC_GUESS_LEARNED && (!p->d_guess_weights || p->n % 16 != 0))
        return fail("learned guess needs d_guess_weights and n % 16 == 0");
    return true;
}

Layout make_layout(const pisoc_params* p) {
    Layout L{};
    const size_t N = (size_t)p->n * p->n * p->n;
    const size_t es = p->precision == PISOC_FP64 ? sizeof(double) : sizeof(float);
    const Launch lc = make_launch(p->n);
    L.max_blocks = std::max(lc.nblocks, make_tiled_launch(p->n).nblocks);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.state = take(sizeof(DevState));
    L.partials = take(sizeof(double) * PS_COLUMNS * (size_t)L.max_blocks);
    size_t* one[] = {&L.rn, &L.rk, &L.aP, &L.divu, &L.pn, &L.w, &L.p0, &L.r, &L.x, &L.diag,
                     &L.pp0, &L.pp1, &L.q, &L.Y0, &L.Y1};
    for (size_t* o : one) *o = take(es * N);
    size_t* three[] = {&L.u3[0], &L.u3[1], &L.u3[2], &L.phin, &L.phik, &L.src, &L.hbya,
                       &L.phiH, &L.acc, &L.G};
    for (size_t* o : three) *o = take(3 * es * N);
    L.rhop = take(es * N * (size_t)std::max(p->n_classes, 1));
    L.rhop1 = take(es * N * (size_t)std::max(p->n_classes, 1));
    L.snap = p->capture ? take(4 * sizeof(double) * N) : 0;
    if (p->guess == PISOC_GUESS_LEARNED) {
        L.wpk = take(net_packed_bytes());
        L.nx4 = take(4 * 2 * N);
        L.na = take(16 * 2 * N);
        L.nb = take(16 * 2 * N);
        L.ny = take(4 * N);
        L.bsave = take(es * N);
    }
    if (p->precision == PISOC_FP32_REFINED) {
        L.b64 = take(sizeof(double) * N);
        L.x64a = take(sizeof(double) * N);
        L.x64b = take(sizeof(double) * N);
    }
    L.total = off;
    return L;
}

}  // namespace

struct pisoc_ctx {
    pisoc_params prm;
    hipStream_t stream;
    char* ws;
    Layout lay;
    Phys ph;
    Launch L;
    Launch TL;      // tiled z-marching launch (nblocks = 0 when not available)
    DevState* st;
    DevState* hst;  // pinned host copy
    double* partials;
    // rotating buffers
    int u_idx[3];   // which of lay.u3 holds u^n, work a, work b
    size_t rn, rk, phin, phik, rhop, rhop1;
    double t, dt_prev;
    int64_t steps;
    int last_iters[PISOC_MAX_CORR];
    int last_first[PISOC_MAX_CORR];  // FP32 mode: iterations of the first inner solve
    size_t es;      // bytes per field element (8 or 4)
    Prof prof;
    std::string err;

    template <typename T> T* f(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    size_t N() const { return (size_t)prm.n * prm.n * prm.n; }
    // partial-sum column `slot` (num_blocks doubles per column)
    double* part(int slot) const { return partials + (size_t)slot * lay.max_blocks; }
};

namespace {

pisoc_status hip_fail(pisoc_ctx* ctx, hipError_t e, const char* where) {
    if (ctx) ctx->err = std::string(where) + ": " + hipGetErrorString(e);
    return PISOC_ERR_HIP;
}

#define HIP_TRY(ctx, expr)                                      \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

// Run `launch` (one kernel launch), bracketed by events when profiling.
template <class F>
void timed(pisoc_ctx* ctx, int cls, double words, int k, F&& launch) {
    Prof& P = ctx->prof;
    if (!P.on) {
        launch();
        return;
    }
    const size_t a = P.take(), b = P.take();
    if (a == (size_t)-1 || b == (size_t)-1) {
        launch();
        return;
    }
    (void)hipEventRecord(P.pool[a], ctx->stream);
    launch();
    (void)hipEventRecord(P.pool[b], ctx->stream);
    P.pending.push_back({cls, a, b, words * (double)ctx->es * (double)ctx->N(), k});
}

pisoc_status sync_state(pisoc_ctx* ctx) {
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->hst, ctx->st, sizeof(DevState), hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PISOC_OK;
}

Phys make_phys(const pisoc_params* p, double rho_ref) {
    Phys ph{};
    ph.n = p->n;
    ph.cz = make_launch(p->n).cz;
    ph.h = kTwoPi / p->n;
    ph.inv_h = 1.0 / ph.h;
    ph.inv_h2 = 1.0 / (ph.h * ph.h);
    ph.V = ph.h * ph.h * ph.h;
    ph.inv_V = 1.0 / ph.V;
    ph.A = ph.h * ph.h;
    ph.gamma = p->gamma;
    ph.C = p->C;
    ph.mu = p->mu;
    ph.rho_ref = rho_ref;
    ph.p_ref = p->C * std::pow(rho_ref, p->gamma);
    return ph;
}

// CG on the system already set up by corr_rhs / helm_start (which left the
// partials r0.z0, r0.r0, b.b).  Launches the first half of iteration 0, then
// batches of (second half k, first half k+1) pairs; the first half of k+1
// tests convergence, so a batch always ends on a test.  Launches after the
// stop return at once.
template <typename T>
pisoc_status run_pcg(pisoc_ctx* ctx, T* r, T* x, T* diag, T* w, T* pp0, T* pp1, T* q,
                     double tol, int predicted, int32_t* iters, double* relres, bool* converged) {
    using O = Ops<T>;
    const int maxit = ctx->prm.p_maxit;
    T* pp[2] = {pp0, pp1};
    double* pu = ctx->part(PS_U);
    double* ps = ctx->part(PS_S);
    auto spmv = [&](int k) {
        timed(ctx, KC_PCG_SPMV, k == 0 ? 5.0 : 6.0, k, [&] {
            O::pcg_spmv(ctx->L, ctx->TL, ctx->stream, ctx->ph, ctx->st, k, r, diag, w,
                        pp[(k + 1) & 1], pp[k & 1], q, pu, ps, tol * tol, maxit);
        });
    };
    auto update = [&](int k) {
        timed(ctx, KC_PCG_UPDATE, 7.0, k, [&] {
            O::pcg_update(ctx->L, ctx->TL, ctx->stream, ctx->ph, ctx->st, k, r, q, diag, x, pp[k & 1],
                          ps, pu);
        });
    };
    spmv(0);
    int k = 0;  // first halves launched: 0..k
    int batch = std::max(1, predicted);
    for (;;) {
        const int kend = std::min(k + batch, maxit);
        for (; k < kend; ++k) {
            update(k);
            spmv(k + 1);
        }
        pisoc_status s = sync_state(ctx);
        if (s != PISOC_OK) return s;
        if (ctx->prof.on) ctx->prof.resolve(ctx->hst->pcg.it_stop);
        if (ctx->hst->flags & PISOC_FLAG_BAD_DT) break;
        if (ctx->hst->pcg.it_stop != kIterInf || k >= maxit) break;
        batch = 2;
    }
    const PcgState& g = ctx->hst->pcg;
    *iters = g.iters;
    *relres = g.bb > 0.0 ? std::sqrt(g.rr / g.bb) : 0.0;
    *converged = g.converged != 0;
    return PISOC_OK;
}

// FP32 storage: mixed-precision iterative refinement of M p' = b.  Inner
// solves are FP32 CG to a relative tolerance tau; after each, k_refine adds the
// correction to the FP64 accumulator and evaluates the true residual in FP64;
// the loop ends when ||r64|| <= p_tol ||b64||.
pisoc_status refine_solve(pisoc_ctx* ctx, float* r, float* x, float* diag, float* w, float* pp0,
                          float* pp1, float* q, int corr, int32_t* iters, double* relres,
                          bool* converged, int32_t* rounds) {
    const pisoc_params& p = ctx->prm;
    double* b64 = ctx->f<double>(ctx->lay.b64);
    double* xa = ctx->f<double>(ctx->lay.x64a);
    double* xb = ctx->f<double>(ctx->lay.x64b);
    const size_t N = ctx->N();
    int32_t it = 0, total = 0;
    double rel = 0.0;
    bool conv = false;
    const int pred0 = ctx->last_first[corr] > 0 ? ctx->last_first[corr] : 8;
    const double tau0 = std::min(0.5, std::max(0.5 * p.p_tol, p.inner_tol));
    pisoc_status st = run_pcg<float>(ctx, r, x, diag, w, pp0, pp1, q, tau0, pred0, &it, &rel,
                                     &conv);
    if (st != PISOC_OK) return st;
    ctx->last_first[corr] = it;
    total += it;
    const double bb = ctx->hst->pcg.bb;
    double rr = bb;
    int nround = 0;
    if (bb > 0.0) {
        for (;;) {
            timed(ctx, KC_REFINE, 10, -1, [&] {
                Ops<float>::refine(ctx->L, ctx->stream, ctx->ph, ctx->st, xa, x, xb, b64, w, diag, r,
                                   ctx->part(PS_U));
            });
            std::swap(xa, xb);
            // column 1 (||r64||^2) of the 3-column block written with L.nblocks blocks
            finalize_sums(ctx->stream, ctx->part(PS_U) + ctx->L.nblocks, ctx->L.nblocks, 1,
                          ctx->st->red);
            if ((st = sync_state(ctx)) != PISOC_OK) return st;
            if (ctx->prof.on) ctx->prof.resolve(kIterInf);
            rr = ctx->hst->red[0];
            ++nround;
            if (rr <= p.p_tol * p.p_tol * bb || nround >= p.max_refine || !std::isfinite(rr)) break;
            double tau = 0.5 * p.p_tol * std::sqrt(bb / rr);
            tau = std::min(0.5, std::max(tau, p.inner_tol));
            Ops<float>::zero(ctx->stream, x, N);
            st = run_pcg<float>(ctx, r, x, diag, w, pp0, pp1, q, tau, 2, &it, &rel, &conv);
            if (st != PISOC_OK) return st;
            total += it;
        }
    }
    // the corrector uses the FP32 copy of the FP64 solution
    Ops<float>::cast_in(ctx->stream, xa, x, N, 0.0);
    *iters = total;
    *relres = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    *converged = rr <= p.p_tol * p.p_tol * bb;
    *rounds = nround;
    return PISOC_OK;
}

// The learned initial guess of one pressure solve: scaled inputs from the
// system just set up, the network on the matrix cores, CG restarted from
// x0 = alpha s1 y (alpha energy-optimal); rejected (back to x0 = 0) unless
// ||b - M x0|| < ||b||.
template <typename T>
pisoc_status learned_guess(pisoc_ctx* ctx, T* r, T* x, T* dg, T* w, T* p0, T* gbuf, T* mgbuf,
                           int* flags) {
    using O = Ops<T>;
    const Layout& Y = ctx->lay;
    const bool f32 = sizeof(T) == sizeof(float);
    hipStream_t s = ctx->stream;
    double* x64 = f32 ? ctx->f<double>(Y.x64a) : nullptr;
    double* b64 = f32 ? ctx->f<double>(Y.b64) : nullptr;
    T* bsave = ctx->f<T>(Y.bsave);
    timed(ctx, KC_NET, 2, -1, [&] {
        O::net_stats(ctx->L, s, ctx->ph, r, dg, p0, ctx->part(PS_STAT));
        O::net_input(ctx->L, s, ctx->ph, ctx->st, ctx->part(PS_STAT), r, dg, p0,
                     ctx->f<uint16_t>(Y.nx4), nullptr, nullptr, nullptr);
        net_forward(s, ctx->prm.n, 1, ctx->ws + Y.wpk, ctx->f<uint16_t>(Y.nx4),
                    ctx->f<uint16_t>(Y.na), ctx->f<uint16_t>(Y.nb), ctx->f<float>(Y.ny), 1.f);
        O::guess_start(ctx->L, s, ctx->ph, ctx->st, ctx->f<float>(Y.ny), w, dg, r, b64, gbuf,
                       mgbuf, ctx->part(PS_STAT));
        O::guess_apply(ctx->L, s, ctx->ph, ctx->st, ctx->part(PS_STAT), gbuf, mgbuf, dg, r, x,
                       x64, b64, bsave, ctx->part(PS_U));
    });
    // totals of r0.z0, ||r0||^2, ||b||^2 (3 columns written with L.nblocks blocks)
    const unsigned nb = ctx->L.nblocks;
    finalize_sums(s, ctx->part(PS_U), nb, 3, ctx->st->red);
    pisoc_status st = sync_state(ctx);
    if (st != PISOC_OK) return st;
    if (ctx->prof.on) ctx->prof.resolve(kIterInf);
    const double rr = ctx->hst->red[1], bb = ctx->hst->red[2];
    if (!(rr < bb)) {
        *flags |= PISOC_FLAG_GUESS_FALLBACK;
        O::guess_revert(ctx->L, s, ctx->ph, r, x, x64, b64, bsave, dg, ctx->part(PS_U));
    }
    return PISOC_OK;
}

template <typename T>
pisoc_status one_step(pisoc_ctx* ctx, pisoc_step_info* info) {
    using O = Ops<T>;
    const pisoc_params& p = ctx->prm;
    const Phys& ph = ctx->ph;
    const Launch& L = ctx->L;
    hipStream_t s = ctx->stream;
    const size_t N = ctx->N();
    DevState* st = ctx->st;
    auto F = [&](size_t off) { return ctx->f<T>(off); };
    const Layout& Y = ctx->lay;

    T* rn = F(ctx->rn);
    T* rk = F(ctx->rk);
    T* un = F(Y.u3[ctx->u_idx[0]]);
    T* ua = F(Y.u3[ctx->u_idx[1]]);
    T* ub = F(Y.u3[ctx->u_idx[2]]);
    T* phin = F(ctx->phin);
    T* phik = F(ctx->phik);
    T *aP = F(Y.aP), *divu = F(Y.divu), *pn = F(Y.pn), *src = F(Y.src), *hb = F(Y.hbya);
    T *w = F(Y.w), *p0 = F(Y.p0), *phiH = F(Y.phiH), *r = F(Y.r), *x = F(Y.x), *dg = F(Y.diag);
    T *pp0 = F(Y.pp0), *pp1 = F(Y.pp1), *q = F(Y.q);
    double* snap = p.capture ? reinterpret_cast<double*>(ctx->ws + Y.snap) : nullptr;
    const bool f32 = sizeof(T) == sizeof(float);

    pisoc_step_info rec{};
    int flags = 0;
    pisoc_status worst = PISOC_OK;

    HIP_TRY(ctx, hipMemsetAsync(&st->flags, 0, sizeof(int32_t), s));
    timed(ctx, KC_CFL, 4, -1, [&] { O::cfl(L, s, ph, rn, phin, ctx->part(PS_CFL)); });
    timed(ctx, KC_PREDICT, 11, -1, [&] {
        O::predict(L, s, ph, st, ctx->part(PS_CFL), p.dt_fixed, p.cfl, p.dt_growth, ctx->dt_prev,
                   p.dt_max, rn, un, phin, rk, aP, divu, pn);
    });
    timed(ctx, KC_MOM_SOURCE, 8, -1, [&] { O::mom_source(L, s, ph, st, rn, un, divu, src); });
    T* uin = un;
    for (int i = 0; i < p.n_mom_sweeps; ++i) {
        T* uout = (i & 1) ? ub : ua;
        timed(ctx, KC_MOM_SWEEP, 14, -1, [&] { O::mom_sweep(L, s, ph, uin, uout, phin, aP, src, pn); });
        uin = uout;
    }
    T* ucur = uin;
    const int ucur_slot = (ucur == ua) ? 1 : 2;

    for (int corr = 0; corr < p.n_corr; ++corr) {
        timed(ctx, KC_HBYA, 16, -1, [&] { O::hbya(L, s, ph, ucur, hb, phin, aP, src, rk, w, p0); });
        const bool cap = snap && corr == 0;
        timed(ctx, KC_CORR_RHS, f32 ? 17 : 13, -1, [&] {
            O::corr_rhs(L, s, ph, st, rn, rk, w, hb, p0, phiH, r, x, dg, ctx->part(PS_U),
                        cap ? snap : nullptr, cap ? snap + N : nullptr,
                        cap ? snap + 2 * N : nullptr, f32 ? ctx->f<double>(Y.b64) : nullptr,
                        f32 ? ctx->f<double>(Y.x64a) : nullptr);
        });
        if (p.guess == PISOC_GUESS_LEARNED) {
            pisoc_status gs = learned_guess<T>(ctx, r, x, dg, w, p0, pp0, q, &flags);
            if (gs != PISOC_OK) return gs;
            if (flags & PISOC_FLAG_GUESS_FALLBACK) worst = std::max(worst, PISOC_WARN_GUESS_FALLBACK);
        }
        int32_t it = 0, rounds = 0;
        double rel = 0.0;
        bool conv = false;
        const int pred = ctx->last_iters[corr] > 0 ? ctx->last_iters[corr] : 8;
        pisoc_status ps;
        if constexpr (sizeof(T) == sizeof(float))
            ps = refine_solve(ctx, r, x, dg, w, pp0, pp1, q, corr, &it, &rel, &conv, &rounds);
        else
            ps = run_pcg<T>(ctx, r, x, dg, w, pp0, pp1, q, p.p_tol, pred, &it, &rel, &conv);
        if (ps != PISOC_OK) return ps;
        rec.refinements[corr] = rounds;
        if (ctx->hst->flags & PISOC_FLAG_BAD_DT) {
            ctx->err = "time step undefined or non-positive (zero velocity needs dt_fixed or dt_max)";
            return PISOC_ERR_INVALID;
        }
        ctx->last_iters[corr] = it;
        rec.pcg_iters[corr] = it;
        rec.pcg_relres[corr] = rel;
        if (!conv) {
            flags |= PISOC_FLAG_PCG_MAXIT;
            worst = PISOC_WARN_NOT_CONVERGED;
        }
        timed(ctx, KC_CORR_FLUX, 10, -1, [&] {
            O::corr_flux(L, s, ph, p0, x, w, phiH, phik, q, cap ? snap + 3 * N : nullptr);
        });
        timed(ctx, KC_CORR_UPDATE, 13, -1, [&] {
            O::corr_update(L, s, ph, st, corr == p.n_corr - 1, rn, phik, hb, q, aP, rk, ucur,
                           ctx->part(PS_MASS));
        });
    }

    if (p.n_classes > 0) {
        T* acc = F(Y.acc);
        T* G = F(Y.G);
        T* Ya = F(Y.Y0);
        T* Yb = F(Y.Y1);
        T* rj = F(ctx->rhop);
        T* rj1 = F(ctx->rhop1);
        timed(ctx, KC_DUDT, 9, -1, [&] { O::dudt(L, s, ph, st, un, ucur, acc); });
        for (int c = 0; c < p.n_classes; ++c) {
            timed(ctx, KC_DUST_FLUX, 13, -1, [&] {
                O::dust_flux(L, s, ph, p.tau_p[c], phik, rk, acc, G, rj + c * N, rn, Ya);
            });
            T* yin = Ya;
            T* yout = Yb;
            for (int i = 0; i < p.n_dust_sweeps; ++i) {
                timed(ctx, KC_DUST_SWEEP, 7, -1,
                      [&] { O::dust_sweep(L, s, ph, st, yin, yout, G, rj + c * N, rk); });
                std::swap(yin, yout);
            }
            timed(ctx, KC_DUST_FACEFLUX, 7, -1, [&] { O::dust_faceflux(L, s, ph, yin, G); });
            timed(ctx, KC_DUST_FINISH, 5, -1,
                  [&] { O::dust_finish(L, s, ph, st, rj + c * N, G, rj1 + c * N, ctx->part(PS_DUST + c)); });
        }
    }
    step_finish(s, ph, st, ctx->part(PS_MASS), ctx->part(PS_DUST), p.n_classes, L.nblocks,
                Y.max_blocks);

    pisoc_status ss = sync_state(ctx);
    if (ss != PISOC_OK) return ss;
    if (ctx->prof.on) ctx->prof.resolve(kIterInf);
    const DevState& h = *ctx->hst;
    flags |= h.flags;
    if (h.flags & PISOC_FLAG_BAD_DT) {
        ctx->err = "time step undefined or non-positive";
        return PISOC_ERR_INVALID;
    }
    bool bad = (h.flags & (PISOC_FLAG_NONFINITE | PISOC_FLAG_RHO_NONPOS)) != 0;
    for (int c = 0; c < p.n_classes; ++c)
        if (!std::isfinite(h.mass_p[c])) bad = true;
    if (bad) {
        ctx->err = "step diverged (non-finite field or non-positive density); state kept";
        if (info) {
            rec.flags = flags | PISOC_FLAG_NONFINITE;
            rec.dt = h.dt;
            rec.t = ctx->t;
            *info = rec;
        }
        return PISOC_ERR_DIVERGED;
    }
    // commit
    std::swap(ctx->rn, ctx->rk);
    std::swap(ctx->phin, ctx->phik);
    std::swap(ctx->u_idx[0], ctx->u_idx[ucur_slot]);
    if (p.n_classes > 0) std::swap(ctx->rhop, ctx->rhop1);
    ctx->t += h.dt;
    ctx->dt_prev = h.dt;
    ctx->steps += 1;
    rec.t = ctx->t;
    rec.dt = h.dt;
    rec.courant = h.sigma * h.dt;
    rec.flags = flags;
    rec.mass_gas = h.mass_gas;
    for (int c = 0; c < p.n_classes; ++c) rec.mass_p[c] = h.mass_p[c];
    if (info) *info = rec;
    return worst;
}

}  // namespace

// ============================================================ C ABI
extern "C" {

size_t pisoc_workspace_bytes(const pisoc_params* prm) {
    if (!valid_params(prm, nullptr)) return 0;
    return make_layout(prm).total;
}

const char* pisoc_status_string(pisoc_status st) {
    switch (st) {
        case PISOC_OK: return "ok";
        case PISOC_WARN_NOT_CONVERGED: return "pressure solve did not converge";
        case PISOC_WARN_GUESS_FALLBACK: return "learned guess rejected";
        case PISOC_ERR_INVALID: return "invalid argument";
        case PISOC_ERR_HIP: return "HIP error";
        case PISOC_ERR_DIVERGED: return "diverged";
        case PISOC_ERR_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

pisoc_status pisoc_init(const pisoc_params* prm, void* d_workspace, size_t ws_bytes,
                        const double* d_rho, const double* d_u, const double* d_rho_p,
                        void* hip_stream, pisoc_ctx** out) {
    if (!out) return PISOC_ERR_INVALID;
    *out = nullptr;
    std::string why;
    if (!valid_params(prm, &why)) return PISOC_ERR_INVALID;
    if (!d_rho || !d_u || (prm->n_classes > 0 && !d_rho_p)) return PISOC_ERR_INVALID;
    Layout lay = make_layout(prm);
    if (!d_workspace || ws_bytes < lay.total ||
        (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return PISOC_ERR_WORKSPACE;

    pisoc_ctx* ctx = new (std::nothrow) pisoc_ctx();
    if (!ctx) return PISOC_ERR_INVALID;
    ctx->prm = *prm;
    ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
    ctx->ws = reinterpret_cast<char*>(d_workspace);
    ctx->lay = lay;
    ctx->L = make_launch(prm->n);
    ctx->TL = make_tiled_launch(prm->n);
    // PISOC_UNTILED=1 selects the untiled CG kernel (kernel-comparison tests)
    if (const char* e = std::getenv("PISOC_UNTILED"); e && e[0] == '1') ctx->TL = Launch{};
    ctx->st = reinterpret_cast<DevState*>(ctx->ws + lay.state);
    ctx->partials = reinterpret_cast<double*>(ctx->ws + lay.partials);
    ctx->u_idx[0] = 0;
    ctx->u_idx[1] = 1;
    ctx->u_idx[2] = 2;
    ctx->rn = lay.rn;
    ctx->rk = lay.rk;
    ctx->phin = lay.phin;
    ctx->phik = lay.phik;
    ctx->rhop = lay.rhop;
    ctx->rhop1 = lay.rhop1;
    ctx->t = 0.0;
    ctx->dt_prev = __builtin_inf();
    ctx->steps = 0;
    ctx->es = prm->precision == PISOC_FP64 ? sizeof(double) : sizeof(float);
    ctx->prof.reset();
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&ctx->hst), sizeof(DevState),
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
        delete ctx;
        return PISOC_ERR_HIP;
    }
    auto fail = [&](pisoc_status st) {
        pisoc_destroy(ctx);
        return st;
    };
    hipStream_t s = ctx->stream;
    const size_t N = ctx->N();
    if (hipMemsetAsync(ctx->st, 0, sizeof(DevState), s) != hipSuccess) return fail(PISOC_ERR_HIP);

    // reference density = mean of the initial density (FP64 reduction of the input)
    Phys ph0 = make_phys(prm, 1.0);
    Ops<double>::sum_affine_sq(ctx->L, s, ph0, d_rho, 0.0, 0.0, ctx->part(PS_STAT));
    finalize_sums(s, ctx->part(PS_STAT), ctx->L.nblocks, 2, ctx->st->red);
    if (sync_state(ctx) != PISOC_OK) return fail(PISOC_ERR_HIP);
    const double rho_ref = ctx->hst->red[1] / (double)N;
    if (!(rho_ref > 0.0) || !std::isfinite(rho_ref)) return fail(PISOC_ERR_INVALID);
    ctx->ph = make_phys(prm, rho_ref);

    DevState init{};
    init.pcg.tol2 = prm->p_tol * prm->p_tol;
    init.pcg.maxit = prm->p_maxit;
    init.pcg.it_stop = kIterInf;
    *ctx->hst = init;
    if (hipMemcpyAsync(ctx->st, ctx->hst, sizeof(DevState), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(PISOC_ERR_HIP);

    auto convert = [&](auto tag) {
        using T = decltype(tag);
        Ops<T>::cast_in(s, d_rho, ctx->f<T>(ctx->rn), N, rho_ref);
        Ops<T>::cast_in(s, d_u, ctx->f<T>(lay.u3[0]), 3 * N, 0.0);
        if (prm->n_classes > 0)
            Ops<T>::cast_in(s, d_rho_p, ctx->f<T>(ctx->rhop), (size_t)prm->n_classes * N, 0.0);
        Ops<T>::init_phi(ctx->L, s, ctx->ph, ctx->f<T>(ctx->rn), ctx->f<T>(lay.u3[0]),
                         ctx->f<T>(ctx->phin));
    };
    if (prm->precision == PISOC_FP64) convert(double{});
    else convert(float{});
    if (prm->guess == PISOC_GUESS_LEARNED)
        net_pack_forward(s, reinterpret_cast<const float*>(prm->d_guess_weights), ctx->ws + lay.wpk);
    if (sync_state(ctx) != PISOC_OK) return fail(PISOC_ERR_HIP);
    *out = ctx;
    return PISOC_OK;
}

pisoc_status pisoc_step(pisoc_ctx* ctx, int32_t n_steps, pisoc_step_info* h_info) {
    if (!ctx || n_steps < 0) return PISOC_ERR_INVALID;
    pisoc_status worst = PISOC_OK;
    for (int i = 0; i < n_steps; ++i) {
        pisoc_status s = ctx->prm.precision == PISOC_FP64
                             ? one_step<double>(ctx, h_info ? h_info + i : nullptr)
                             : one_step<float>(ctx, h_info ? h_info + i : nullptr);
        if (s < 0) return s;
        if (s > worst) worst = s;
    }
    return worst;
}

pisoc_status pisoc_fields(pisoc_ctx* ctx, uint32_t which, double* const* d_dst) {
    if (!ctx || !d_dst) return PISOC_ERR_INVALID;
    const size_t N = ctx->N();
    hipStream_t s = ctx->stream;
    const bool f64 = ctx->prm.precision == PISOC_FP64;
    int slot = 0;
    auto cast = [&](size_t off, double* dst, size_t count, double shift) {
        if (f64) Ops<double>::cast_out(s, ctx->f<double>(off), dst, count, shift);
        else Ops<float>::cast_out(s, ctx->f<float>(off), dst, count, shift);
    };
    const double* snap = ctx->prm.capture ? reinterpret_cast<double*>(ctx->ws + ctx->lay.snap)
                                          : nullptr;
    for (int bit = 0; bit < 32; ++bit) {
        const uint32_t m = 1u << bit;
        if (!(which & m)) continue;
        double* dst = d_dst[slot++];
        if (!dst) return PISOC_ERR_INVALID;
        switch (m) {
            case PISOC_FIELD_RHO: cast(ctx->rn, dst, N, ctx->ph.rho_ref); break;
            case PISOC_FIELD_U: cast(ctx->lay.u3[ctx->u_idx[0]], dst, 3 * N, 0.0); break;
            case PISOC_FIELD_PHI: cast(ctx->phin, dst, 3 * N, 0.0); break;
            case PISOC_FIELD_RHO_P:
                if (ctx->prm.n_classes > 0)
                    cast(ctx->rhop, dst, (size_t)ctx->prm.n_classes * N, 0.0);
                break;
            case PISOC_FIELD_P:
                if (f64) Ops<double>::pressure_out(s, ctx->ph, ctx->f<double>(ctx->rn), dst);
                else Ops<float>::pressure_out(s, ctx->ph, ctx->f<float>(ctx->rn), dst);
                break;
            case PISOC_FIELD_PSOLVE_B:
            case PISOC_FIELD_PSOLVE_DIAG:
            case PISOC_FIELD_P_PREV:
            case PISOC_FIELD_PSOLVE_X: {
                if (!snap) {
                    ctx->err = "captured pressure system requested without params.capture";
                    return PISOC_ERR_INVALID;
                }
                const int idx = m == PISOC_FIELD_PSOLVE_B ? 0
                                : m == PISOC_FIELD_PSOLVE_DIAG ? 1
                                : m == PISOC_FIELD_P_PREV ? 2 : 3;
                HIP_TRY(ctx, hipMemcpyAsync(dst, snap + idx * N, N * sizeof(double),
                                            hipMemcpyDeviceToDevice, s));
                break;
            }
            default: ctx->err = "unknown field bit"; return PISOC_ERR_INVALID;
        }
    }
    HIP_TRY(ctx, hipGetLastError());
    return PISOC_OK;
}

pisoc_status pisoc_get_stats(pisoc_ctx* ctx, pisoc_stats* out) {
    if (!ctx || !out) return PISOC_ERR_INVALID;
    std::memset(out, 0, sizeof(*out));
    const double N = (double)ctx->N();
    const Phys& ph = ctx->ph;
    hipStream_t s = ctx->stream;
    const bool f64 = ctx->prm.precision == PISOC_FP64;
    auto gas = [&](auto tag) {
        using T = decltype(tag);
        Ops<T>::stats_gas(ctx->L, s, ph, ctx->f<T>(ctx->rn), ctx->f<T>(ctx->lay.u3[ctx->u_idx[0]]),
                          ctx->part(PS_STAT));
        finalize_sums(s, ctx->part(PS_STAT), ctx->L.nblocks, 4, ctx->st->red);
    };
    auto affine = [&](auto tag, size_t off, double a, double b) {
        using T = decltype(tag);
        Ops<T>::sum_affine_sq(ctx->L, s, ph, ctx->f<T>(off), a, b, ctx->part(PS_STAT));
        finalize_sums(s, ctx->part(PS_STAT), ctx->L.nblocks, 2, ctx->st->red + 4);
    };
    if (f64) gas(double{}); else gas(float{});
    pisoc_status st = sync_state(ctx);
    if (st != PISOC_OK) return st;
    const double ke = ctx->hst->red[0], ens = ctx->hst->red[1], usq = ctx->hst->red[2],
                 rsum = ctx->hst->red[3];
    const double rbar = rsum / N;
    if (f64) affine(double{}, ctx->rn, 1.0, -rbar); else affine(float{}, ctx->rn, 1.0, -rbar);
    if ((st = sync_state(ctx)) != PISOC_OK) return st;
    const double rvar = ctx->hst->red[4];
    const double rmean = ph.rho_ref + rbar;
    out->ke = ke / N;
    out->enstrophy = ens / N;
    out->rho_rms = std::sqrt(rvar / N) / rmean;
    const double c0 = std::sqrt(ph.gamma * ph.C * std::pow(rmean, ph.gamma - 1.0));
    out->mach_rms = std::sqrt(usq / N) / c0;
    out->mass_gas = rmean * N * ph.V;
    const size_t Nc = ctx->N();
    for (int c = 0; c < ctx->prm.n_classes; ++c) {
        const size_t off = ctx->rhop + (f64 ? sizeof(double) : sizeof(float)) * Nc * c;
        if (f64) affine(double{}, off, 0.0, 0.0); else affine(float{}, off, 0.0, 0.0);
        if ((st = sync_state(ctx)) != PISOC_OK) return st;
        const double m = ctx->hst->red[5] / N;
        if (m != 0.0) {
            if (f64) affine(double{}, off, 1.0 / m, -1.0); else affine(float{}, off, 1.0 / m, -1.0);
            if ((st = sync_state(ctx)) != PISOC_OK) return st;
            out->conc_var[c] = ctx->hst->red[4] / N;
        }
        out->mass_p[c] = m * N * ph.V;
    }
    return PISOC_OK;
}

pisoc_status pisoc_profile(pisoc_ctx* ctx, int32_t enable) {
    if (!ctx) return PISOC_ERR_INVALID;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return PISOC_ERR_HIP;
    ctx->prof.reset();
    ctx->prof.on = enable != 0;
    return PISOC_OK;
}

int32_t pisoc_profile_read(const pisoc_ctx* ctx, pisoc_kernel_stat* out, int32_t max) {
    if (!ctx || !out) return 0;
    int32_t n = 0;
    for (int i = 0; i < KC_COUNT && n < max; ++i)
        if (ctx->prof.stat[i].launches > 0) out[n++] = ctx->prof.stat[i];
    return n;
}

double pisoc_time(const pisoc_ctx* ctx) { return ctx ? ctx->t : 0.0; }
int64_t pisoc_steps_done(const pisoc_ctx* ctx) { return ctx ? ctx->steps : 0; }

void pisoc_destroy(pisoc_ctx* ctx) {
    if (!ctx) return;
    if (ctx->hst) (void)hipHostFree(ctx->hst);
    delete ctx;
}

const char* pisoc_last_error(const pisoc_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

// ---------------------------------------------------------------- Helmholtz
static Layout helm_layout(int32_t n) {
    Layout L{};
    const size_t N = (size_t)n * n * n;
    const Launch lc = make_launch(n);
    L.max_blocks = std::max(lc.nblocks, make_tiled_launch(n).nblocks);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.state = take(sizeof(DevState));
    L.partials = take(sizeof(double) * PS_COLUMNS * (size_t)L.max_blocks);
    L.r = take(8 * N);
    L.diag = take(8 * N);
    L.pp0 = take(8 * N);
    L.pp1 = take(8 * N);
    L.q = take(8 * N);
    L.total = off;
    return L;
}

size_t pisoc_helm_workspace_bytes(int32_t n) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N) return 0;
    return helm_layout(n).total;
}

pisoc_status pisoc_helm_apply(int32_t n, const double* d_psidt, const double* d_w,
                              const double* d_x, double* d_y, void* hip_stream) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_psidt || !d_w || !d_x || !d_y)
        return PISOC_ERR_INVALID;
    pisoc_params p{};
    p.n = n;
    p.gamma = 1.4;
    p.C = 1.0;
    Phys ph = make_phys(&p, 1.0);
    Launch L = make_launch(n);
    Ops<double>::helm_apply(L, reinterpret_cast<hipStream_t>(hip_stream), ph, d_psidt, d_w, d_x, d_y);
    return hipGetLastError() == hipSuccess ? PISOC_OK : PISOC_ERR_HIP;
}

pisoc_status pisoc_helm_solve(int32_t n, const double* d_psidt, const double* d_w,
                              const double* d_b, double* d_x, double tol, int32_t maxit,
                              void* d_workspace, size_t ws_bytes, void* hip_stream,
                              int32_t* iters, double* relres) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_psidt || !d_w || !d_b || !d_x ||
        !(tol > 0.0) || !(tol < 1.0) || maxit < 1)
        return PISOC_ERR_INVALID;
    Layout lay = helm_layout(n);
    if (!d_workspace || ws_bytes < lay.total ||
        (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return PISOC_ERR_WORKSPACE;
    pisoc_ctx ctx{};
    ctx.prm.n = n;
    ctx.prm.p_maxit = maxit;
    ctx.prm.gamma = 1.4;
    ctx.prm.C = 1.0;
    ctx.stream = reinterpret_cast<hipStream_t>(hip_stream);
    ctx.ws = reinterpret_cast<char*>(d_workspace);
    ctx.lay = lay;
    ctx.ph = make_phys(&ctx.prm, 1.0);
    ctx.L = make_launch(n);
    ctx.TL = make_tiled_launch(n);
    ctx.st = reinterpret_cast<DevState*>(ctx.ws + lay.state);
    ctx.partials = reinterpret_cast<double*>(ctx.ws + lay.partials);
    if (hipHostMalloc(reinterpret_cast<void**>(&ctx.hst), sizeof(DevState), hipHostMallocDefault) !=
        hipSuccess)
        return PISOC_ERR_HIP;
    DevState init{};
    init.pcg.tol2 = tol * tol;
    init.pcg.maxit = maxit;
    init.pcg.it_stop = kIterInf;
    *ctx.hst = init;
    pisoc_status st = PISOC_OK;
    if (hipMemcpyAsync(ctx.st, ctx.hst, sizeof(DevState), hipMemcpyHostToDevice, ctx.stream) !=
        hipSuccess) {
        st = PISOC_ERR_HIP;
    } else {
        double* r = ctx.f<double>(lay.r);
        double* dg = ctx.f<double>(lay.diag);
        Ops<double>::helm_start(ctx.L, ctx.stream, ctx.ph, ctx.st, d_psidt, d_w, d_b, d_x, r, dg,
                                ctx.part(PS_U));
        int32_t it = 0;
        double rel = 0.0;
        bool conv = false;
        st = run_pcg<double>(&ctx, r, d_x, dg, const_cast<double*>(d_w), ctx.f<double>(lay.pp0),
                             ctx.f<double>(lay.pp1), ctx.f<double>(lay.q), tol, 16, &it, &rel,
                             &conv);
        if (st == PISOC_OK) {
            if (iters) *iters = it;
            if (relres) *relres = rel;
            if (!conv) st = PISOC_WARN_NOT_CONVERGED;
        }
    }
    (void)hipHostFree(ctx.hst);
    ctx.hst = nullptr;
    return st;
}

pisoc_status pisoc_net_inputs(int32_t n, const double* d_b, const double* d_diag,
                              const double* d_p0, const double* d_psol, float* d_x, float* d_t,
                              double* h_scales, void* d_workspace, size_t ws_bytes,
                              void* hip_stream) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_b || !d_diag || !d_p0 || !d_x ||
        (d_t && !d_psol))
        return PISOC_ERR_INVALID;
    Layout lay = helm_layout(n);
    if (!d_workspace || ws_bytes < lay.total ||
        (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return PISOC_ERR_WORKSPACE;
    pisoc_params p{};
    p.n = n;
    p.gamma = 1.4;
    p.C = 1.0;
    Phys ph = make_phys(&p, 1.0);
    Launch L = make_launch(n);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    char* ws = reinterpret_cast<char*>(d_workspace);
    DevState* st = reinterpret_cast<DevState*>(ws + lay.state);
    double* part = reinterpret_cast<double*>(ws + lay.partials) + (size_t)PS_STAT * lay.max_blocks;
    Ops<double>::net_stats(L, s, ph, d_b, d_diag, d_p0, part);
    Ops<double>::net_input(L, s, ph, st, part, d_b, d_diag, d_p0, nullptr, d_x, d_psol, d_t);
    if (hipGetLastError() != hipSuccess) return PISOC_ERR_HIP;
    if (h_scales) {
        if (hipMemcpyAsync(h_scales, &st->red[6], 2 * sizeof(double), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PISOC_ERR_HIP;
    }
    return PISOC_OK;
}

}  // extern "C"
