// pisoc.hip -- host orchestration of the PISO step and the C ABI (pisoc.h).
//
// The library owns no device memory: every field, the CG vectors, the
// reduction partials and the device-side state live in the caller's
// workspace.
//
// A context holds `batch` members of one grid size stacked along z: every
// kernel covers all of them in one launch, and every per-member quantity (dt,
// the reference density and pressure, particle response times, the CG state)
// lives in the member's DevState.  Two ways of running a step share one launch
// sequence:
//  - eager (pisoc_step, the ensemble's calibration): the host waits on the
//    stream only to learn when every member's pressure solve has stopped (one
//    wait per batch of CG iterations, sized from the previous solve), between
//    FP64 refinement rounds, and at the end of the step to check it before
//    committing it;
//  - captured (ensembles): CG to a fixed iteration cap with early exit per
//    member, a fixed number of refinement rounds, the commit on the device;
//    captured once per buffer parity into one HIP graph for all size classes
//    (one branch per class) and replayed, one graph launch per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
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
constexpr unsigned kMaxTuneBlocks = 4096;   // blocks per member of a launch-shape candidate

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Launch-shape candidates of the field kernels for grid size n: (bx, cz).
std::vector<std::pair<int, int>> shape_candidates(int n) {
    std::vector<std::pair<int, int>> out;
    for (int bx : {16, 32, 64, 128}) {
        if (bx > 2 * n) continue;
        for (int cz : {1, 2, 4, 8, 16}) {
            if (cz > n) continue;
            const Launch L = make_launch_shaped(n, 1, bx, cz);
            if (L.nblocks <= kMaxTuneBlocks) out.push_back({bx, cz});
        }
    }
    return out;
}

// Byte offsets of every buffer inside the workspace (all members of a batch).
struct Layout {
    size_t state, partials;
    size_t rn, rk, aP, divu, pn, w, p0, r, r2, x, diag, pp0, pp1, pp2, q, q2, Y0, Y1;
    size_t u3[3], phin, phik, src, hbya, phiH, acc, G;
    size_t rhop, rhop1;
    size_t fd0, fd1, fm;   // two-way coupling: dust mass fluxes (two rotating), mixture flux
    // FP64 fields when capturing: b, diag, p0, p', w = rho/a_P (snapshot slots
    // 0-4), u* (5-7), and with the learned guess g and the solve start x0 (8, 9)
    size_t snap;
    size_t b64, x64a, x64b, xf;  // FP64 refinement fields, FP32 solution copy (FP32 storage only)
    size_t wpk, nx4, na, nb, ny, bsave;  // learned guess: packed weights, activations
    size_t xprev;  // previous-step guess: each corrector's last solution
    size_t t0, t1, tw, eaT, esT;  // Fourier closure: T (two rotating), sweep scratch, a_T, s_T
    size_t rm1, um1, rjm1;        // BDF2: rho, u, rho_j at t^{n-1}
    size_t bicg;                  // momentum BiCGStab: r, rh, p, v, y, s, z, t (3 N each)
    size_t total;
    unsigned max_blocks;     // column length of the partials (all members)
};

// Kernel classes for the optional per-launch event timing.
enum KCls {
    KC_CFL, KC_PREDICT, KC_MOM_SOURCE, KC_MOM_SWEEP, KC_HBYA, KC_CORR_RHS, KC_PCG_SPMV,
    KC_CORR_FLUX, KC_CORR_UPDATE, KC_DUDT, KC_DUST_FLUX, KC_DUST_SWEEP,
    KC_DUST_FACEFLUX, KC_DUST_FINISH, KC_REFINE, KC_NET, KC_MIXTURE, KC_PREV_GUESS, KC_COUNT
};
const char* const kKernelName[KC_COUNT] = {
    "k_cfl", "k_predict", "k_mom_source", "k_mom_sweep", "k_hbya", "k_corr_rhs",
    "k_pcg_spmv", "k_corr_flux", "k_corr_update", "k_dudt", "k_dust_flux",
    "k_dust_sweep", "k_dust_faceflux", "k_dust_finish", "k_refine", "learned_guess",
    "k_mixture", "previous_guess"};

struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    // k: CG iteration (-1 for other kernels); stop_bytes: what the CG launch
    // moves if the solve stops at it (the last x update)
    struct Rec { int cls; size_t ea, eb; double bytes; int k; double stop_bytes; };
    std::vector<Rec> pending;
    pisoc_kernel_stat stat[KC_COUNT];

    // timing-only events: recorded without the system-scope fence (its L2
    // write-back and invalidation would be charged to the bracketed kernel
    // and cool the cache for the next one); their times are read after a
    // stream synchronisation
    size_t take() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
                return (size_t)-1;
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
    // Attribute completed launches.  CG launch k < it_stop is an iteration;
    // k == it_stop made the solve's last x update (its stop_bytes); later ones
    // returned at once.  Records sharing one pair of events are a run of
    // back-to-back launches of one class: the run's time goes to its working
    // launches (those that returned at once inside it are charged to them).
    void resolve(int it_stop) {
        for (size_t i = 0; i < pending.size();) {
            const Rec& r0 = pending[i];
            size_t j = i;
            int working = 0;
            double bytes = 0.0;
            for (; j < pending.size() && pending[j].ea == r0.ea && pending[j].eb == r0.eb; ++j) {
                const Rec& r = pending[j];
                if (r.k < 0 || r.k < it_stop) {
                    working += 1;
                    bytes += r.bytes;
                } else if (r.k == it_stop && r.stop_bytes > 0.0) {
                    working += 1;
                    bytes += r.stop_bytes;
                }
            }
            float ms = 0.f;
            // the GPU is past both events (see sync_state); the wait only
            // lets the runtime see it
            if (working > 0 && hipEventSynchronize(pool[r0.eb]) == hipSuccess &&
                hipEventElapsedTime(&ms, pool[r0.ea], pool[r0.eb]) == hipSuccess) {
                stat[r0.cls].launches += working;
                stat[r0.cls].ms += ms;
                stat[r0.cls].bytes += bytes;
            }
            i = j;
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
    if (p->guess != PISOC_GUESS_ZERO && p->guess != PISOC_GUESS_LEARNED &&
        p->guess != PISOC_GUESS_PREVIOUS)
        return fail("unknown guess");
    if (p->guess == PISOC_GUESS_LEARNED && (!p->d_guess_weights || p->n % 16 != 0))
        return fail("learned guess needs d_guess_weights and n % 16 == 0");
    if (p->guess_audit < 0) return fail("guess_audit must be >= 0");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->gravity[d])) return fail("gravity must be finite");
    if (p->closure != PISOC_BAROTROPIC && p->closure != PISOC_FOURIER) return fail("unknown closure");
    if (p->time_scheme != PISOC_BDF1 && p->time_scheme != PISOC_BDF2) return fail("unknown time scheme");
    if (!(p->mom_tol >= 0.0) || !(p->mom_tol < 1.0)) return fail("mom_tol must be in [0, 1)");
    if (p->mom_tol > 0.0 && (p->mom_maxit < 1 || p->precision != PISOC_FP64))
        return fail("a tolerance-solved momentum predictor needs mom_maxit >= 1 and FP64");
    if (p->time_scheme == PISOC_BDF2 &&
        (p->precision != PISOC_FP64 || p->closure != PISOC_BAROTROPIC || p->two_way))
        return fail("BDF2 needs FP64, the barotropic closure and two_way = 0");
    if (p->closure == PISOC_FOURIER) {
        if (!(p->R_gas > 0.0) || !(p->cv > 0.0) || !(p->kappa >= 0.0) || !(p->T0 > 0.0))
            return fail("Fourier closure needs R_gas > 0, cv > 0, kappa >= 0 and T0 > 0");
        if (p->precision != PISOC_FP64) return fail("Fourier closure needs FP64");
        if (p->two_way) return fail("Fourier closure with two_way is not supported");
    }
    return true;
}

Layout make_layout(const pisoc_params* p, int batch) {
    Layout L{};
    const size_t N = (size_t)p->n * p->n * p->n * (size_t)batch;
    const size_t es = p->precision == PISOC_FP64 ? sizeof(double) : sizeof(float);
    unsigned mb = std::max({make_launch(p->n, batch).nblocks, make_tiled_launch(p->n, batch).nblocks,
                            make_spmv_launch(p->n, batch, (int)es).nblocks});
    for (int c : {8, 16, 32}) {   // the chunks the autotuner may choose
        mb = std::max(mb, make_spmv_launch(p->n, batch, (int)es, c).nblocks);
        mb = std::max(mb, make_tiled_launch(p->n, batch, c).nblocks);
    }
    for (auto [bx, cz] : shape_candidates(p->n))
        mb = std::max(mb, make_launch_shaped(p->n, batch, bx, cz).nblocks);
    L.max_blocks = mb;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.state = take(sizeof(DevState) * (size_t)batch);
    L.partials = take(sizeof(double) * PS_COLUMNS * (size_t)L.max_blocks);
    size_t* one[] = {&L.rn, &L.rk, &L.aP, &L.divu, &L.pn, &L.w, &L.p0, &L.r, &L.r2, &L.x,
                     &L.diag, &L.pp0, &L.pp1, &L.pp2, &L.q, &L.q2, &L.Y0, &L.Y1};
    for (size_t* o : one) *o = take(es * N);
    size_t* three[] = {&L.u3[0], &L.u3[1], &L.u3[2], &L.phin, &L.phik, &L.src, &L.hbya,
                       &L.phiH, &L.acc, &L.G};
    for (size_t* o : three) *o = take(3 * es * N);
    L.rhop = take(es * N * (size_t)std::max(p->n_classes, 1));
    L.rhop1 = take(es * N * (size_t)std::max(p->n_classes, 1));
    if (p->two_way) {
        L.fd0 = take(3 * es * N);
        L.fd1 = take(3 * es * N);
        L.fm = take(3 * es * N);
    }
    L.snap = p->capture ? take((p->guess != PISOC_GUESS_ZERO ? 10 : 8) * sizeof(double) * N)
                        : 0;
    if (p->mom_tol > 0.0) L.bicg = take(8 * 3 * es * N);
    if (p->time_scheme == PISOC_BDF2) {   // FP64 only
        L.rm1 = take(sizeof(double) * N);
        L.um1 = take(3 * sizeof(double) * N);
        L.rjm1 = take(sizeof(double) * N * (size_t)std::max(p->n_classes, 1));
    }
    if (p->closure == PISOC_FOURIER) {   // FP64 only
        L.t0 = take(sizeof(double) * N);
        L.t1 = take(sizeof(double) * N);
        L.tw = take(sizeof(double) * N);
        L.eaT = take(sizeof(double) * N);
        L.esT = take(sizeof(double) * N);
    }
    if (p->guess == PISOC_GUESS_PREVIOUS) {
        // each corrector's solution of the last step, and the saved b of a fallback
        L.xprev = take(es * N * (size_t)p->n_corr);
        L.bsave = take(es * N);
    }
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
        L.xf = take(sizeof(float) * N);
    }
    L.total = off;
    return L;
}

}  // namespace

struct pisoc_ctx {
    pisoc_params prm;
    int batch = 1;
    hipStream_t stream;
    char* ws;
    Layout lay;
    Phys ph;
    Launch L;
    Launch TL;      // tiled z-marching launch of the field kernels (nblocks = 0: none)
    unsigned nb_start = 0;   // partials in PS_U of the current solve's start (its set-up kernel)
    unsigned nb_mass = 0;    // partials in PS_MASS (the last corrector update)
    // Courant partials of the current state: nb_cfl of them at cfl_part,
    // written by k_cfl (PS_CFL) or, when cfl_ready, by the final corrector
    // pass of the last accepted eager step (the column after the mass
    // partials); nb_cfl_next: that pass in the step being enqueued (0: none)
    bool cfl_ready = false;
    unsigned nb_cfl = 0, nb_cfl_next = 0;
    const double* cfl_part = nullptr;
    Launch TS;      // tiled launch of the CG kernel (nblocks = 0: none)
    DevState* st;
    DevState* hst = nullptr;  // pinned host copy (batch entries)
    // publication of the state without a copy engine (see sync_state): hst is
    // coherent host memory followed by a sequence number; hst_dev, seq_dev
    // their device addresses (null: the plain copy and stream sync)
    DevState* hst_dev = nullptr;
    unsigned long long* seq_host = nullptr;
    unsigned long long* seq_dev = nullptr;
    unsigned long long seq = 0;
    double* partials;
    // rotating buffers
    int u_idx[3];   // which of lay.u3 holds u^n, work a, work b
    int ucur_slot;  // u_idx slot holding u* after the predictor sweeps (1 or 2)
    size_t rn, rk, phin, phik, rhop, rhop1;
    size_t fdn, fdk;   // two-way coupling: dust mass fluxes of the last step / this one
    size_t tn, tk;     // Fourier closure: T^n / T* of the step being enqueued
    size_t rm1, um1, rjm1;   // BDF2: the state at t^{n-1}
    double t;
    int64_t steps;
    int pred_first[PISOC_MAX_CORR];  // CG iterations of the last first solve (all members)
    int pred_later;                  // ... of the last later refinement round
    // captured mode: CG pairs per first solve, per later round, refinement rounds
    // (tracked over the steps), and those the current graphs were built with
    int caps[PISOC_MAX_CORR];
    int cap_later;
    int rounds;
    int caps_built[PISOC_MAX_CORR];
    int cap_later_built;
    size_t es;      // bytes per field element (8 or 4)
    // learned-guess audit of eager steps (guess_audit > 0): running means of the
    // CG iterations of each corrector's solve with and without the guess, and
    // of the guess's cost in CG-iteration equivalents (timed with events);
    // < 0: not measured yet
    struct Audit {
        double it_zero[PISOC_MAX_CORR], it_guess[PISOC_MAX_CORR];
        double cost;
        bool use[PISOC_MAX_CORR];   // this step's choice
        int64_t steps;
        // probes of the choice the verdict rejects: the next one at step
        // next_probe; the interval doubles (up to kMaxProbeFactor guess_audit)
        // while probes confirm the verdict, and starts again at guess_audit
        // when one overturns it
        int64_t next_probe, period;
        bool probing, verdict[PISOC_MAX_CORR];
        hipEvent_t ev[PISOC_MAX_CORR][3];
        bool have_events;
    } audit;
    Prof prof;
    std::string err;
    std::vector<double> rho_ref, p_ref;  // per member

    template <typename T> T* f(size_t off) const { return reinterpret_cast<T*>(ws + off); }
    size_t N() const { return (size_t)prm.n * prm.n * prm.n; }
    size_t NT() const { return N() * (size_t)batch; }
    // partial-sum column `slot` (max_blocks doubles per column)
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
    P.pending.push_back({cls, a, b, words * (double)ctx->es * (double)ctx->NT(), k, 0.0});
}

// The device state published to the host: one wavefront copies the records
// into the coherent pinned buffer, waits for its stores to complete at system
// scope, then stores the sequence number v (release, system scope).  After
// every earlier launch on the stream, so seeing v means those have finished.
__global__ void __launch_bounds__(64) k_publish(const unsigned long long* __restrict__ src,
                                                unsigned long long* dst, unsigned words,
                                                unsigned long long* seq, unsigned long long v) {
    for (unsigned i = threadIdx.x; i < words; i += 64) dst[i] = src[i];
    __threadfence_system();
    if (threadIdx.x == 0) __hip_atomic_store(seq, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Bring the device state to ctx->hst once the stream's work so far is done.
// With the publication buffer the host spins on the sequence number (no copy
// engine, no sleep in the runtime's wait: the GPU stays idle for less time
// between the work before and the launches the host then makes); after
// kPublishSpin without it, the stream sync decides (a long queue, or an
// error on the stream).
constexpr auto kPublishSpin = std::chrono::milliseconds(50);

pisoc_status sync_state(pisoc_ctx* ctx) {
    HIP_TRY(ctx, hipGetLastError());
    if (ctx->seq_host) {
        const unsigned long long v = ++ctx->seq;
        static_assert(sizeof(DevState) % 8 == 0, "DevState is copied in 8-byte words");
        hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, ctx->stream,
                           reinterpret_cast<const unsigned long long*>(ctx->st),
                           reinterpret_cast<unsigned long long*>(ctx->hst_dev),
                           (unsigned)(sizeof(DevState) / 8 * (size_t)ctx->batch), ctx->seq_dev, v);
        HIP_TRY(ctx, hipGetLastError());
        const auto t0 = std::chrono::steady_clock::now();
        for (unsigned spin = 1;; ++spin) {
            if (__atomic_load_n(ctx->seq_host, __ATOMIC_ACQUIRE) == v) return PISOC_OK;
            if ((spin & 1023u) == 0 && std::chrono::steady_clock::now() - t0 > kPublishSpin) break;
            __builtin_ia32_pause();
        }
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        if (__atomic_load_n(ctx->seq_host, __ATOMIC_ACQUIRE) == v) return PISOC_OK;
        ctx->err = "state publication not seen after the stream completed";
        return PISOC_ERR_HIP;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->hst, ctx->st, sizeof(DevState) * (size_t)ctx->batch,
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PISOC_OK;
}

Phys make_phys(const pisoc_params* p, const Launch& L, int batch) {
    Phys ph{};
    ph.n = p->n;
    ph.cz = L.cz;
    ph.nz = L.nz;
    ph.batch = batch;
    ph.N = (size_t)p->n * p->n * p->n;
    ph.NT = ph.N * (size_t)batch;
    ph.h = kTwoPi / p->n;
    ph.inv_h = 1.0 / ph.h;
    ph.inv_h2 = 1.0 / (ph.h * ph.h);
    ph.V = ph.h * ph.h * ph.h;
    ph.inv_V = 1.0 / ph.V;
    ph.A = ph.h * ph.h;
    ph.gamma = p->gamma;
    ph.C = p->C;
    ph.mu = p->mu;
    for (int d = 0; d < 3; ++d) ph.g[d] = p->gravity[d];
    ph.fourier = p->closure == PISOC_FOURIER ? 1 : 0;
    ph.bdf2 = p->time_scheme == PISOC_BDF2 ? 1 : 0;
    ph.R = p->R_gas;
    ph.cv = p->cv;
    ph.kappa = p->kappa;
    return ph;
}

void set_shape(pisoc_ctx* ctx, const Launch& L) {
    ctx->L = L;
    ctx->ph.cz = L.cz;
    ctx->ph.nz = L.nz;
}

// The vectors of one CG solve: r_k, p_k and q_k in r[k & 1], p[k % 3],
// q[k & 1] (the set-up kernel leaves r_0 in r[0]).
template <typename T>
struct CgVecs {
    T *r[2], *p[3], *q[2];
    T *x, *diag, *w;
};

// CG on the system already set up by corr_rhs / helm_start / guess_apply /
// k_refine (which left r_0 and the partials r0.z0, r0.r0, b.b written by
// nb_first blocks), to the tolerance already set in each member's state.
// Launches iterations 0, 1, ...: iteration k tests convergence of r_k, and
// every launch after a member's stop returns at once for that member.  eager:
// iterations in batches, the first batch of `iters` after iteration 0, the
// host waiting after each until every member has stopped; otherwise exactly
// `iters` after iteration 0 (capture).  Returns the largest iteration count
// (eager).  cap > 0: the solve stops at iteration cap at the latest (taking x
// up to date), as at p_maxit.
template <typename T>
pisoc_status run_pcg(pisoc_ctx* ctx, const CgVecs<T>& v, bool fresh, int iters, bool eager,
                     int* iters_max, bool xzero, unsigned nb_first, int cap = 0) {
    using O = Ops<T>;
    const int maxit = cap > 0 ? std::min(cap, ctx->prm.p_maxit) : ctx->prm.p_maxit;
    const unsigned nb_cg = ctx->TS.nblocks ? ctx->TS.nblocks : ctx->L.nblocks;
    auto launch = [&](int k) {
        CgArgs<T> a;
        a.rin = v.r[k == 0 ? 0 : (k + 1) & 1];
        a.rout = v.r[k & 1];
        a.diag = v.diag;
        a.w = v.w;
        a.pold = v.p[(k + 2) % 3];
        a.pold2 = v.p[(k + 1) % 3];
        a.pnew = v.p[k % 3];
        a.qold = v.q[(k + 1) & 1];
        a.q = v.q[k & 1];
        a.x = v.x;
        a.part_in = k == 0 ? ctx->part(PS_U) : ctx->part(PS_CG + kCgCols * ((k + 1) & 1));
        a.nb_in = k == 0 ? nb_first : nb_cg;
        a.part_out = ctx->part(PS_CG + kCgCols * (k & 1));
        a.fresh = fresh ? 1 : 0;
        a.maxit = maxit;
        a.xzero = xzero ? 1 : 0;
        O::pcg_iter(ctx->L, ctx->TS, ctx->stream, ctx->ph, ctx->st, k, a);
    };
    // launches k0..k1-1, back to back; when profiling, bracketed as one run
    // (per-launch events would add their own packets between the launches)
    auto run = [&](int k0, int k1) {
        Prof& pf = ctx->prof;
        const size_t ea = pf.on ? pf.take() : (size_t)-1;
        const size_t eb = pf.on ? pf.take() : (size_t)-1;
        const bool bracket = ea != (size_t)-1 && eb != (size_t)-1;
        if (bracket) (void)hipEventRecord(pf.pool[ea], ctx->stream);
        for (int k = k0; k < k1; ++k) launch(k);
        if (!bracket) return;
        (void)hipEventRecord(pf.pool[eb], ctx->stream);
        // words of an iteration: r, diag, w read, p, q written; from k = 1 also
        // q, p_old read and r written; at even k >= 2 also p_{k-2} read and x
        // updated.  Stopping at k >= 1: x += alpha p_old (odd k) or the two
        // pending updates (even k), x not read while it has not been written
        // (zero start, k <= 2).
        const double cell = (double)ctx->es * (double)ctx->NT();
        for (int k = k0; k < k1; ++k) {
            const double words = k == 0 ? 5.0 : (k & 1) ? 8.0 : 11.0;
            const double xread = xzero && k <= 2 ? 0.0 : 1.0;
            const double stop = k == 0 ? 0.0 : ((k & 1) ? 2.0 : 3.0) + xread;
            pf.pending.push_back({KC_PCG_SPMV, ea, eb, words * cell, k, stop * cell});
        }
    };
    int k = 0;  // iterations launched: 0..k
    if (!eager) {
        const int cap = std::min(std::max(1, iters), maxit);
        run(0, cap + 1);
        return PISOC_OK;
    }
    int batch = std::max(1, iters);
    int most = 0;
    for (bool first = true;; first = false) {
        const int kend = std::min(k + batch, maxit);
        run(first ? 0 : k + 1, kend + 1);
        k = std::max(k, kend);
        pisoc_status s = sync_state(ctx);
        if (s != PISOC_OK) return s;
        bool all = true, bad_dt = false;
        int stop_max = 0;
        for (int m = 0; m < ctx->batch; ++m) {
            all = all && ctx->hst[m].pcg.it_stop != kIterInf;
            stop_max = std::max(stop_max, ctx->hst[m].pcg.it_stop);
            bad_dt = bad_dt || (ctx->hst[m].flags & PISOC_FLAG_BAD_DT);
        }
        // launches with k >= the latest stop did no work for any member
        if (ctx->prof.on) ctx->prof.resolve(all ? stop_max : kIterInf);
        if (all || bad_dt || k >= maxit) break;
        batch = 2;
    }
    for (int m = 0; m < ctx->batch; ++m) most = std::max(most, ctx->hst[m].pcg.iters);
    if (iters_max) *iters_max = most;
    return PISOC_OK;
}

// The initial guess of one pressure solve, every member: the learned one
// (scaled inputs from the system just set up, the network on the matrix cores,
// g = s1 y) or the previous step's solution of the same corrector (g = gprev);
// CG then starts from x0 = alpha g (alpha energy-optimal); a member whose guess
// does not lower ||b - M x0|| below ||b|| falls back to x0 = 0 (decided on the
// device).
template <typename T>
void guess_solve_start(pisoc_ctx* ctx, const T* gprev, T* r, T* x, T* dg, T* w, T* p0, T* gbuf,
                       T* mgbuf) {
    using O = Ops<T>;
    const Layout& Y = ctx->lay;
    const bool f32 = sizeof(T) == sizeof(float);
    hipStream_t s = ctx->stream;
    double* x64 = f32 ? ctx->f<double>(Y.x64a) : nullptr;
    double* b64 = f32 ? ctx->f<double>(Y.b64) : nullptr;
    T* bsave = ctx->f<T>(Y.bsave);
    const bool learned = ctx->prm.guess == PISOC_GUESS_LEARNED;
    timed(ctx, learned ? KC_NET : KC_PREV_GUESS, 2, -1, [&] {
        if (learned) {
            O::net_stats(ctx->L, s, ctx->ph, r, dg, p0, ctx->part(PS_STAT));
            O::net_input(ctx->L, s, ctx->ph, ctx->st, ctx->part(PS_STAT), r, dg, p0,
                         ctx->f<uint16_t>(Y.nx4), nullptr, nullptr, nullptr);
            net_forward(s, ctx->prm.n, ctx->batch, ctx->ws + Y.wpk, ctx->f<uint16_t>(Y.nx4),
                        ctx->f<uint16_t>(Y.na), ctx->f<uint16_t>(Y.nb), ctx->f<float>(Y.ny), 1.f);
        }
        O::guess_start(ctx->L, s, ctx->ph, ctx->st, learned ? ctx->f<float>(Y.ny) : nullptr,
                       learned ? nullptr : gprev, w, dg, r, b64, gbuf, mgbuf, ctx->part(PS_STAT));
        O::guess_apply(ctx->L, s, ctx->ph, ctx->st, ctx->part(PS_STAT), gbuf, mgbuf, dg, r, x,
                       x64, b64, bsave, ctx->part(PS_U));
        // totals of r0.z0, ||r0||^2, ||b||^2 into red[0..2], then the fallback test
        finalize_sums(s, ctx->part(PS_U), ctx->L.nblocks, ctx->batch, 3, ctx->st, 0);
        O::guess_revert(ctx->L, s, ctx->ph, ctx->st, r, x, x64, b64, bsave, dg, ctx->part(PS_U));
    });
}

// Pointers of the current buffer rotation.
template <typename T>
struct StepPtrs {
    T *rn, *rk, *un, *ua, *ub, *phin, *phik;
    T *aP, *divu, *pn, *src, *hb, *w, *p0, *phiH, *r, *r2, *x, *dg, *pp0, *pp1, *pp2, *q, *q2;
    T *acc, *G, *Ya, *Yb, *rj, *rj1;
    // two-way coupling: dust fluxes of the last step and of this one, the
    // mixture flux; mflux: the momentum equation's convecting flux (phin or fm)
    T *fdn, *fdk, *fm, *mflux;
    double *snap, *b64, *x64a, *x64b;
    T* xf;   // FP32: the refinement's rounded solution (exchanged with x after a solve)
};

template <typename T>
StepPtrs<T> step_ptrs(const pisoc_ctx* ctx) {
    const Layout& Y = ctx->lay;
    auto F = [&](size_t off) { return ctx->f<T>(off); };
    StepPtrs<T> P;
    P.rn = F(ctx->rn);
    P.rk = F(ctx->rk);
    P.un = F(Y.u3[ctx->u_idx[0]]);
    P.ua = F(Y.u3[ctx->u_idx[1]]);
    P.ub = F(Y.u3[ctx->u_idx[2]]);
    P.phin = F(ctx->phin);
    P.phik = F(ctx->phik);
    P.aP = F(Y.aP);
    P.divu = F(Y.divu);
    P.pn = F(Y.pn);
    P.src = F(Y.src);
    P.hb = F(Y.hbya);
    P.w = F(Y.w);
    P.p0 = F(Y.p0);
    P.phiH = F(Y.phiH);
    P.r = F(Y.r);
    P.r2 = F(Y.r2);
    P.x = F(Y.x);
    P.dg = F(Y.diag);
    P.pp0 = F(Y.pp0);
    P.pp1 = F(Y.pp1);
    P.pp2 = F(Y.pp2);
    P.q = F(Y.q);
    P.q2 = F(Y.q2);
    P.acc = F(Y.acc);
    P.G = F(Y.G);
    P.Ya = F(Y.Y0);
    P.Yb = F(Y.Y1);
    P.rj = F(ctx->rhop);
    P.rj1 = F(ctx->rhop1);
    const bool tw = ctx->prm.two_way != 0;
    P.fdn = tw ? F(ctx->fdn) : nullptr;
    P.fdk = tw ? F(ctx->fdk) : nullptr;
    P.fm = tw ? F(Y.fm) : nullptr;
    P.mflux = tw ? P.fm : P.phin;
    P.snap = ctx->prm.capture ? reinterpret_cast<double*>(ctx->ws + Y.snap) : nullptr;
    const bool f32 = sizeof(T) == sizeof(float);
    P.b64 = f32 ? ctx->f<double>(Y.b64) : nullptr;
    P.x64a = f32 ? ctx->f<double>(Y.x64a) : nullptr;
    P.x64b = f32 ? ctx->f<double>(Y.x64b) : nullptr;
    P.xf = f32 ? F(Y.xf) : nullptr;
    return P;
}

template <typename T>
CgVecs<T> cg_vecs(const StepPtrs<T>& S) {
    CgVecs<T> v;
    v.r[0] = S.r;
    v.r[1] = S.r2;
    v.p[0] = S.pp0;
    v.p[1] = S.pp1;
    v.p[2] = S.pp2;
    v.q[0] = S.q;
    v.q[1] = S.q2;
    v.x = S.x;
    v.diag = S.dg;
    v.w = S.w;
    return v;
}

// dt, density predictor, momentum source and predictor sweeps (u* ends in
// the u slot ctx->ucur_slot).
// cfl_ready: the Courant partials of the current state are already in PS_CFL.
template <typename T>
pisoc_status enqueue_front(pisoc_ctx* ctx, StepPtrs<T>& S, bool cfl_ready) {
    using O = Ops<T>;
    const pisoc_params& p = ctx->prm;
    const Phys& ph = ctx->ph;
    const Launch& L = ctx->L;
    hipStream_t s = ctx->stream;
    DevState* st = ctx->st;
    clear_flags(s, st, ctx->batch);
    if (!cfl_ready) {
        timed(ctx, KC_CFL, 4, -1, [&] { O::cfl(L, s, ph, st, S.rn, S.phin, ctx->part(PS_CFL)); });
        ctx->nb_cfl = L.nblocks;
        ctx->cfl_part = ctx->part(PS_CFL);
    }
    timed(ctx, KC_PREDICT, 11, -1, [&] {
        O::predict(L, ctx->TL, s, ph, st, ctx->cfl_part, ctx->nb_cfl, p.dt_fixed, p.cfl,
                   p.dt_growth, p.dt_max, S.rn, S.un, S.phin, S.rk, S.aP, S.divu, S.pn);
    });
    timed(ctx, KC_MOM_SOURCE, 8, -1,
          [&] { O::mom_source(L, ctx->TL, s, ph, st, S.rn, S.un, S.divu, S.src); });
    if (p.two_way) {
        // words: rho^n, u^n x3, rho_j x K, phi x3, F_d x3, a_P and s x3 read;
        // F_m x3, a_P, s x3 written
        timed(ctx, KC_MIXTURE, 18.0 + p.n_classes, -1, [&] {
            O::mixture(L, s, ph, st, p.n_classes, S.rn, S.un, S.rj, S.phin, S.fdn, S.fm, S.aP,
                       S.src);
        });
    }
    T* uin = S.un;
    if (p.mom_tol > 0.0) {
        // BiCGStab from u^n, in place in the u* slot; batches of 8 iterations
        // with a host wait after each until the solve has stopped
        T* x = ucur_of(ctx, S);
        T* w = ctx->f<T>(ctx->lay.bicg);
        const size_t n3 = 3 * ctx->NT();
        T* r = w;
        T* rh = w + n3;
        // p, v, y = K^-1 p, s, z = K^-1 s, t
        T* const wk[6] = {w + 2 * n3, w + 3 * n3, w + 4 * n3, w + 5 * n3, w + 6 * n3, w + 7 * n3};
        if (hipMemcpyAsync(x, S.un, n3 * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess) {
            ctx->err = "hipMemcpyAsync failed";
            return PISOC_ERR_HIP;
        }
        double* pres = ctx->part(PS_CG + kBicgRes);
        O::bicg_init(L, s, ph, st, x, S.mflux, S.aP, S.src, S.pn, r, rh, pres);
        const double tol2 = p.mom_tol * p.mom_tol;
        for (int i = 1;; i += 8) {
            for (int k = i; k < i + 8; ++k)
                O::bicg_iter(L, ctx->TL, s, ph, st, k, tol2, p.mom_maxit, x, r, rh, wk, S.mflux, S.aP, pres,
                             ctx->part(PS_CG + kBicgV), ctx->part(PS_CG + kBicgTs));
            pisoc_status ss = sync_state(ctx);
            if (ss != PISOC_OK) return ss;
            bool all = true;
            for (int m = 0; m < ctx->batch; ++m) all = all && ctx->hst[m].bicg.it_stop != kIterInf;
            if (all) break;
        }
        uin = x;
    } else {
        for (int i = 0; i < p.n_mom_sweeps; ++i) {
            T* uout = (i & 1) ? S.ub : S.ua;
            timed(ctx, KC_MOM_SWEEP, 14, -1,
                  [&] { O::mom_sweep(L, ctx->TL, s, ph, st, uin, uout, S.mflux, S.aP, S.src, S.pn); });
            uin = uout;
        }
    }
    if (S.snap)   // the predictor's output u*
        for (int d = 0; d < 3; ++d)
            O::cast_out(s, uin + d * ctx->NT(), S.snap + (5 + d) * ctx->NT(), ctx->NT(), 0.0);
    if (ph.fourier) {
        // energy predictor: T* in tk after the sweeps (ping-pong with tw)
        double* aT = ctx->f<double>(ctx->lay.eaT);
        double* sT = ctx->f<double>(ctx->lay.esT);
        double* tk = ctx->f<double>(ctx->tk);
        double* tw = ctx->f<double>(ctx->lay.tw);
        O::energy_setup(L, s, ph, st, S.rn, S.rk, S.phin, S.divu, S.pn, aT, sT);
        const double* tin = ph.tn;
        for (int i = 0; i < p.n_mom_sweeps; ++i) {
            double* tout = ((p.n_mom_sweeps - 1 - i) & 1) ? tw : tk;
            O::energy_sweep(L, ctx->TL, s, ph, st, tin, tout, S.phin, aT, sT);
            tin = tout;
        }
    }
    return PISOC_OK;
}

template <typename T>
T* ucur_of(const pisoc_ctx* ctx, StepPtrs<T>& S) { return ctx->ucur_slot == 1 ? S.ua : S.ub; }

template <typename T>
void enqueue_corr_setup(pisoc_ctx* ctx, StepPtrs<T>& S, int corr, bool guess) {
    using O = Ops<T>;
    const Phys& ph = ctx->ph;
    const Launch& L = ctx->L;
    hipStream_t s = ctx->stream;
    const size_t N = ctx->NT();
    const bool f32 = sizeof(T) == sizeof(float);
    T* ucur = ucur_of(ctx, S);
    timed(ctx, KC_HBYA, 16, -1,
          [&] { O::hbya(L, ctx->TL, s, ph, ctx->st, ucur, S.hb, S.mflux, S.aP, S.src, S.rk, S.w, S.p0); });
    const bool cap = S.snap && corr == 0;
    if (cap) O::cast_out(s, S.w, S.snap + 4 * N, N, 0.0);   // the operator's w = rho/a_P
    timed(ctx, KC_CORR_RHS, f32 ? 14 : 12, -1, [&] {
        ctx->nb_start = O::corr_rhs(L, ctx->TL, s, ph, ctx->st, S.rn, S.rk, S.w, S.hb, S.p0, S.phiH,
                                    S.r, S.dg, ctx->part(PS_U), cap ? S.snap : nullptr,
                                    cap ? S.snap + N : nullptr, cap ? S.snap + 2 * N : nullptr,
                                    S.b64);
    });
    if (guess) {
        const T* gprev = ctx->prm.guess == PISOC_GUESS_PREVIOUS
                             ? ctx->f<T>(ctx->lay.xprev) + (size_t)corr * N
                             : nullptr;
        guess_solve_start<T>(ctx, gprev, S.r, S.x, S.dg, S.w, S.p0, S.pp0, S.q);
        ctx->nb_start = L.nblocks;   // the guess rewrites the start's partials
        if (cap) {
            // the network's guess g (left in pp0) and the solve's start x0 (x, or
            // x64 in FP32 storage, where x holds the zero inner correction)
            O::cast_out(s, S.pp0, S.snap + 8 * N, N, 0.0);
            if (f32)
                (void)hipMemcpyAsync(S.snap + 9 * N, S.x64a, N * sizeof(double),
                                     hipMemcpyDeviceToDevice, s);
            else
                O::cast_out(s, S.x, S.snap + 9 * N, N, 0.0);
        }
    }
}

template <typename T>
void enqueue_corr_finish(pisoc_ctx* ctx, StepPtrs<T>& S, int corr) {
    using O = Ops<T>;
    const Phys& ph = ctx->ph;
    const Launch& L = ctx->L;
    hipStream_t s = ctx->stream;
    const size_t N = ctx->NT();
    const bool cap = S.snap && corr == 0;
    T* ucur = ucur_of(ctx, S);
    const bool last = corr == ctx->prm.n_corr - 1;
    if (ctx->TL.nblocks) {
        // flux correction and update in one tiled pass (words: w, p0, p', phiH x3,
        // HbyA x3, rho^n, a_P read; phi x3, rho_k, u x3 written)
        timed(ctx, KC_CORR_UPDATE, 18, -1, [&] {
            // the last pass also leaves the Courant partials of the new state
            ctx->nb_mass = O::corr_finish_fused(ctx->TL, s, ph, ctx->st, last, S.p0, S.x, S.w,
                                                S.phiH, S.phik, cap ? S.snap + 3 * N : nullptr,
                                                S.rn, S.hb, S.aP, S.rk, ucur, ctx->part(PS_MASS));
        });
        if (last) ctx->nb_cfl_next = ctx->nb_mass;
        return;
    }
    timed(ctx, KC_CORR_FLUX, 10, -1, [&] {
        O::corr_flux(L, ctx->TL, s, ph, ctx->st, S.p0, S.x, S.w, S.phiH, S.phik, S.q,
                     cap ? S.snap + 3 * N : nullptr);
    });
    timed(ctx, KC_CORR_UPDATE, 13, -1, [&] {
        ctx->nb_mass = O::corr_update(L, ctx->TL, s, ph, ctx->st, last, S.rn, S.phik, S.hb, S.q,
                                      S.aP, S.rk, ucur, ctx->part(PS_MASS));
    });
}

template <typename T>
void enqueue_dust(pisoc_ctx* ctx, StepPtrs<T>& S) {
    using O = Ops<T>;
    const pisoc_params& p = ctx->prm;
    unsigned nb_dust = ctx->L.nblocks;   // partials of the dust finish
    unsigned nb_diag = ctx->L.nblocks;   // ... of the first dust sweep (its diagonal check)
    const Phys& ph = ctx->ph;
    const Launch& L = ctx->L;
    hipStream_t s = ctx->stream;
    DevState* st = ctx->st;
    const size_t N = ctx->NT();
    T* ucur = ucur_of(ctx, S);
    if (p.n_classes > 0) {
        timed(ctx, KC_DUDT, 9, -1, [&] { O::dudt(L, ctx->TL, s, ph, st, S.un, ucur, S.acc); });
        for (int c = 0; c < p.n_classes; ++c) {
            timed(ctx, KC_DUST_FLUX, 13, -1, [&] {
                O::dust_flux(L, ctx->TL, s, ph, st, c, S.phik, S.rk, S.acc, S.G, S.rj + c * N, S.rn,
                             S.Ya);
            });
            T* yin = S.Ya;
            T* yout = S.Yb;
            Phys phc = ph;   // BDF2: this class's bulk density at t^{n-1}
            if (ph.bdf2) phc.rjm1 = ph.rjm1 + c * N;
            for (int i = 0; i < p.n_dust_sweeps; ++i) {
                // the first sweep also checks the implicit diagonal (the same in every sweep)
                double* chk = i == 0 ? ctx->part(PS_DDIAG + 2 * c) : nullptr;
                timed(ctx, KC_DUST_SWEEP, 7, -1, [&] {
                    const unsigned nb =
                        O::dust_sweep(L, ctx->TL, s, phc, st, yin, yout, S.G, S.rj + c * N, S.rk, chk);
                    if (chk) nb_diag = nb;
                });
                std::swap(yin, yout);
            }
            // two-way coupling: the class's face fluxes add up to the next step's F_d
            const double fdw = S.fdk ? (c == 0 ? 3.0 : 6.0) : 0.0;
            if (ctx->TL.nblocks) {
                // face fluxes and finish in one tiled pass (words: Y, G, rho_j read, rho_j' written)
                timed(ctx, KC_DUST_FINISH, 6 + fdw, -1, [&] {
                    nb_dust = O::dust_finish_fused(ctx->TL, s, phc, st, yin, S.G, S.rj + c * N,
                                                   S.rj1 + c * N, ctx->part(PS_DUST + 2 * c),
                                                   S.fdk, c == 0);
                });
            } else {
                timed(ctx, KC_DUST_FACEFLUX, 7, -1, [&] { O::dust_faceflux(L, s, ph, yin, S.G); });
                timed(ctx, KC_DUST_FINISH, 5 + fdw, -1, [&] {
                    O::dust_finish(L, s, phc, st, S.rj + c * N, S.G, S.rj1 + c * N,
                                   ctx->part(PS_DUST + 2 * c), S.fdk, c == 0);
                });
            }
        }
    }
    step_finish(s, ph, st, ctx->part(PS_MASS), ctx->nb_mass, ctx->part(PS_DUST), p.n_classes,
                nb_dust, ctx->part(PS_DDIAG), nb_diag, ctx->lay.max_blocks);
}

// Iterations past a solve's predicted count that an eager FP32 first round
// runs before it is stopped.
constexpr int kSpecMargin = 2;

// Latest stop iteration of corrector corr's first round over the members
// (launches from it on did no CG work), from the state the host last read.
int first_stop(const pisoc_ctx* ctx, int corr) {
    int k = 0;
    for (int m = 0; m < ctx->batch; ++m) k = std::max(k, ctx->hst[m].it_first[corr]);
    return k;
}

// FP32 storage: mixed-precision iterative refinement of M p' = b for every
// member.  guess: the first inner solve starts from the learned guess (x and
// x64 set), else from zero.  The first inner FP32 solve runs to tau0 = max(p_tol/2, inner_tol)
// of ||b||; after each inner solve k_refine adds the correction to the FP64
// accumulator and evaluates the true residual in FP64; each later round aims
// at half the requested residual (reducing the current one by no more than
// the factor inner_tol); a member is done when ||r64|| <= p_tol ||b||.
// eager: rounds until every member is done or max_refine; otherwise exactly
// ctx->rounds rounds with ctx->caps / cap_later CG pairs.  The FP64 solution
// ends in x64a and its FP32 copy in x.
void solve_fp32(pisoc_ctx* ctx, StepPtrs<float>& S, int corr, bool guess, bool eager,
                pisoc_status* err) {
    const pisoc_params& p = ctx->prm;
    hipStream_t s = ctx->stream;
    const int B = ctx->batch;
    double* xa = S.x64a;
    double* xb = S.x64b;
    const double tau0 = std::min(0.5, std::max(0.5 * p.p_tol, p.inner_tol));
    *err = PISOC_OK;
    set_tol(s, ctx->st, B, tau0 * tau0);
    int most = 0;
    // An eager first round does not wait for the host: it runs the
    // iterations of the last step's first round plus kSpecMargin, the last
    // of them stopping the solve; a round stopped there unconverged is taken
    // up by the refinement.  The count is updated after the step.
    const int cap0 = eager ? std::min((ctx->pred_first[corr] > 0 ? ctx->pred_first[corr] : 8) +
                                          kSpecMargin, p.p_maxit)
                           : ctx->caps[corr];
    if ((*err = run_pcg<float>(ctx, cg_vecs(S), true, cap0, false, nullptr, !guess, ctx->nb_start,
                               cap0)) != PISOC_OK)
        return;
    record_solve(s, ctx->st, B, corr, /*round=*/1, /*add=*/1, /*fin=*/0);
    bool waited = false;   // the host has seen the state since the first round
    const int max_rounds = eager ? p.max_refine : ctx->rounds;
    int round = 0;
    unsigned nb_ref = ctx->L.nblocks;   // partials of the last refinement
    // An eager first round from zero leaves its correction d as the solution
    // (x64 = d exactly) and stores no copy of it; should a later round follow,
    // x64 is then made from d.
    bool sol_in_x = false;
    for (;;) {
        const bool from_zero = round == 0 && !guess;
        const bool store_x = !(from_zero && eager);
        timed(ctx, KC_REFINE, from_zero ? (store_x ? 9 : 6) : 11, -1, [&] {
            nb_ref = Ops<float>::refine(ctx->L, ctx->TL, s, ctx->ph, ctx->st, xa, S.x, xb, S.xf,
                                        S.b64, S.w, S.dg, S.r, ctx->part(PS_U), from_zero,
                                        store_x);
        });
        if (store_x) std::swap(xa, xb);
        else sol_in_x = true;
        ++round;
        // column 1 (||r64||^2) of the 3 columns written with nb_ref blocks
        finalize_sums(s, ctx->part(PS_U) + nb_ref, nb_ref, B, 1, ctx->st, 0, true);
        if (round >= max_rounds) break;
        if (eager) {
            if ((*err = sync_state(ctx)) != PISOC_OK) return;
            if (ctx->prof.on) ctx->prof.resolve(waited ? kIterInf : first_stop(ctx, corr));
            waited = true;
            bool done = true;
            for (int m = 0; m < B; ++m) {
                const DevState& h = ctx->hst[m];
                if (!(h.red[0] <= h.pcg.tol_final * h.pcg.bb) && std::isfinite(h.red[0])) done = false;
            }
            if (done) break;
        }
        if (sol_in_x) {
            // x64 = d before the next round's solve overwrites d, and the
            // FP32 copy xf = d: a member already converged skips the later
            // rounds' refinement, which would otherwise have written xf, and
            // the corrector takes its solution from xf
            Ops<float>::cast_out(s, S.x, xa, ctx->NT(), 0.0);
            if (hipMemcpyAsync(S.xf, S.x, sizeof(float) * ctx->NT(), hipMemcpyDeviceToDevice, s) !=
                hipSuccess) {
                ctx->err = "hipMemcpyAsync failed";
                *err = PISOC_ERR_HIP;
                return;
            }
            sol_in_x = false;
        }
        set_tol_refine(s, ctx->st, B, p.inner_tol);
        // the inner correction of this round starts from zero (not written)
        const int pairs = eager ? std::max(2, ctx->pred_later) : ctx->cap_later;
        if ((*err = run_pcg<float>(ctx, cg_vecs(S), false, pairs, eager,
                                   &most, true, nb_ref, eager ? 0 : pairs)) != PISOC_OK)
            return;
        if (eager) ctx->pred_later = most;
        record_solve(s, ctx->st, B, corr, round + 1, /*add=*/1, /*fin=*/0);
    }
    if (eager && ctx->prof.on && !waited) {
        // attribute the first round's launches before later solves add more
        if ((*err = sync_state(ctx)) != PISOC_OK) return;
        ctx->prof.resolve(first_stop(ctx, corr));
    }
    record_solve(s, ctx->st, B, corr, round, /*add=*/0, /*fin=*/2);
    // the corrector uses the FP32 copy of the FP64 solution, which the last
    // refinement wrote to xf: exchange the two buffers' roles for the rest of
    // the step (x is free again until the next solve writes it); after a
    // single round from zero it is x itself
    if (!sol_in_x) std::swap(S.x, S.xf);
}

bool audit_on(const pisoc_ctx* ctx) {
    return ctx->prm.guess != PISOC_GUESS_ZERO && ctx->prm.guess_audit > 0 && ctx->audit.have_events;
}

// A guess exists for this step: the learned one always, the previous-step one
// once a step has been taken.
bool guess_available(const pisoc_ctx* ctx) {
    return ctx->prm.guess == PISOC_GUESS_LEARNED ||
           (ctx->prm.guess == PISOC_GUESS_PREVIOUS && ctx->steps > 0);
}

// The guess is used for a solve when the iterations it saves exceed its cost
// (both as running means); until both options have been measured each is
// tried once, and every guess_audit-th step takes the other option once so
// that the mean of the unused one stays current (not a rejected guess whose
// cost is at least the zero-start solve's iterations: no saving could pay it).
constexpr int kMaxProbeFactor = 16;
bool audit_measured(const pisoc_ctx* ctx);

bool audit_pays(const pisoc_ctx* ctx, int c) {
    const auto& A = ctx->audit;
    return A.it_zero[c] - A.it_guess[c] > std::max(A.cost, 0.0);
}

void audit_decide(pisoc_ctx* ctx) {
    auto& A = ctx->audit;
    const bool measured = audit_measured(ctx);
    A.probing = measured && A.steps >= A.next_probe;
    for (int c = 0; c < ctx->prm.n_corr; ++c) {
        bool use;
        if (A.it_guess[c] < 0.0) use = true;
        else if (A.it_zero[c] < 0.0) use = false;
        else {
            const bool pays = audit_pays(ctx, c);
            A.verdict[c] = pays;
            // a rejected guess whose cost reaches the whole zero-start solve
            // could not pay even by saving every iteration: no trial of it
            const bool hopeless = !pays && A.cost >= A.it_zero[c];
            use = A.probing && !hopeless ? !pays : pays;
        }
        A.use[c] = use;
    }
}

// The choice a captured step is built with: the audit's current verdict for
// each corrector, without the periodic probe (a choice not measured yet
// counts as paying).
void audit_decide_capture(pisoc_ctx* ctx) {
    auto& A = ctx->audit;
    for (int c = 0; c < ctx->prm.n_corr; ++c)
        A.use[c] = A.it_guess[c] < 0.0 || A.it_zero[c] < 0.0 ||
                   A.it_zero[c] - A.it_guess[c] > std::max(A.cost, 0.0);
}

// Both choices measured for every corrector (the capture can take a verdict).
bool audit_measured(const pisoc_ctx* ctx) {
    for (int c = 0; c < ctx->prm.n_corr; ++c)
        if (ctx->audit.it_guess[c] < 0.0 || ctx->audit.it_zero[c] < 0.0) return false;
    return true;
}

// After the step's last synchronisation: fold its iterations and timings in.
void audit_update(pisoc_ctx* ctx) {
    auto& A = ctx->audit;
    auto mean = [](double old, double x) { return old < 0.0 ? x : 0.5 * (old + x); };
    for (int c = 0; c < ctx->prm.n_corr; ++c) {
        int it = 0;
        for (int m = 0; m < ctx->batch; ++m) it = std::max(it, ctx->hst[m].it_corr[c]);
        if (!A.use[c]) {
            A.it_zero[c] = mean(A.it_zero[c], it);
            continue;
        }
        A.it_guess[c] = mean(A.it_guess[c], it);
        float t_guess = 0.f, t_solve = 0.f;
        if (hipEventSynchronize(A.ev[c][2]) == hipSuccess &&
            hipEventElapsedTime(&t_guess, A.ev[c][0], A.ev[c][1]) == hipSuccess &&
            hipEventElapsedTime(&t_solve, A.ev[c][1], A.ev[c][2]) == hipSuccess && t_solve > 0.f)
            A.cost = mean(A.cost, (double)t_guess / ((double)t_solve / std::max(it, 1)));
    }
    if (A.probing) {
        bool confirmed = true;
        for (int c = 0; c < ctx->prm.n_corr; ++c)
            confirmed = confirmed && audit_pays(ctx, c) == A.verdict[c];
        const int64_t base = ctx->prm.guess_audit;
        A.period = confirmed ? std::min(2 * A.period, kMaxProbeFactor * base) : base;
        A.next_probe = A.steps + A.period;
        A.probing = false;
    }
    A.steps += 1;
}

// Launch sequence of one step of every member.  eager: with host waits in the
// pressure solves; otherwise the fixed sequence for graph capture.
template <typename T>
pisoc_status enqueue_step(pisoc_ctx* ctx, bool eager) {
    const pisoc_params& p = ctx->prm;
    StepPtrs<T> S = step_ptrs<T>(ctx);
    hipStream_t s = ctx->stream;
    // an eager step reuses the Courant partials the previous accepted step left
    const bool cfl_ready = eager && ctx->cfl_ready;
    ctx->cfl_ready = false;
    ctx->nb_cfl_next = 0;
    if (ctx->ph.fourier) {   // this step's temperature buffers
        ctx->ph.tn = ctx->f<double>(ctx->tn);
        ctx->ph.ts = ctx->f<double>(ctx->tk);
    }
    if (ctx->ph.bdf2) {      // the state at t^{n-1}
        ctx->ph.rm1 = ctx->f<double>(ctx->rm1);
        ctx->ph.um1 = ctx->f<double>(ctx->um1);
        ctx->ph.rjm1 = ctx->f<double>(ctx->rjm1);
    }
    if (pisoc_status fs = enqueue_front<T>(ctx, S, cfl_ready); fs != PISOC_OK) return fs;
    // with the audit on, an eager step takes this step's decision and a
    // captured one the verdict it was built with (audit_decide_capture)
    const bool audit = eager && audit_on(ctx);
    for (int corr = 0; corr < p.n_corr; ++corr) {
        // a step without a guess available counts as one without the guess
        if (audit && !guess_available(ctx)) ctx->audit.use[corr] = false;
        const bool guess = guess_available(ctx) && (!audit_on(ctx) || ctx->audit.use[corr]);
        if (audit && guess) (void)hipEventRecord(ctx->audit.ev[corr][0], s);
        enqueue_corr_setup<T>(ctx, S, corr, guess);
        if (audit && guess) (void)hipEventRecord(ctx->audit.ev[corr][1], s);
        pisoc_status err = PISOC_OK;
        if constexpr (sizeof(T) == sizeof(float)) {
            solve_fp32(ctx, S, corr, guess, eager, &err);
        } else {
            set_tol(s, ctx->st, ctx->batch, p.p_tol * p.p_tol);
            int most = 0;
            const int pairs =
                eager ? (ctx->pred_first[corr] > 0 ? ctx->pred_first[corr] : 8) : ctx->caps[corr];
            // a captured solve stops at its cap at the latest: its last launch
            // brings x up to date with the residual it reports
            err = run_pcg<T>(ctx, cg_vecs(S), true, pairs, eager, &most,
                             !guess, ctx->nb_start, eager ? 0 : pairs);
            if (eager) ctx->pred_first[corr] = most;
            record_solve(s, ctx->st, ctx->batch, corr, /*round=*/0, /*add=*/1, /*fin=*/1);
        }
        if (err != PISOC_OK) return err;
        if (audit && guess) (void)hipEventRecord(ctx->audit.ev[corr][2], s);
        if (p.guess == PISOC_GUESS_PREVIOUS) {
            // the solution the corrector applies: the next step's guess
            T* xp = ctx->f<T>(ctx->lay.xprev) + (size_t)corr * ctx->NT();
            if (hipMemcpyAsync(xp, S.x, sizeof(T) * ctx->NT(), hipMemcpyDeviceToDevice, s) !=
                hipSuccess) {
                ctx->err = "hipMemcpyAsync failed";
                return PISOC_ERR_HIP;
            }
        }
        if (eager) {
            for (int m = 0; m < ctx->batch; ++m)
                if (ctx->hst[m].flags & PISOC_FLAG_BAD_DT) {
                    ctx->err = "time step undefined or non-positive (zero velocity needs dt_fixed "
                               "or dt_max)";
                    return PISOC_ERR_INVALID;
                }
        }
        enqueue_corr_finish<T>(ctx, S, corr);
    }
    enqueue_dust<T>(ctx, S);
    if (!eager) commit(s, ctx->st, ctx->batch);
    return PISOC_OK;
}

// Host-side rotation after an accepted step (period 2).
void rotate(pisoc_ctx* ctx) {
    const bool bdf2 = ctx->prm.time_scheme == PISOC_BDF2;
    if (bdf2) {   // t^n becomes t^{n-1}; its old buffers take the next step's values
        size_t t = ctx->rm1;
        ctx->rm1 = ctx->rn;
        ctx->rn = ctx->rk;
        ctx->rk = t;
    } else {
        std::swap(ctx->rn, ctx->rk);
    }
    std::swap(ctx->phin, ctx->phik);
    std::swap(ctx->u_idx[0], ctx->u_idx[ctx->ucur_slot]);
    // the old u^n now sits in a work slot: it becomes u^{n-1}
    if (bdf2) std::swap(ctx->lay.u3[ctx->u_idx[ctx->ucur_slot]], ctx->um1);
    if (ctx->prm.n_classes > 0) {
        if (bdf2) {
            size_t t = ctx->rjm1;
            ctx->rjm1 = ctx->rhop;
            ctx->rhop = ctx->rhop1;
            ctx->rhop1 = t;
        } else {
            std::swap(ctx->rhop, ctx->rhop1);
        }
    }
    // two-way with dust: this step's F_d becomes the next step's (without dust
    // both stay zero)
    if (ctx->prm.two_way && ctx->prm.n_classes > 0) std::swap(ctx->fdn, ctx->fdk);
    if (ctx->prm.closure == PISOC_FOURIER) std::swap(ctx->tn, ctx->tk);
}

// Step record of member m from its device state.
void fill_info(const pisoc_ctx* ctx, const DevState& h, bool committed, pisoc_step_info* out) {
    pisoc_step_info rec{};
    rec.dt = h.dt;
    rec.t = committed ? h.t : h.t + h.dt;
    rec.courant = h.sigma * h.dt;
    rec.flags = h.flags;
    rec.mass_gas = h.mass_gas;
    for (int c = 0; c < ctx->prm.n_corr; ++c) {
        rec.pcg_iters[c] = h.it_corr[c];
        rec.pcg_relres[c] = h.rel_corr[c];
        rec.refinements[c] = h.rounds_corr[c];
    }
    for (int c = 0; c < ctx->prm.n_classes; ++c) rec.mass_p[c] = h.mass_p[c];
    rec.courant_dust = h.courant_dust;
    rec.mom_iters = h.bicg.iters;
    rec.mom_relres = h.bicg.bb > 0.0 ? std::sqrt(h.bicg.rr / h.bicg.bb) : 0.0;
    *out = rec;
}

bool member_bad(const pisoc_ctx* ctx, const DevState& h) {
    bool bad = (h.flags & (PISOC_FLAG_NONFINITE | PISOC_FLAG_RHO_NONPOS |
                           PISOC_FLAG_DUST_NONFINITE)) != 0;
    for (int c = 0; c < ctx->prm.n_classes; ++c)
        if (!std::isfinite(h.mass_p[c])) bad = true;
    return bad;
}

pisoc_status flag_status(int flags) {
    if (flags & (PISOC_FLAG_PCG_MAXIT | PISOC_FLAG_MOM_MAXIT)) return PISOC_WARN_NOT_CONVERGED;
    if (flags & (PISOC_FLAG_DUST_NEG | PISOC_FLAG_DUST_DIAG | PISOC_FLAG_DUST_COURANT))
        return PISOC_WARN_DUST;
    if (flags & PISOC_FLAG_GUESS_FALLBACK) return PISOC_WARN_GUESS_FALLBACK;
    return PISOC_OK;
}

pisoc_status combine_status(pisoc_status a, pisoc_status b) {
    if (a < 0 || b < 0) return std::min(a, b);
    if (a == PISOC_WARN_NOT_CONVERGED || b == PISOC_WARN_NOT_CONVERGED) return PISOC_WARN_NOT_CONVERGED;
    return std::max(a, b);
}

// One eager step of every member of ctx; info (may be NULL) receives batch
// records.  The step is checked before it is committed: if any member
// diverged, no member advances.
pisoc_status eager_step(pisoc_ctx* ctx, pisoc_step_info* info) {
    if (audit_on(ctx)) audit_decide(ctx);
    pisoc_status st = ctx->prm.precision == PISOC_FP64 ? enqueue_step<double>(ctx, true)
                                                       : enqueue_step<float>(ctx, true);
    if (st != PISOC_OK) return st;
    if ((st = sync_state(ctx)) != PISOC_OK) return st;
    if (ctx->prof.on) ctx->prof.resolve(kIterInf);
    // first-round iteration counts: the next step's predictions
    for (int c = 0; c < ctx->prm.n_corr; ++c) {
        const int it = first_stop(ctx, c);
        if (it > 0) ctx->pred_first[c] = it;
    }
    int skipped = 0;
    if (audit_on(ctx)) {
        audit_update(ctx);
        for (int c = 0; c < ctx->prm.n_corr; ++c) skipped |= ctx->audit.use[c] ? 0 : PISOC_FLAG_GUESS_SKIPPED;
    }
    pisoc_status worst = PISOC_OK;
    bool bad = false;
    for (int m = 0; m < ctx->batch; ++m) {
        const DevState& h = ctx->hst[m];
        if (h.flags & PISOC_FLAG_BAD_DT) {
            ctx->err = "time step undefined or non-positive";
            return PISOC_ERR_INVALID;
        }
        if (member_bad(ctx, h)) bad = true;
        worst = combine_status(worst, flag_status(h.flags));
    }
    if (bad) {
        ctx->err = "step diverged (non-finite field, non-positive density or non-finite dust "
                   "density); state kept";
        if (info)
            for (int m = 0; m < ctx->batch; ++m) {
                fill_info(ctx, ctx->hst[m], false, info + m);
                info[m].t = ctx->hst[m].t;
                if (member_bad(ctx, ctx->hst[m])) info[m].flags |= PISOC_FLAG_NONFINITE;
            }
        return PISOC_ERR_DIVERGED;
    }
    if (info)
        for (int m = 0; m < ctx->batch; ++m) {
            fill_info(ctx, ctx->hst[m], false, info + m);
            info[m].flags |= skipped;
        }
    rotate(ctx);
    commit(ctx->stream, ctx->st, ctx->batch);
    ctx->cfl_ready = ctx->nb_cfl_next > 0;
    if (ctx->cfl_ready) {
        // column 3 of the pass's block_partials, nb_cfl_next apart
        ctx->nb_cfl = ctx->nb_cfl_next;
        ctx->cfl_part = ctx->part(PS_MASS) + 3 * (size_t)ctx->nb_cfl;
    }
    ctx->t += ctx->hst[0].dt;
    ctx->steps += 1;
    return worst;
}

// Common initialisation of a context for `batch` members of one size.
// mprm[m]: per-member parameters (identical except C and tau_p); inputs per member.
pisoc_status init_ctx(pisoc_ctx* ctx, const pisoc_params* mprm, int batch, char* ws,
                      const double* const* d_rho, const double* const* d_u,
                      const double* const* d_rho_p, hipStream_t stream) {
    const pisoc_params* prm = &mprm[0];
    ctx->prm = *prm;
    ctx->batch = batch;
    ctx->stream = stream;
    ctx->ws = ws;
    ctx->lay = make_layout(prm, batch);
    const Layout& lay = ctx->lay;
    ctx->TL = make_tiled_launch(prm->n, batch);
    ctx->TS = make_spmv_launch(prm->n, batch, prm->precision == PISOC_FP64 ? 8 : 4);
    // PISOC_UNTILED=1 selects the untiled kernels (kernel-comparison tests)
    if (const char* e = std::getenv("PISOC_UNTILED"); e && e[0] == '1') ctx->TL = ctx->TS = Launch{};
    // (the tiled forms carry the Fourier closure and BDF2 as the gathered ones)
    ctx->L = make_launch(prm->n, batch);
    ctx->ph = make_phys(prm, ctx->L, batch);
    ctx->st = reinterpret_cast<DevState*>(ctx->ws + lay.state);
    ctx->partials = reinterpret_cast<double*>(ctx->ws + lay.partials);
    ctx->u_idx[0] = 0;
    ctx->u_idx[1] = 1;
    ctx->u_idx[2] = 2;
    ctx->ucur_slot = (prm->n_mom_sweeps & 1) ? 1 : 2;
    ctx->rn = lay.rn;
    ctx->rk = lay.rk;
    ctx->phin = lay.phin;
    ctx->phik = lay.phik;
    ctx->rhop = lay.rhop;
    ctx->rhop1 = lay.rhop1;
    ctx->fdn = lay.fd0;
    ctx->fdk = lay.fd1;
    ctx->t = 0.0;
    ctx->steps = 0;
    for (int c = 0; c < PISOC_MAX_CORR; ++c) {
        ctx->pred_first[c] = 0;
        ctx->caps[c] = 0;
    }
    ctx->pred_later = 0;
    ctx->cap_later = 0;
    ctx->rounds = 0;
    for (int c = 0; c < PISOC_MAX_CORR; ++c) {
        ctx->audit.it_zero[c] = -1.0;
        ctx->audit.it_guess[c] = -1.0;
        ctx->audit.use[c] = true;
    }
    ctx->audit.cost = -1.0;
    ctx->audit.steps = 0;
    ctx->audit.period = std::max(prm->guess_audit, 1);
    ctx->audit.next_probe = ctx->audit.period - 1;
    ctx->audit.probing = false;
    ctx->audit.have_events = false;
    if (prm->guess != PISOC_GUESS_ZERO && prm->guess_audit > 0) {
        bool ok = true;
        for (auto& row : ctx->audit.ev)
            for (auto& e : row)   // timing only, as the profiler's
                ok = ok && hipEventCreateWithFlags(&e, hipEventDisableSystemFence) == hipSuccess;
        ctx->audit.have_events = ok;
        if (!ok) {
            ctx->err = "hipEventCreate failed";
            return PISOC_ERR_HIP;
        }
    }
    ctx->es = prm->precision == PISOC_FP64 ? sizeof(double) : sizeof(float);
    ctx->prof.reset();
    // the records, then the publication's sequence number (coherent memory:
    // the GPU's stores reach the host while the stream still runs)
    const size_t hbytes = sizeof(DevState) * (size_t)batch;
    bool coherent = hipHostMalloc(reinterpret_cast<void**>(&ctx->hst), hbytes + 64,
                                  hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess;
    if (!coherent) {   // the plain pinned copy and the stream sync then
        (void)hipGetLastError();
        if (hipHostMalloc(reinterpret_cast<void**>(&ctx->hst), hbytes + 64, hipHostMallocDefault) !=
            hipSuccess) {
            ctx->hst = nullptr;
            ctx->err = "hipHostMalloc failed";
            return PISOC_ERR_HIP;
        }
    }
    if (coherent) {
        void* dev = nullptr;
        unsigned long long* seq = reinterpret_cast<unsigned long long*>(
            reinterpret_cast<char*>(ctx->hst) + hbytes);
        *seq = 0;
        if (hipHostGetDevicePointer(&dev, ctx->hst, 0) == hipSuccess && dev) {
            ctx->hst_dev = reinterpret_cast<DevState*>(dev);
            ctx->seq_dev = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(dev) + hbytes);
            ctx->seq_host = seq;
        } else {
            (void)hipGetLastError();   // the plain copy path then
        }
    }
    hipStream_t s = ctx->stream;
    const size_t N = ctx->N();
    HIP_TRY(ctx, hipMemsetAsync(ctx->st, 0, sizeof(DevState) * (size_t)batch, s));

    // reference density of each member = mean of its initial density (FP64)
    const Launch L1 = make_launch(prm->n, 1);
    const Phys ph1 = make_phys(prm, L1, 1);
    for (int m = 0; m < batch; ++m) {
        Ops<double>::sum_affine_sq(L1, s, ph1, nullptr, d_rho[m], 0.0, 0.0, ctx->part(PS_STAT));
        finalize_sums(s, ctx->part(PS_STAT), L1.nblocks, 1, 2, ctx->st + m, 0);
    }
    pisoc_status ss = sync_state(ctx);
    if (ss != PISOC_OK) return ss;
    ctx->rho_ref.assign(batch, 1.0);
    ctx->p_ref.assign(batch, 1.0);
    // two-way coupling: the mean mixture density (conserved: gas and dust
    // masses are), from the initial fields
    std::vector<double> rhom(batch, 0.0);
    if (prm->two_way) {
        for (int m = 0; m < batch; ++m) rhom[m] = ctx->hst[m].red[1] / (double)N;
        for (int c = 0; c < prm->n_classes; ++c) {
            for (int m = 0; m < batch; ++m) {
                Ops<double>::sum_affine_sq(L1, s, ph1, nullptr, d_rho_p[m] + c * N, 0.0, 0.0,
                                           ctx->part(PS_STAT));
                finalize_sums(s, ctx->part(PS_STAT), L1.nblocks, 1, 2, ctx->st + m, 0);
            }
            pisoc_status sd = sync_state(ctx);
            if (sd != PISOC_OK) return sd;
            for (int m = 0; m < batch; ++m) rhom[m] += ctx->hst[m].red[1] / (double)N;
        }
        // the gas sums above were overwritten: take them again
        for (int m = 0; m < batch; ++m) {
            Ops<double>::sum_affine_sq(L1, s, ph1, nullptr, d_rho[m], 0.0, 0.0, ctx->part(PS_STAT));
            finalize_sums(s, ctx->part(PS_STAT), L1.nblocks, 1, 2, ctx->st + m, 0);
        }
        pisoc_status sg = sync_state(ctx);
        if (sg != PISOC_OK) return sg;
    }
    for (int m = 0; m < batch; ++m) {
        const double rr = ctx->hst[m].red[1] / (double)N;
        if (!(rr > 0.0) || !std::isfinite(rr)) {
            ctx->err = "initial density must have a positive finite mean";
            return PISOC_ERR_INVALID;
        }
        ctx->rho_ref[m] = rr;
        ctx->p_ref[m] = prm->closure == PISOC_FOURIER ? rr * prm->R_gas * prm->T0
                                                      : mprm[m].C * std::pow(rr, prm->gamma);
    }
    for (int m = 0; m < batch; ++m) {
        DevState init{};
        init.pcg.tol2 = prm->p_tol * prm->p_tol;
        init.pcg.tol_final = prm->p_tol * prm->p_tol;
        init.pcg.maxit = prm->p_maxit;
        init.pcg.it_stop = kIterInf;
        init.dt_prev = __builtin_inf();
        init.rho_ref = ctx->rho_ref[m];
        init.p_ref = ctx->p_ref[m];
        for (int c = 0; c < prm->n_classes; ++c) init.tau[c] = mprm[m].tau_p[c];
        init.rhom_mean = rhom[m];
        ctx->hst[m] = init;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->st, ctx->hst, sizeof(DevState) * (size_t)batch,
                                hipMemcpyHostToDevice, s));
    const size_t NT = ctx->NT();
    auto convert = [&](auto tag) {
        using T = decltype(tag);
        for (int m = 0; m < batch; ++m) {
            const size_t off = (size_t)m * N;
            Ops<T>::cast_in(s, d_rho[m], ctx->f<T>(ctx->rn) + off, N, ctx->rho_ref[m]);
            for (int d = 0; d < 3; ++d)
                Ops<T>::cast_in(s, d_u[m] + d * N, ctx->f<T>(lay.u3[0]) + d * NT + off, N, 0.0);
            for (int c = 0; c < prm->n_classes; ++c)
                Ops<T>::cast_in(s, d_rho_p[m] + c * N, ctx->f<T>(ctx->rhop) + c * NT + off, N, 0.0);
        }
        Ops<T>::init_phi(ctx->L, s, ctx->ph, ctx->st, ctx->f<T>(ctx->rn), ctx->f<T>(lay.u3[0]),
                         ctx->f<T>(ctx->phin));
        if (prm->two_way) {
            // F_d of the initial state; the other buffer starts at zero (it
            // stays so without dust)
            (void)hipMemsetAsync(ctx->f<T>(ctx->fdk), 0, 3 * sizeof(T) * NT, s);
            if (prm->n_classes > 0)
                Ops<T>::init_fd(ctx->L, s, ctx->ph, prm->n_classes, ctx->f<T>(ctx->rhop),
                                ctx->f<T>(lay.u3[0]), ctx->f<T>(ctx->fdn));
            else
                (void)hipMemsetAsync(ctx->f<T>(ctx->fdn), 0, 3 * sizeof(T) * NT, s);
        }
    };
    if (prm->precision == PISOC_FP64) convert(double{});
    else convert(float{});
    if (prm->closure == PISOC_FOURIER) {
        ctx->tn = lay.t0;
        ctx->tk = lay.t1;
        fill_value(s, ctx->f<double>(ctx->tn), NT, prm->T0);
    }
    if (prm->time_scheme == PISOC_BDF2) {
        // t^{n-1} starts as the initial state (weighted by c2 = 0 in the first
        // step, but it must hold finite values)
        ctx->rm1 = lay.rm1;
        ctx->um1 = lay.um1;
        ctx->rjm1 = lay.rjm1;
        HIP_TRY(ctx, hipMemcpyAsync(ctx->f<double>(ctx->rm1), ctx->f<double>(ctx->rn),
                                    NT * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->f<double>(ctx->um1), ctx->f<double>(lay.u3[0]),
                                    3 * NT * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (prm->n_classes > 0)
            HIP_TRY(ctx, hipMemcpyAsync(ctx->f<double>(ctx->rjm1), ctx->f<double>(ctx->rhop),
                                        (size_t)prm->n_classes * NT * sizeof(double),
                                        hipMemcpyDeviceToDevice, s));
    }
    if (prm->guess == PISOC_GUESS_LEARNED)
        net_pack_forward(s, reinterpret_cast<const float*>(prm->d_guess_weights), ctx->ws + lay.wpk);
    return sync_state(ctx);
}

void free_ctx(pisoc_ctx* ctx) {
    if (!ctx) return;
    if (ctx->audit.have_events)
        for (auto& row : ctx->audit.ev)
            for (auto& e : row) (void)hipEventDestroy(e);
    // no publication may still be on its way into the buffer
    if (ctx->seq_host && ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->hst) (void)hipHostFree(ctx->hst);
    delete ctx;
}

// Copy out fields of member m (asynchronous).
pisoc_status member_fields(pisoc_ctx* ctx, int m, uint32_t which, double* const* d_dst) {
    const size_t N = ctx->N(), NT = ctx->NT(), off = (size_t)m * N;
    hipStream_t s = ctx->stream;
    const bool f64 = ctx->prm.precision == PISOC_FP64;
    int slot = 0;
    auto cast = [&](size_t boff, size_t comp_off, double* dst, double shift) {
        if (f64) Ops<double>::cast_out(s, ctx->f<double>(boff) + comp_off + off, dst, N, shift);
        else Ops<float>::cast_out(s, ctx->f<float>(boff) + comp_off + off, dst, N, shift);
    };
    const double* snap = ctx->prm.capture ? reinterpret_cast<double*>(ctx->ws + ctx->lay.snap)
                                          : nullptr;
    for (int bit = 0; bit < 32; ++bit) {
        const uint32_t mk = 1u << bit;
        if (!(which & mk)) continue;
        double* dst = d_dst[slot++];
        if (!dst) {
            ctx->err = "NULL destination";
            return PISOC_ERR_INVALID;
        }
        switch (mk) {
            case PISOC_FIELD_RHO: cast(ctx->rn, 0, dst, ctx->rho_ref[m]); break;
            case PISOC_FIELD_U:
                for (int d = 0; d < 3; ++d) cast(ctx->lay.u3[ctx->u_idx[0]], d * NT, dst + d * N, 0.0);
                break;
            case PISOC_FIELD_PHI:
                for (int d = 0; d < 3; ++d) cast(ctx->phin, d * NT, dst + d * N, 0.0);
                break;
            case PISOC_FIELD_RHO_P:
                for (int c = 0; c < ctx->prm.n_classes; ++c) cast(ctx->rhop, c * NT, dst + c * N, 0.0);
                break;
            case PISOC_FIELD_P:
                if (f64)
                    Ops<double>::pressure_out(s, ctx->ph, ctx->rho_ref[m], ctx->p_ref[m],
                                              ctx->f<double>(ctx->rn) + off, dst,
                                              ctx->ph.fourier ? ctx->f<double>(ctx->tn) + off
                                                              : nullptr);
                else
                    Ops<float>::pressure_out(s, ctx->ph, ctx->rho_ref[m], ctx->p_ref[m],
                                             ctx->f<float>(ctx->rn) + off, dst);
                break;
            case PISOC_FIELD_T:
                if (!ctx->ph.fourier) {
                    ctx->err = "temperature requested without the Fourier closure";
                    return PISOC_ERR_INVALID;
                }
                HIP_TRY(ctx, hipMemcpyAsync(dst, ctx->f<double>(ctx->tn) + off, N * sizeof(double),
                                            hipMemcpyDeviceToDevice, s));
                break;
            case PISOC_FIELD_PSOLVE_PSIDT:
                if (!snap) {
                    ctx->err = "captured pressure system requested without params.capture";
                    return PISOC_ERR_INVALID;
                }
                psidt_of(s, ctx->prm.n, snap + NT + off, snap + 4 * NT + off, dst);
                break;
            case PISOC_FIELD_PSOLVE_B:
            case PISOC_FIELD_PSOLVE_DIAG:
            case PISOC_FIELD_P_PREV:
            case PISOC_FIELD_PSOLVE_X:
            case PISOC_FIELD_PSOLVE_W:
            case PISOC_FIELD_USTAR:
            case PISOC_FIELD_GUESS:
            case PISOC_FIELD_GUESS_X0: {
                if (!snap) {
                    ctx->err = "captured pressure system requested without params.capture";
                    return PISOC_ERR_INVALID;
                }
                const bool gsel = mk == PISOC_FIELD_GUESS || mk == PISOC_FIELD_GUESS_X0;
                if (gsel && ctx->prm.guess == PISOC_GUESS_ZERO) {
                    ctx->err = "captured guess requested without a guess";
                    return PISOC_ERR_INVALID;
                }
                const int idx = mk == PISOC_FIELD_PSOLVE_B ? 0
                                : mk == PISOC_FIELD_PSOLVE_DIAG ? 1
                                : mk == PISOC_FIELD_P_PREV ? 2
                                : mk == PISOC_FIELD_PSOLVE_X ? 3
                                : mk == PISOC_FIELD_PSOLVE_W ? 4
                                : mk == PISOC_FIELD_USTAR ? 5
                                : mk == PISOC_FIELD_GUESS ? 8 : 9;
                const int comps = mk == PISOC_FIELD_USTAR ? 3 : 1;
                for (int d = 0; d < comps; ++d)
                    HIP_TRY(ctx, hipMemcpyAsync(dst + d * N, snap + (idx + d) * NT + off,
                                                N * sizeof(double), hipMemcpyDeviceToDevice, s));
                break;
            }
            default: ctx->err = "unknown field bit"; return PISOC_ERR_INVALID;
        }
    }
    HIP_TRY(ctx, hipGetLastError());
    return PISOC_OK;
}

// Statistics of every member (FP64 reductions); member m's in out[m].
pisoc_status all_stats(pisoc_ctx* ctx, pisoc_stats* out) {
    const double N = (double)ctx->N();
    const Phys& ph = ctx->ph;
    hipStream_t s = ctx->stream;
    const int B = ctx->batch;
    const bool f64 = ctx->prm.precision == PISOC_FP64;
    const unsigned nb = ctx->L.nblocks;
    auto gas = [&](auto tag) {
        using T = decltype(tag);
        Ops<T>::stats_gas(ctx->L, s, ph, ctx->st, ctx->f<T>(ctx->rn),
                          ctx->f<T>(ctx->lay.u3[ctx->u_idx[0]]), ctx->part(PS_STAT));
    };
    auto affine = [&](auto tag, size_t boff, size_t comp_off) {
        using T = decltype(tag);
        Ops<T>::sum_affine_sq(ctx->L, s, ph, ctx->st, ctx->f<T>(boff) + comp_off, 0.0, 0.0,
                              ctx->part(PS_STAT));
    };
    if (f64) gas(double{}); else gas(float{});
    finalize_sums(s, ctx->part(PS_STAT), nb, B, 4, ctx->st, 0);
    // density variance about the member's mean
    set_affine(s, ctx->st, B, 0, N);
    if (f64) affine(double{}, ctx->rn, 0); else affine(float{}, ctx->rn, 0);
    finalize_sums(s, ctx->part(PS_STAT), nb, B, 2, ctx->st, 4);
    if (ph.fourier) {   // sum T into red[6]
        Ops<double>::sum_affine_sq(ctx->L, s, ph, nullptr, ctx->f<double>(ctx->tn), 0.0, 0.0,
                                   ctx->part(PS_STAT));
        finalize_sums(s, ctx->part(PS_STAT), nb, B, 2, ctx->st, 5);
    }
    pisoc_status st = sync_state(ctx);
    if (st != PISOC_OK) return st;
    for (int m = 0; m < B; ++m) {
        const DevState& h = ctx->hst[m];
        pisoc_stats& o = out[m];
        std::memset(&o, 0, sizeof(o));
        const double rmean = ctx->rho_ref[m] + h.red[3] / N;
        const double C = ctx->p_ref[m] / std::pow(ctx->rho_ref[m], ph.gamma);
        o.ke = h.red[0] / N;
        o.enstrophy = h.red[1] / N;
        o.rho_rms = std::sqrt(h.red[4] / N) / rmean;
        // sound speed of the mean state: gamma C <rho>^(gamma-1), or for the
        // ideal gas (1 + R/c_v) R <T>
        const double c0sq = ph.fourier ? (1.0 + ph.R / ph.cv) * ph.R * (h.red[6] / N)
                                       : ph.gamma * C * std::pow(rmean, ph.gamma - 1.0);
        o.mach_rms = std::sqrt(h.red[2] / N) / std::sqrt(c0sq);
        o.mass_gas = rmean * N * ph.V;
    }
    const size_t NT = ctx->NT();
    for (int c = 0; c < ctx->prm.n_classes; ++c) {
        set_affine(s, ctx->st, B, 1, N);
        if (f64) affine(double{}, ctx->rhop, c * NT); else affine(float{}, ctx->rhop, c * NT);
        finalize_sums(s, ctx->part(PS_STAT), nb, B, 2, ctx->st, 4);
        set_affine(s, ctx->st, B, 2, N);
        if (f64) affine(double{}, ctx->rhop, c * NT); else affine(float{}, ctx->rhop, c * NT);
        finalize_sums(s, ctx->part(PS_STAT), nb, B, 1, ctx->st, 6);
        if ((st = sync_state(ctx)) != PISOC_OK) return st;
        for (int m = 0; m < B; ++m) {
            const double mean = ctx->hst[m].red[5] / N;
            out[m].conc_var[c] = mean != 0.0 ? ctx->hst[m].red[6] / N : 0.0;
            out[m].mass_p[c] = mean * N * ph.V;
        }
    }
    return PISOC_OK;
}

// ---------------------------------------------------------------- autotuner
// Launch shapes of the field kernels are tuned per (n, members, precision,
// dust classes): each candidate (bx, cz) times a representative set of field
// kernels -- a predictor sweep, H/A, the corrector set-up, kProbeCgIters CG
// iterations and a dust sweep -- on the context's own buffers (all of them
// scratch between steps; the persistent state is only read), and the fastest
// wins; the tiled kernels' and the CG kernel's z-chunks are then chosen the
// same way.  Winners are kept in a small JSON object
// {"key": [bx, cz, CG planes, tile planes], ...}.
std::string tune_key(const pisoc_ctx* ctx) {
    char b[96];
    std::snprintf(b, sizeof(b), "n%d_b%d_%s_k%d_g%d", ctx->prm.n, ctx->batch,
                  ctx->prm.precision == PISOC_FP64 ? "fp64" : "fp32", ctx->prm.n_classes,
                  ctx->prm.guess);
    return b;
}

// An entry is [block x, cells per thread along z, CG tile planes, field tile
// planes] (0: that kernel has no tile form at this size).
bool cache_lookup(const std::string& text, const std::string& key, int* bx, int* cz, int* cgz,
                  int* tlz) {
    const std::string pat = "\"" + key + "\"";
    size_t at = text.find(pat);
    if (at == std::string::npos) return false;
    at = text.find('[', at + pat.size());
    if (at == std::string::npos) return false;
    return std::sscanf(text.c_str() + at, "[%d , %d , %d , %d]", bx, cz, cgz, tlz) == 4 ||
           std::sscanf(text.c_str() + at, "[%d,%d,%d,%d]", bx, cz, cgz, tlz) == 4;
}

std::string read_file(const char* path) {
    std::string out;
    if (!path) return out;
    FILE* f = std::fopen(path, "rb");
    if (!f) return out;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) out.append(buf, k);
    std::fclose(f);
    return out;
}

// Rewrite the cache with the entry for key replaced or added.
bool cache_store(const char* path, const std::string& key, int bx, int cz, int cgz, int tlz) {
    std::string text = read_file(path);
    std::vector<std::pair<std::string, std::array<int, 4>>> entries;
    size_t pos = 0;
    for (;;) {
        const size_t q0 = text.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = text.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const std::string k = text.substr(q0 + 1, q1 - q0 - 1);
        int a, b, c, d;
        if (cache_lookup(text.substr(q0), k, &a, &b, &c, &d) && k != key)
            entries.push_back({k, {a, b, c, d}});
        pos = text.find(']', q1);
        if (pos == std::string::npos) break;
    }
    entries.push_back({key, {bx, cz, cgz, tlz}});
    FILE* f = std::fopen(path, "wb");
    if (!f) return false;
    std::fprintf(f, "{\n");
    for (size_t i = 0; i < entries.size(); ++i)
        std::fprintf(f, "  \"%s\": [%d, %d, %d, %d]%s\n", entries[i].first.c_str(),
                     entries[i].second[0], entries[i].second[1], entries[i].second[2],
                     entries[i].second[3], i + 1 < entries.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    return true;
}

// CG iterations in a launch-shape probe
constexpr int kProbeCgIters = 12;
template <typename T>
void enqueue_probe(pisoc_ctx* ctx) {
    using O = Ops<T>;
    StepPtrs<T> S = step_ptrs<T>(ctx);
    const Phys& ph = ctx->ph;
    const Launch& L = ctx->L;
    hipStream_t s = ctx->stream;
    DevState* st = ctx->st;
    O::mom_sweep(L, ctx->TL, s, ph, st, S.un, S.ua, S.phin, S.aP, S.src, S.pn);
    O::hbya(L, ctx->TL, s, ph, st, S.ua, S.hb, S.phin, S.aP, S.src, S.rk, S.w, S.p0);
    const unsigned nb0 = O::corr_rhs(L, ctx->TL, s, ph, st, S.rn, S.rk, S.w, S.hb, S.p0, S.phiH,
                                     S.r, S.dg, ctx->part(PS_U), nullptr, nullptr, nullptr, S.b64);
    // CG iterations that cannot converge (tolerance 0), about as many against
    // the field kernels as in a step (two solves of 10-20 iterations each
    // against 6-8 momentum sweeps)
    set_tol(s, st, ctx->batch, 0.0);
    (void)run_pcg<T>(ctx, cg_vecs(S), true, kProbeCgIters, false, nullptr, true, nb0);
    if (ctx->prm.n_classes > 0)
        (void)O::dust_sweep(L, ctx->TL, s, ph, st, S.Ya, S.Yb, S.G, S.rj, S.rk, nullptr);
}

// The CG kernel's tile launch with z-chunks of cgz planes (0: the default).
void set_cg_chunk(pisoc_ctx* ctx, int cgz) {
    ctx->TS = make_spmv_launch(ctx->prm.n, ctx->batch, (int)ctx->es, cgz);
}

// Only the tile form of the CG kernel takes a tuned z-chunk.
bool cg_tunable(const pisoc_ctx* ctx) { return ctx->TS.nblocks && ctx->TS.v == 0; }

// The default chunk d0, then 8, 16 and 32 planes (at most n), each once.
std::vector<int> chunk_candidates(int n, int d0) {
    std::vector<int> out{d0};
    for (int c : {8, 16, 32})
        if (c <= n && std::find(out.begin(), out.end(), c) == out.end()) out.push_back(c);
    return out;
}
std::vector<int> cg_chunk_candidates(const pisoc_ctx* ctx) {
    return chunk_candidates(ctx->prm.n, make_spmv_launch(ctx->prm.n, ctx->batch, (int)ctx->es).cz);
}

// The same for the tiled field kernels' launch.
void set_tl_chunk(pisoc_ctx* ctx, int tlz) { ctx->TL = make_tiled_launch(ctx->prm.n, ctx->batch, tlz); }
bool tl_tunable(const pisoc_ctx* ctx) { return ctx->TL.nblocks != 0; }
std::vector<int> tl_chunk_candidates(const pisoc_ctx* ctx) {
    return chunk_candidates(ctx->prm.n, make_tiled_launch(ctx->prm.n, ctx->batch).cz);
}

// Launch shapes of one size class: the gathered kernels' block and cells per
// thread (timed over the shape candidates), then, with that shape, the tiled
// field kernels' z-chunk and last the CG kernel's tile z-chunk (each timed
// over its chunk candidates), each by the probe step; or the cached choice.
pisoc_status tune_ctx(pisoc_ctx* ctx, const char* cache_path, int force, int* bx_out, int* cz_out) {
    const std::string key = tune_key(ctx);
    const bool cgt = cg_tunable(ctx), tlt = tl_tunable(ctx);
    int bx = 0, cz = 0, cgz = 0, tlz = 0;
    if (!force && cache_lookup(read_file(cache_path), key, &bx, &cz, &cgz, &tlz)) {
        bool ok = false, okc = !cgt && cgz == 0, okt = !tlt && tlz == 0;
        for (auto [a, b] : shape_candidates(ctx->prm.n)) ok = ok || (a == bx && b == cz);
        if (cgt)
            for (int c : cg_chunk_candidates(ctx)) okc = okc || c == cgz;
        if (tlt)
            for (int c : tl_chunk_candidates(ctx)) okt = okt || c == tlz;
        if (ok && okc && okt) {
            set_shape(ctx, make_launch_shaped(ctx->prm.n, ctx->batch, bx, cz));
            if (tlt) set_tl_chunk(ctx, tlz);
            if (cgt) set_cg_chunk(ctx, cgz);
            *bx_out = bx;
            *cz_out = cz;
            return PISOC_OK;
        }
    }
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    auto probe = [&] {
        if (ctx->prm.precision == PISOC_FP64) enqueue_probe<double>(ctx);
        else enqueue_probe<float>(ctx);
    };
    // time of three probe steps after a warm-up one, or a negative value
    auto time_probe = [&]() -> float {
        probe();
        (void)hipEventRecord(e0, ctx->stream);
        for (int rep = 0; rep < 3; ++rep) probe();
        (void)hipEventRecord(e1, ctx->stream);
        if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
        float ms = 0.f;
        return hipEventElapsedTime(&ms, e0, e1) == hipSuccess ? ms : -1.f;
    };
    float best = 1e30f;
    int best_bx = 0, best_cz = 0, best_cgz = 0, best_tlz = 0;
    const Launch L0 = ctx->L;
    for (auto [a, b] : shape_candidates(ctx->prm.n)) {
        set_shape(ctx, make_launch_shaped(ctx->prm.n, ctx->batch, a, b));
        const float ms = time_probe();
        if (ms < 0.f) break;
        if (ms < best) {
            best = ms;
            best_bx = a;
            best_cz = b;
        }
    }
    if (best_bx != 0) set_shape(ctx, make_launch_shaped(ctx->prm.n, ctx->batch, best_bx, best_cz));
    if (best_bx != 0 && tlt) {
        float best_t = 1e30f;
        for (int c : tl_chunk_candidates(ctx)) {
            set_tl_chunk(ctx, c);
            const float ms = time_probe();
            if (ms < 0.f) break;
            if (ms < best_t) {
                best_t = ms;
                best_tlz = c;
            }
        }
        set_tl_chunk(ctx, best_tlz);
    }
    if (best_bx != 0 && cgt) {
        float best_c = 1e30f;
        for (int c : cg_chunk_candidates(ctx)) {
            set_cg_chunk(ctx, c);
            const float ms = time_probe();
            if (ms < 0.f) break;
            if (ms < best_c) {
                best_c = ms;
                best_cgz = c;
            }
        }
        set_cg_chunk(ctx, best_cgz);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->prof.on = prof;
    HIP_TRY(ctx, hipGetLastError());
    if (best_bx == 0 || (cgt && best_cgz == 0) || (tlt && best_tlz == 0)) {
        set_shape(ctx, L0);
        if (tlt) set_tl_chunk(ctx, 0);
        if (cgt) set_cg_chunk(ctx, 0);
        ctx->err = "no launch shape could be timed";
        return PISOC_ERR_HIP;
    }
    if (cache_path && !cache_store(cache_path, key, best_bx, best_cz, best_cgz, best_tlz)) {
        ctx->err = std::string("cannot write ") + cache_path;
        return PISOC_ERR_INVALID;
    }
    *bx_out = best_bx;
    *cz_out = best_cz;
    return PISOC_OK;
}

}  // namespace

// ============================================================ ensemble object
struct pisoc_ens {
    int count = 0;
    std::vector<pisoc_ctx*> cls;                  // one context per grid size
    std::vector<std::pair<int, int>> where;       // member -> (class, index in class)
    std::vector<std::vector<int>> members;        // class -> member ids
    std::vector<hipStream_t> streams;             // one per class
    // captured step of each class (replayed on its own stream), per buffer parity
    std::vector<std::array<hipGraphExec_t, 2>> exec;
    // or, in one_graph mode, one graph holding every class's step as a branch
    // (forked from and joined into the first class's stream), per parity
    std::array<hipGraphExec_t, 2> one{nullptr, nullptr};
    bool one_graph = false;        // which kind the built graphs are
    std::vector<hipEvent_t> fork_join;   // [0]: fork; [c]: join of class c
    int parity = 0;
    bool built = false;
    int64_t steps = 0;
    std::string err;
};

namespace {

void drop_graphs(pisoc_ens* e) {
    for (auto& pair : e->exec)
        for (auto& g : pair)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    for (auto& g : e->one)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    e->built = false;
}

// CG caps of the captured step from the iterations the members needed
// (margin 25% + 2), and the refinement rounds (one more than needed: the
// rounds a solve takes vary from step to step by one where the residual after
// a round lands near the tolerance).
void set_caps(pisoc_ctx* ctx, const int* first, int later, int rounds) {
    for (int c = 0; c < ctx->prm.n_corr; ++c)
        ctx->caps[c] = std::max(ctx->caps[c], (int)std::ceil(1.25 * first[c]) + 2);
    ctx->cap_later = std::max(ctx->cap_later, (int)std::ceil(1.25 * later) + 2);
    ctx->rounds = std::max(ctx->rounds, std::max(1, std::min(rounds + 1, ctx->prm.max_refine)));
}

// One graph per parity holding every class's step: the capture begins on the
// first class's stream, the other class streams join it through a fork event
// and are joined back before it ends, so each class is a branch of the graph.
pisoc_status build_one_graph(pisoc_ens* e) {
    drop_graphs(e);
    for (pisoc_ctx* ctx : e->cls)
        if (audit_on(ctx)) audit_decide_capture(ctx);
    const size_t C = e->cls.size();
    if (e->fork_join.size() != C) {
        for (hipEvent_t ev : e->fork_join) (void)hipEventDestroy(ev);
        e->fork_join.assign(C, nullptr);
        for (size_t c = 0; c < C; ++c)
            if (hipEventCreateWithFlags(&e->fork_join[c], hipEventDisableTiming) != hipSuccess) {
                e->err = "hipEventCreate failed";
                return PISOC_ERR_HIP;
            }
    }
    hipStream_t origin = e->cls[0]->stream;
    auto fail = [&](int par, pisoc_status st, const std::string& why) {
        e->err = why;
        if (par == 1)
            for (pisoc_ctx* ctx : e->cls) rotate(ctx);
        drop_graphs(e);
        return st;
    };
    for (int par = 0; par < 2; ++par) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(par, PISOC_ERR_HIP, "hipStreamBeginCapture failed");
        bool ok = hipEventRecord(e->fork_join[0], origin) == hipSuccess;
        for (size_t c = 1; c < C && ok; ++c)
            ok = hipStreamWaitEvent(e->cls[c]->stream, e->fork_join[0], 0) == hipSuccess;
        pisoc_status st = PISOC_OK;
        for (size_t c = 0; c < C && ok && st == PISOC_OK; ++c) {
            pisoc_ctx* ctx = e->cls[c];
            st = ctx->prm.precision == PISOC_FP64 ? enqueue_step<double>(ctx, false)
                                                  : enqueue_step<float>(ctx, false);
            if (st != PISOC_OK) e->err = ctx->err;
        }
        for (size_t c = 1; c < C && ok; ++c)
            ok = hipEventRecord(e->fork_join[c], e->cls[c]->stream) == hipSuccess &&
                 hipStreamWaitEvent(origin, e->fork_join[c], 0) == hipSuccess;
        const hipError_t rc_end = hipStreamEndCapture(origin, &g);
        if (!ok || st != PISOC_OK || rc_end != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return fail(par, st != PISOC_OK ? st : PISOC_ERR_HIP,
                        std::string("graph capture failed: ") +
                            (st != PISOC_OK ? e->err : std::string(hipGetErrorString(rc_end))));
        }
        const hipError_t rc = hipGraphInstantiate(&e->one[par], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (rc != hipSuccess) {
            e->one[par] = nullptr;
            return fail(par, PISOC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(rc));
        }
        for (pisoc_ctx* ctx : e->cls) rotate(ctx);
    }
    for (pisoc_ctx* ctx : e->cls) {
        std::copy(ctx->caps, ctx->caps + PISOC_MAX_CORR, ctx->caps_built);
        ctx->cap_later_built = ctx->cap_later;
    }
    e->built = true;
    e->one_graph = true;
    e->parity = 0;
    return PISOC_OK;
}

// Capture one step of each class on its own stream into exec[c][0], then,
// with the buffers rotated, into exec[c][1]; rotations restored.  The classes
// are independent graphs so that their replays on the class streams overlap.
pisoc_status build_class_graphs(pisoc_ens* e) {
    drop_graphs(e);
    e->exec.assign(e->cls.size(), {nullptr, nullptr});
    for (pisoc_ctx* ctx : e->cls)
        if (audit_on(ctx)) audit_decide_capture(ctx);
    // on failure: no graph kept, the buffers' rotation as before the call
    auto fail = [&](int par, pisoc_status st, const std::string& why) {
        e->err = why;
        if (par == 1)
            for (pisoc_ctx* ctx : e->cls) rotate(ctx);
        drop_graphs(e);
        return st;
    };
    for (int par = 0; par < 2; ++par) {
        for (size_t c = 0; c < e->cls.size(); ++c) {
            pisoc_ctx* ctx = e->cls[c];
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return fail(par, PISOC_ERR_HIP, "hipStreamBeginCapture failed");
            const pisoc_status st = ctx->prm.precision == PISOC_FP64 ? enqueue_step<double>(ctx, false)
                                                                     : enqueue_step<float>(ctx, false);
            const hipError_t rc_end = hipStreamEndCapture(ctx->stream, &g);
            if (st != PISOC_OK || rc_end != hipSuccess || !g) {
                if (g) (void)hipGraphDestroy(g);
                return fail(par, st != PISOC_OK ? st : PISOC_ERR_HIP,
                            std::string("graph capture failed: ") +
                                (st != PISOC_OK ? ctx->err : std::string(hipGetErrorString(rc_end))));
            }
            const hipError_t rc = hipGraphInstantiate(&e->exec[c][par], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (rc != hipSuccess) {
                e->exec[c][par] = nullptr;
                return fail(par, PISOC_ERR_HIP,
                            std::string("hipGraphInstantiate: ") + hipGetErrorString(rc));
            }
        }
        for (pisoc_ctx* ctx : e->cls) rotate(ctx);
    }
    for (pisoc_ctx* ctx : e->cls) {
        std::copy(ctx->caps, ctx->caps + PISOC_MAX_CORR, ctx->caps_built);
        ctx->cap_later_built = ctx->cap_later;
    }
    e->built = true;
    e->one_graph = false;
    e->parity = 0;
    return PISOC_OK;
}

// The graphs of the kind a captured mode replays (mode PISOC_ENS_GRAPH: one per
// class; PISOC_ENS_GRAPH_ONE: one for the whole ensemble).
pisoc_status build_graphs(pisoc_ens* e, bool one) {
    return one ? build_one_graph(e) : build_class_graphs(e);
}

bool same_class_params(const pisoc_params& a, const pisoc_params& b) {
    return a.n_classes == b.n_classes && a.gamma == b.gamma && a.mu == b.mu && a.cfl == b.cfl &&
           a.dt_growth == b.dt_growth && a.dt_fixed == b.dt_fixed && a.dt_max == b.dt_max &&
           a.n_corr == b.n_corr && a.n_mom_sweeps == b.n_mom_sweeps &&
           a.n_dust_sweeps == b.n_dust_sweeps && a.p_tol == b.p_tol && a.p_maxit == b.p_maxit &&
           a.precision == b.precision && a.guess == b.guess &&
           a.d_guess_weights == b.d_guess_weights && a.inner_tol == b.inner_tol &&
           a.max_refine == b.max_refine && a.capture == b.capture &&
           a.guess_audit == b.guess_audit && a.two_way == b.two_way &&
           a.gravity[0] == b.gravity[0] && a.gravity[1] == b.gravity[1] &&
           a.gravity[2] == b.gravity[2];
}

// Size classes in order of first appearance; returns false on invalid input.
bool ens_classes(const pisoc_params* members, int32_t count, std::vector<std::vector<int>>* out,
                 std::string* why) {
    out->clear();
    if (!members || count < 1) {
        if (why) *why = "no members";
        return false;
    }
    for (int m = 0; m < count; ++m) {
        if (!valid_params(&members[m], why)) return false;
        if (members[m].closure != PISOC_BAROTROPIC || members[m].time_scheme != PISOC_BDF1 ||
            members[m].mom_tol > 0.0) {
            if (why) *why = "ensembles take the barotropic closure, backward Euler and the "
                            "swept momentum predictor only";
            return false;
        }
        if (!same_class_params(members[m], members[0])) {
            if (why) *why = "members may differ only in n, C and tau_p";
            return false;
        }
        bool placed = false;
        for (auto& c : *out)
            if (members[c[0]].n == members[m].n) {
                c.push_back(m);
                placed = true;
                break;
            }
        if (!placed) out->push_back({m});
    }
    return true;
}

std::vector<size_t> ens_offsets(const pisoc_params* members,
                                const std::vector<std::vector<int>>& classes, size_t* total) {
    std::vector<size_t> off;
    size_t o = 0;
    for (const auto& c : classes) {
        off.push_back(o);
        o = align_up(o + make_layout(&members[c[0]], (int)c.size()).total);
    }
    *total = o;
    return off;
}

// Every class synchronised and its device state copied to the host.
pisoc_status ens_sync(pisoc_ens* e) {
    for (pisoc_ctx* ctx : e->cls) {
        pisoc_status st = sync_state(ctx);
        if (st != PISOC_OK) {
            e->err = ctx->err;
            return st;
        }
    }
    return PISOC_OK;
}

}  // namespace

// ============================================================ C ABI
extern "C" {

size_t pisoc_workspace_bytes(const pisoc_params* prm) {
    if (!valid_params(prm, nullptr)) return 0;
    return make_layout(prm, 1).total;
}

const char* pisoc_status_string(pisoc_status st) {
    switch (st) {
        case PISOC_OK: return "ok";
        case PISOC_WARN_NOT_CONVERGED: return "pressure solve did not converge";
        case PISOC_WARN_GUESS_FALLBACK: return "learned guess rejected";
        case PISOC_WARN_DUST: return "dust density negative or dust diagonal non-positive";
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
    const Layout lay = make_layout(prm, 1);
    if (!d_workspace || ws_bytes < lay.total ||
        (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return PISOC_ERR_WORKSPACE;
    pisoc_ctx* ctx = new (std::nothrow) pisoc_ctx();
    if (!ctx) return PISOC_ERR_INVALID;
    const pisoc_status st = init_ctx(ctx, prm, 1, reinterpret_cast<char*>(d_workspace), &d_rho,
                                     &d_u, &d_rho_p, reinterpret_cast<hipStream_t>(hip_stream));
    if (st != PISOC_OK) {
        free_ctx(ctx);
        return st;
    }
    *out = ctx;
    return PISOC_OK;
}

pisoc_status pisoc_step(pisoc_ctx* ctx, int32_t n_steps, pisoc_step_info* h_info) {
    if (!ctx || n_steps < 0) return PISOC_ERR_INVALID;
    pisoc_status worst = PISOC_OK;
    for (int i = 0; i < n_steps; ++i) {
        const pisoc_status s = eager_step(ctx, h_info ? h_info + i : nullptr);
        if (s < 0) return s;
        worst = combine_status(worst, s);
    }
    return worst;
}

pisoc_status pisoc_fields(pisoc_ctx* ctx, uint32_t which, double* const* d_dst) {
    if (!ctx || !d_dst) return PISOC_ERR_INVALID;
    return member_fields(ctx, 0, which, d_dst);
}

pisoc_status pisoc_set_temperature(pisoc_ctx* ctx, const double* d_T) {
    if (!ctx || !d_T) return PISOC_ERR_INVALID;
    if (!ctx->ph.fourier) {
        ctx->err = "pisoc_set_temperature needs the Fourier closure";
        return PISOC_ERR_INVALID;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->f<double>(ctx->tn), d_T, ctx->N() * sizeof(double),
                                hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PISOC_OK;
}

pisoc_status pisoc_get_stats(pisoc_ctx* ctx, pisoc_stats* out) {
    if (!ctx || !out) return PISOC_ERR_INVALID;
    return all_stats(ctx, out);
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

void pisoc_destroy(pisoc_ctx* ctx) { free_ctx(ctx); }

const char* pisoc_last_error(const pisoc_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

// ---------------------------------------------------------------- ensembles
size_t pisoc_ens_workspace_bytes(const pisoc_params* members, int32_t count) {
    std::vector<std::vector<int>> classes;
    if (!ens_classes(members, count, &classes, nullptr)) return 0;
    size_t total = 0;
    (void)ens_offsets(members, classes, &total);
    return total;
}

pisoc_status pisoc_ens_init(const pisoc_params* members, int32_t count, void* d_workspace,
                            size_t ws_bytes, const double* const* d_rho, const double* const* d_u,
                            const double* const* d_rho_p, void* hip_stream, pisoc_ens** out) {
    if (!out) return PISOC_ERR_INVALID;
    *out = nullptr;
    std::vector<std::vector<int>> classes;
    if (!ens_classes(members, count, &classes, nullptr) || !d_rho || !d_u) return PISOC_ERR_INVALID;
    for (int m = 0; m < count; ++m)
        if (!d_rho[m] || !d_u[m] || (members[m].n_classes > 0 && (!d_rho_p || !d_rho_p[m])))
            return PISOC_ERR_INVALID;
    size_t total = 0;
    const std::vector<size_t> off = ens_offsets(members, classes, &total);
    if (!d_workspace || ws_bytes < total || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return PISOC_ERR_WORKSPACE;
    pisoc_ens* e = new (std::nothrow) pisoc_ens();
    if (!e) return PISOC_ERR_INVALID;
    e->count = count;
    e->members = classes;
    e->where.assign(count, {0, 0});
    pisoc_status st = PISOC_OK;
    // class streams wait for the caller's stream (the inputs) before the set-up
    hipEvent_t ready = nullptr;
    if (st == PISOC_OK &&
        (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
         hipEventRecord(ready, reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess))
        st = PISOC_ERR_HIP;
    for (size_t c = 0; c < classes.size() && st == PISOC_OK; ++c) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            st = PISOC_ERR_HIP;
            break;
        }
        e->streams.push_back(s);
        if (hipStreamWaitEvent(s, ready, 0) != hipSuccess) {
            st = PISOC_ERR_HIP;
            break;
        }
        std::vector<pisoc_params> mp;
        std::vector<const double*> r, u, rp;
        for (size_t i = 0; i < classes[c].size(); ++i) {
            const int m = classes[c][i];
            e->where[m] = {(int)c, (int)i};
            mp.push_back(members[m]);
            r.push_back(d_rho[m]);
            u.push_back(d_u[m]);
            rp.push_back(d_rho_p ? d_rho_p[m] : nullptr);
        }
        pisoc_ctx* ctx = new (std::nothrow) pisoc_ctx();
        if (!ctx) {
            st = PISOC_ERR_INVALID;
            break;
        }
        e->cls.push_back(ctx);
        st = init_ctx(ctx, mp.data(), (int)mp.size(), reinterpret_cast<char*>(d_workspace) + off[c],
                      r.data(), u.data(), rp.data(), s);
        if (st != PISOC_OK) e->err = ctx->err;
    }
    if (ready) (void)hipEventDestroy(ready);
    if (st != PISOC_OK) {
        pisoc_ens_destroy(e);
        return st;
    }
    *out = e;
    return PISOC_OK;
}

pisoc_status pisoc_ens_step(pisoc_ens* e, int32_t n_steps, int32_t mode, pisoc_step_info* h_info) {
    if (!e || n_steps < 0 ||
        (mode != PISOC_ENS_EAGER && mode != PISOC_ENS_GRAPH && mode != PISOC_ENS_GRAPH_ONE))
        return PISOC_ERR_INVALID;
    if (n_steps == 0) return PISOC_OK;
    pisoc_status worst = PISOC_OK;
    std::vector<pisoc_step_info> rec(e->count);
    const bool one = mode == PISOC_ENS_GRAPH_ONE;
    // graphs of the other captured kind are dropped; this call captures its own
    if (mode != PISOC_ENS_EAGER && e->built && e->one_graph != one) drop_graphs(e);
    if (mode == PISOC_ENS_EAGER || !e->built) {
        // eager steps.  A captured call begins with one, which measures the CG
        // iterations that size the graph's caps, or with two where the
        // learned-guess audit has yet to measure both of its choices (the
        // capture takes its verdict); the graph is built once that is done.
        int k = n_steps;
        if (mode != PISOC_ENS_EAGER) {
            int need = 1;
            for (pisoc_ctx* ctx : e->cls)
                if (audit_on(ctx) && !audit_measured(ctx))
                    need = std::max(need, ctx->audit.it_guess[0] < 0.0 ? 2 : 1);
            k = std::min(n_steps, need);
        }
        for (int i = 0; i < k; ++i) {
            for (size_t c = 0; c < e->cls.size(); ++c) {
                pisoc_ctx* ctx = e->cls[c];
                std::vector<pisoc_step_info> ci(ctx->batch);
                const pisoc_status s = eager_step(ctx, ci.data());
                if (s < 0) {
                    e->err = ctx->err;
                    return s;
                }
                worst = combine_status(worst, s);
                // the call's records: each member's last step, flags of all its steps
                for (int j = 0; j < ctx->batch; ++j) {
                    pisoc_step_info& r = rec[e->members[c][j]];
                    const int32_t before = r.flags;
                    r = ci[j];
                    r.flags |= before;
                }
                // iterations for the caps of the captured step
                int first[PISOC_MAX_CORR] = {0, 0, 0, 0};
                int later = 0, rounds = 1;
                for (int j = 0; j < ctx->batch; ++j) {
                    const DevState& h = ctx->hst[j];
                    for (int q = 0; q < ctx->prm.n_corr; ++q) {
                        first[q] = std::max(first[q], h.it_first[q]);
                        rounds = std::max(rounds, h.rounds_corr[q]);
                    }
                    for (int q = 0; q < ctx->prm.n_corr; ++q) later = std::max(later, h.it_later[q]);
                }
                set_caps(ctx, first, later, rounds);
            }
            e->steps += 1;
            // the eager step rotated the buffers: graphs already built stay valid
            // for the other parity (their kernel arguments are the rotation's
            // pointers), so the next replay takes exec[c][parity ^ 1]
            if (e->built) e->parity ^= 1;
        }
        if (mode == PISOC_ENS_EAGER) {
            if (h_info) std::copy(rec.begin(), rec.end(), h_info);
            return worst;
        }
        n_steps -= k;
        bool ready = true;
        for (pisoc_ctx* ctx : e->cls)
            if (audit_on(ctx) && !audit_measured(ctx)) ready = false;
        if (!ready) {
            if (h_info) std::copy(rec.begin(), rec.end(), h_info);
            return worst;
        }
        pisoc_status st = build_graphs(e, one);
        if (st != PISOC_OK) {
            // the eager steps of this call stand; their records go out with the error
            if (h_info) std::copy(rec.begin(), rec.end(), h_info);
            return st;
        }
    }
    if (n_steps > 0) {
        // each class's graph runs on the class stream, after the work already
        // there (set-up, eager steps, copies)
        for (pisoc_ctx* ctx : e->cls) clear_acc(ctx->stream, ctx->st, ctx->batch);
        if (e->one_graph) {
            // the whole-ensemble graph runs on the first class's stream, after
            // the work already on every class stream
            hipStream_t origin = e->cls[0]->stream;
            for (size_t c = 1; c < e->cls.size(); ++c)
                if (hipEventRecord(e->fork_join[c], e->cls[c]->stream) != hipSuccess ||
                    hipStreamWaitEvent(origin, e->fork_join[c], 0) != hipSuccess) {
                    e->err = "hipEventRecord/hipStreamWaitEvent failed";
                    return PISOC_ERR_HIP;
                }
        }
        for (int i = 0; i < n_steps; ++i) {
            if (e->one_graph) {
                const hipError_t rc = hipGraphLaunch(e->one[e->parity], e->cls[0]->stream);
                if (rc != hipSuccess) {
                    e->err = std::string("hipGraphLaunch: ") + hipGetErrorString(rc);
                    return PISOC_ERR_HIP;
                }
            }
            for (size_t c = 0; c < e->cls.size() && !e->one_graph; ++c) {
                const hipError_t rc = hipGraphLaunch(e->exec[c][e->parity], e->cls[c]->stream);
                if (rc != hipSuccess) {
                    e->err = std::string("hipGraphLaunch: ") + hipGetErrorString(rc);
                    return PISOC_ERR_HIP;
                }
            }
            e->parity ^= 1;
            for (pisoc_ctx* ctx : e->cls) {
                rotate(ctx);
                ctx->steps += 1;
            }
            e->steps += 1;
        }
        if (e->one_graph) {
            // every class stream waits for the graphs on the first class's
            // stream before its own next work (the state read-back below first)
            hipStream_t origin = e->cls[0]->stream;
            bool ok = hipEventRecord(e->fork_join[0], origin) == hipSuccess;
            for (size_t c = 1; c < e->cls.size() && ok; ++c)
                ok = hipStreamWaitEvent(e->cls[c]->stream, e->fork_join[0], 0) == hipSuccess;
            if (!ok) {
                e->err = "hipEventRecord/hipStreamWaitEvent failed";
                return PISOC_ERR_HIP;
            }
        }
        pisoc_status st = ens_sync(e);
        if (st != PISOC_OK) return st;
        bool regrow_any = false, near_any = false, bad = false, bad_dt = false;
        for (size_t c = 0; c < e->cls.size(); ++c) {
            pisoc_ctx* ctx = e->cls[c];
            int first[PISOC_MAX_CORR] = {0, 0, 0, 0};
            int later = 0;
            bool regrow = false;
            int skipped = 0;
            if (audit_on(ctx))
                for (int q = 0; q < ctx->prm.n_corr; ++q)
                    skipped |= ctx->audit.use[q] ? 0 : PISOC_FLAG_GUESS_SKIPPED;
            for (int j = 0; j < ctx->batch; ++j) {
                const DevState& h = ctx->hst[j];
                pisoc_step_info& r = rec[e->members[c][j]];
                const int32_t before = r.flags;   // the call's leading eager steps
                fill_info(ctx, h, true, &r);
                r.flags |= h.flags_acc | skipped | before;
                worst = combine_status(worst, flag_status(h.flags_acc));
                if (member_bad(ctx, h) ||
                    (h.flags_acc & (PISOC_FLAG_NONFINITE | PISOC_FLAG_RHO_NONPOS | PISOC_FLAG_DUST_NONFINITE)))
                    bad = true;
                for (int q = 0; q < ctx->prm.n_corr; ++q) first[q] = std::max(first[q], h.it_first_max[q]);
                for (int q = 0; q < ctx->prm.n_corr; ++q) later = std::max(later, h.it_later_max[q]);
                if (h.flags_acc & PISOC_FLAG_PCG_MAXIT) regrow = true;
                if (h.flags_acc & PISOC_FLAG_BAD_DT) bad_dt = true;
            }
            if (regrow) {
                // a solve hit its cap: grow the caps by half and re-capture
                for (int q = 0; q < ctx->prm.n_corr; ++q)
                    if (first[q] >= ctx->caps[q]) ctx->caps[q] = ctx->caps[q] * 3 / 2 + 2;
                if (later >= ctx->cap_later) ctx->cap_later = ctx->cap_later * 3 / 2 + 2;
                ctx->rounds = std::min(ctx->prm.max_refine, ctx->rounds + 1);
            }
            set_caps(ctx, first, later, ctx->rounds - 1);
            regrow_any = regrow_any || regrow;
            // the iterations have come within 10 % + 2 of the caps the graphs
            // hold (they grow as the flow decays, by several within a long
            // call): capture again with the tracked caps (+25 % + 2) before a
            // solve runs into them
            auto near = [](int it, int cap) { return (int)std::ceil(1.1 * it) + 2 > cap; };
            for (int q = 0; q < ctx->prm.n_corr; ++q)
                if (near(first[q], ctx->caps_built[q])) near_any = true;
            if (ctx->rounds > 1 && later > 0 && near(later, ctx->cap_later_built)) near_any = true;
        }
        if ((regrow_any || near_any) && !bad && !bad_dt) {
            // a capture needs no eager step here: the caps are known
            pisoc_status bs = build_graphs(e, e->one_graph);
            if (bs != PISOC_OK) {
                // the steps of this call stand; their records go out with the error
                if (h_info) std::copy(rec.begin(), rec.end(), h_info);
                return bs;
            }
        } else if (regrow_any) {
            drop_graphs(e);
        }
        if (bad_dt) {
            e->err = "time step undefined or non-positive in a member";
            if (h_info) std::copy(rec.begin(), rec.end(), h_info);
            return PISOC_ERR_INVALID;
        }
        if (bad) {
            e->err = "a member diverged (non-finite field, non-positive density or non-finite "
                     "dust density)";
            if (h_info) std::copy(rec.begin(), rec.end(), h_info);
            return PISOC_ERR_DIVERGED;
        }
    }
    if (h_info) std::copy(rec.begin(), rec.end(), h_info);
    return worst;
}

pisoc_status pisoc_ens_fields(pisoc_ens* e, int32_t member, uint32_t which, double* const* d_dst) {
    if (!e || member < 0 || member >= e->count || !d_dst) return PISOC_ERR_INVALID;
    const auto [c, i] = e->where[member];
    const pisoc_status st = member_fields(e->cls[c], i, which, d_dst);
    if (st != PISOC_OK) e->err = e->cls[c]->err;
    return st;
}

pisoc_status pisoc_ens_get_stats(pisoc_ens* e, pisoc_stats* h_out) {
    if (!e || !h_out) return PISOC_ERR_INVALID;
    for (size_t c = 0; c < e->cls.size(); ++c) {
        std::vector<pisoc_stats> s(e->cls[c]->batch);
        const pisoc_status st = all_stats(e->cls[c], s.data());
        if (st != PISOC_OK) {
            e->err = e->cls[c]->err;
            return st;
        }
        for (size_t i = 0; i < s.size(); ++i) h_out[e->members[c][i]] = s[i];
    }
    return PISOC_OK;
}

pisoc_status pisoc_ens_time(pisoc_ens* e, double* h_t) {
    if (!e || !h_t) return PISOC_ERR_INVALID;
    pisoc_status st = ens_sync(e);
    if (st != PISOC_OK) return st;
    for (int m = 0; m < e->count; ++m) {
        const auto [c, i] = e->where[m];
        h_t[m] = e->cls[c]->hst[i].t;
    }
    return PISOC_OK;
}

int64_t pisoc_ens_steps_done(const pisoc_ens* e) { return e ? e->steps : 0; }

int32_t pisoc_ens_num_classes(const pisoc_ens* e) { return e ? (int32_t)e->cls.size() : 0; }

pisoc_status pisoc_ens_class_info(const pisoc_ens* e, int32_t cls, pisoc_ens_class* h_out) {
    if (!e || !h_out || cls < 0 || cls >= (int32_t)e->cls.size()) return PISOC_ERR_INVALID;
    const pisoc_ctx* ctx = e->cls[cls];
    pisoc_ens_class o{};
    o.n = ctx->prm.n;
    o.members = ctx->batch;
    o.block_x = (int32_t)ctx->L.block.x;
    o.block_y = (int32_t)ctx->L.block.y;
    o.cells_z = ctx->L.cz;
    o.blocks = (int32_t)ctx->L.nblocks;
    o.rounds = ctx->rounds;
    o.cap_later = e->built ? ctx->cap_later_built : ctx->cap_later;
    for (int c = 0; c < PISOC_MAX_CORR; ++c) o.caps[c] = e->built ? ctx->caps_built[c] : ctx->caps[c];
    for (int c = 0; c < ctx->prm.n_corr; ++c)
        if (ctx->prm.guess != PISOC_GUESS_ZERO && (!audit_on(ctx) || ctx->audit.use[c]))
            o.guess_mask |= 1 << c;
    o.cg_cells_z = ctx->TS.nblocks ? ctx->TS.cz : 0;
    o.tiled_cells_z = ctx->TL.nblocks ? ctx->TL.cz : 0;
    *h_out = o;
    return PISOC_OK;
}

pisoc_status pisoc_ens_autotune(pisoc_ens* e, const char* cache_path, int32_t force) {
    if (!e) return PISOC_ERR_INVALID;
    if (e->steps < 1) {
        e->err = "autotune needs one completed step (the timed kernels run on its systems)";
        return PISOC_ERR_INVALID;
    }
    pisoc_status st = ens_sync(e);
    if (st != PISOC_OK) return st;
    for (pisoc_ctx* ctx : e->cls) {
        int bx = 0, cz = 0;
        st = tune_ctx(ctx, cache_path, force, &bx, &cz);
        if (st != PISOC_OK) {
            e->err = ctx->err;
            return st;
        }
    }
    drop_graphs(e);
    return ens_sync(e);
}

void pisoc_ens_destroy(pisoc_ens* e) {
    if (!e) return;
    for (pisoc_ctx* ctx : e->cls)
        if (ctx && ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graphs(e);
    for (hipEvent_t ev : e->fork_join) (void)hipEventDestroy(ev);
    for (pisoc_ctx* ctx : e->cls) free_ctx(ctx);
    for (hipStream_t s : e->streams) (void)hipStreamDestroy(s);
    delete e;
}

const char* pisoc_ens_last_error(const pisoc_ens* e) { return e ? e->err.c_str() : ""; }

// ---------------------------------------------------------------- Helmholtz
static Layout helm_layout(int32_t n) {
    Layout L{};
    const size_t N = (size_t)n * n * n;
    L.max_blocks = std::max({make_launch(n, 1).nblocks, make_tiled_launch(n, 1).nblocks,
                             make_spmv_launch(n, 1, 8).nblocks});
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.state = take(sizeof(DevState));
    L.partials = take(sizeof(double) * PS_COLUMNS * (size_t)L.max_blocks);
    L.r = take(8 * N);
    L.r2 = take(8 * N);
    L.diag = take(8 * N);
    L.pp0 = take(8 * N);
    L.pp1 = take(8 * N);
    L.pp2 = take(8 * N);
    L.q = take(8 * N);
    L.q2 = take(8 * N);
    L.total = off;
    return L;
}

static pisoc_params plain_params(int32_t n) {
    pisoc_params p{};
    p.n = n;
    p.gamma = 1.4;
    p.C = 1.0;
    return p;
}

size_t pisoc_helm_workspace_bytes(int32_t n) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N) return 0;
    return helm_layout(n).total;
}

pisoc_status pisoc_helm_apply(int32_t n, const double* d_psidt, const double* d_w,
                              const double* d_x, double* d_y, void* hip_stream) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_psidt || !d_w || !d_x || !d_y)
        return PISOC_ERR_INVALID;
    const pisoc_params p = plain_params(n);
    const Launch L = make_launch(n, 1);
    const Phys ph = make_phys(&p, L, 1);
    Ops<double>::helm_apply(L, reinterpret_cast<hipStream_t>(hip_stream), ph, d_psidt, d_w, d_x, d_y);
    return hipGetLastError() == hipSuccess ? PISOC_OK : PISOC_ERR_HIP;
}

// The solve of pisoc_helm_solve on the workspace ws (laid out as lay), with
// hst a host DevState the state is read back into.
// CG preconditioned by the Chebyshev polynomial on the system helm_start set
// up: per iteration k one residual/preconditioner and one direction/operator
// launch, in batches of 16 iterations with a host wait after each until the
// solve has stopped (at the tolerance or at maxit).
static pisoc_status run_cheb(pisoc_ctx* ctx, const double* psidt, const double* w,
                             const double* diag, double* const r[2], double* const p[2], double* z,
                             double* q, double* x, int maxit) {
    using O = Ops<double>;
    const Launch& L = ctx->L;
    const unsigned nb = L.nblocks;
    hipStream_t s = ctx->stream;
    double* theta = ctx->part(PS_CG + 2 * kChebSet);
    O::cheb_theta(L, s, ctx->ph, psidt, diag, theta);
    for (int k = 0;;) {
        const int kend = std::min(k + 15, maxit);
        for (int kk = k; kk <= kend; ++kk) {
            double* cur = ctx->part(PS_CG + kChebSet * (kk & 1));
            double* prev = ctx->part(PS_CG + kChebSet * ((kk + 1) & 1));
            double* rin = r[kk == 0 ? 0 : (kk - 1) & 1];
            double* pin = p[(kk + 1) & 1];
            O::cheb_res(L, ctx->TL, s, ctx->ph, ctx->st, kk, rin, r[kk & 1], q, pin, diag, w, x, z,
                        theta, nb, prev, cur);
            O::cheb_dir(L, ctx->TL, s, ctx->ph, ctx->st, kk, z, pin, p[kk & 1], q, diag, w,
                        ctx->part(PS_U), nb, prev, cur, maxit);
        }
        pisoc_status st = sync_state(ctx);
        if (st != PISOC_OK) return st;
        if (ctx->hst->pcg.it_stop != kIterInf) return PISOC_OK;
        k = kend + 1;
    }
}

static pisoc_status helm_solve_on(int32_t n, const double* d_psidt, const double* d_w,
                                  const double* d_b, double* d_x, double tol, int32_t maxit,
                                  char* ws, const Layout& lay, DevState* hst, hipStream_t stream,
                                  int32_t* iters, double* relres,
                                  int32_t precond = PISOC_PRECOND_JACOBI) {
    pisoc_ctx ctx{};
    ctx.prm = plain_params(n);
    ctx.prm.p_maxit = maxit;
    ctx.batch = 1;
    ctx.stream = stream;
    ctx.ws = ws;
    ctx.lay = lay;
    ctx.L = make_launch(n, 1);
    ctx.TL = make_tiled_launch(n, 1);
    ctx.TS = make_spmv_launch(n, 1, sizeof(double));
    ctx.ph = make_phys(&ctx.prm, ctx.L, 1);
    ctx.es = sizeof(double);
    ctx.st = reinterpret_cast<DevState*>(ctx.ws + lay.state);
    ctx.partials = reinterpret_cast<double*>(ctx.ws + lay.partials);
    ctx.hst = hst;
    DevState init{};
    init.pcg.tol2 = tol * tol;
    init.pcg.tol_final = tol * tol;
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
        CgVecs<double> v;
        v.r[0] = r;
        v.r[1] = ctx.f<double>(lay.r2);
        v.p[0] = ctx.f<double>(lay.pp0);
        v.p[1] = ctx.f<double>(lay.pp1);
        v.p[2] = ctx.f<double>(lay.pp2);
        v.q[0] = ctx.f<double>(lay.q);
        v.q[1] = ctx.f<double>(lay.q2);
        v.x = d_x;
        v.diag = dg;
        v.w = const_cast<double*>(d_w);
        if (precond == PISOC_PRECOND_CHEB) {
            double* const rr[2] = {v.r[0], v.r[1]};
            double* const pp[2] = {v.p[0], v.p[1]};
            st = run_cheb(&ctx, d_psidt, d_w, dg, rr, pp, v.p[2], v.q[0], d_x, maxit);
        } else {
            st = run_pcg<double>(&ctx, v, true, 16, true, nullptr, false, ctx.L.nblocks);
        }
        if (st == PISOC_OK) {
            const PcgState& g = ctx.hst->pcg;
            if (iters) *iters = g.iters;
            if (relres) *relres = g.bb > 0.0 ? std::sqrt(g.rr / g.bb) : 0.0;
            if (!g.converged) st = PISOC_WARN_NOT_CONVERGED;
        }
    }
    // the host copies of the state are the caller's; the context must not free them
    ctx.hst = nullptr;
    return st;
}

pisoc_status pisoc_helm_solve(int32_t n, const double* d_psidt, const double* d_w,
                              const double* d_b, double* d_x, double tol, int32_t maxit,
                              void* d_workspace, size_t ws_bytes, void* hip_stream,
                              int32_t* iters, double* relres) {
    return pisoc_helm_solve_precond(n, d_psidt, d_w, d_b, d_x, tol, maxit, PISOC_PRECOND_JACOBI,
                                    d_workspace, ws_bytes, hip_stream, iters, relres);
}

pisoc_status pisoc_helm_solve_precond(int32_t n, const double* d_psidt, const double* d_w,
                                      const double* d_b, double* d_x, double tol, int32_t maxit,
                                      int32_t precond, void* d_workspace, size_t ws_bytes,
                                      void* hip_stream, int32_t* iters, double* relres) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_psidt || !d_w || !d_b || !d_x ||
        !(tol > 0.0) || !(tol < 1.0) || maxit < 1 ||
        (precond != PISOC_PRECOND_JACOBI && precond != PISOC_PRECOND_CHEB))
        return PISOC_ERR_INVALID;
    const Layout lay = helm_layout(n);
    if (!d_workspace || ws_bytes < lay.total ||
        (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return PISOC_ERR_WORKSPACE;
    DevState* hst = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&hst), sizeof(DevState), hipHostMallocDefault) !=
        hipSuccess)
        return PISOC_ERR_HIP;
    const pisoc_status st =
        helm_solve_on(n, d_psidt, d_w, d_b, d_x, tol, maxit, reinterpret_cast<char*>(d_workspace),
                      lay, hst, reinterpret_cast<hipStream_t>(hip_stream), iters, relres, precond);
    (void)hipHostFree(hst);
    return st;
}

}  // extern "C"

// ------------------------------------------- pressure solve without allocation
// The scratch of pisoc_helm_solve_noalloc: the workspace pisoc_helm_solve takes
// from its caller (solver state, reduction partials, the CG vectors), here
// a file-scope device array of which every GPU the library runs on holds its
// own copy until the process ends.  In host code `scratch` only names the
// symbol: its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per device and kept in g_scratch_ptr.
static __device__ __align__(256) char scratch[PISOC_HELM_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mtx;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch`.
pisoc_status scratch_on_current_device(char** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PISOC_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PISOC_ERR_HIP;
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return PISOC_OK;
}

}  // namespace

extern "C" {

pisoc_status pisoc_helm_solve_noalloc(int32_t n, const double* d_psidt, const double* d_w,
                                      const double* d_b, double* d_x, double tol, int32_t maxit,
                                      void* hip_stream, int32_t* iters, double* relres) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_psidt || !d_w || !d_b || !d_x ||
        !(tol > 0.0) || !(tol < 1.0) || maxit < 1)
        return PISOC_ERR_INVALID;
    const Layout lay = helm_layout(n);
    if (n > PISOC_HELM_NOALLOC_MAX_N || lay.total > sizeof(scratch)) return PISOC_ERR_WORKSPACE;
    char* ws = nullptr;
    const pisoc_status sp = scratch_on_current_device(&ws);
    if (sp != PISOC_OK) return sp;
    // every scratch value is written before it is read (the state by the copy
    // in helm_solve_on, the partials and CG vectors by the kernels that
    // produce them), so nothing has to be cleared between calls; the state is
    // read back into pageable host memory, no pinned buffer is allocated
    DevState hst{};
    return helm_solve_on(n, d_psidt, d_w, d_b, d_x, tol, maxit, ws, lay, &hst,
                         reinterpret_cast<hipStream_t>(hip_stream), iters, relres);
}

pisoc_status pisoc_net_inputs(int32_t n, const double* d_b, const double* d_diag,
                              const double* d_p0, const double* d_psol, float* d_x, float* d_t,
                              double* h_scales, void* d_workspace, size_t ws_bytes,
                              void* hip_stream) {
    if (n < PISOC_MIN_N || n > PISOC_MAX_N || !d_b || !d_diag || !d_p0 || !d_x ||
        (d_t && !d_psol))
        return PISOC_ERR_INVALID;
    const Layout lay = helm_layout(n);
    if (!d_workspace || ws_bytes < lay.total ||
        (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
        return PISOC_ERR_WORKSPACE;
    const pisoc_params p = plain_params(n);
    const Launch L = make_launch(n, 1);
    const Phys ph = make_phys(&p, L, 1);
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
