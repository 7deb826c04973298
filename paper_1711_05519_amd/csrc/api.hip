// C ABI of librpca (include/rpca.h): argument validation, workspace layout and
// the stream-ordered orchestration of the kernels in stream.hip, stream_mx.hip,
// panel.hip, relax.hip and mlp.hip.
//
// One iteration of the loop ("body") is three launches on the caller's stream
// for FP32 D, four for FP64:
//   stream (one pass over D) -> gather (with the 2r x 2r step for FP32)
//   [-> complement (FP64)] -> update.
// The host keeps one body queued ahead of the GPU and reads the stopping
// decision from the completion record that each body's update kernel writes
// into mapped host memory, one body late; bodies queued past the stop become
// no-ops on the device (Ctrl gating), so the GPU never waits for the host.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rpca.h"
#include "launch.hpp"

using namespace rpca;

namespace {

thread_local int g_last_hip_error = 0;

constexpr int DEFAULT_INIT_MAX_PASSES = 40;
// BF16-product bodies while err_k >= mixed_err; the default 0 keeps them to
// the end (their rounding error scales with err_k)
constexpr double DEFAULT_MIXED_ERR = 0.0;
constexpr int MAX_DEVICES = 64;

#define HIP_TRY(expr)                                    \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) {                          \
            g_last_hip_error = (int)e_;                  \
            return RPCA_EHIP;                            \
        }                                                \
    } while (0)

#define RPCA_TRY(expr)              \
    do {                            \
        int s_ = (expr);            \
        if (s_ < 0) return s_;      \
    } while (0)

// Status slots in mapped, coherent host memory, one per call in flight on a
// device that runs a queue of bodies (rpca_init, rpca_solve).
constexpr int STATUS_SLOTS = 32;

constexpr int BATCH_BUFS = 4;
struct BatchBuf {
    std::mutex mutex;
    void* host = nullptr;
    void* dev = nullptr;
    size_t bytes = 0;
};

struct DeviceInfo {
    bool checked = false;
    bool ok = false;
    int id = 0;
    int cus = 256;
    HostStatus* status_host = nullptr;   // STATUS_SLOTS slots, allocated by the first call that needs one
    HostStatus* status_dev = nullptr;
    uint32_t slots_used = 0;             // bit i: slot i belongs to a call (g_dev_mutex)
    void* scratch = nullptr;             // this device's copy of `scratch` (rpca_step_noalloc)
    // mapped host buffers of rpca_solve_batch, grown on demand and kept; a
    // batched call holds one (its mutex) while it runs, so up to BATCH_BUFS
    // batched calls (from different host threads, on different streams) run
    // on a device at once
    BatchBuf batch[BATCH_BUFS];
};
std::mutex g_dev_mutex;
DeviceInfo g_dev[MAX_DEVICES];

// Device check only: properties of the current device, no allocation.
int device_info(DeviceInfo** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return RPCA_ENODEV;
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    DeviceInfo& d = g_dev[dev];
    if (!d.checked) {
        hipDeviceProp_t prop;
        HIP_TRY(hipGetDeviceProperties(&prop, dev));
        d.checked = true;
        d.id = dev;
        d.ok = std::string(prop.gcnArchName).find("gfx950") != std::string::npos;
        d.cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    }
    if (!d.ok) return RPCA_ENODEV;
    *out = &d;
    return RPCA_OK;
}

// The device's status slots in mapped, coherent host memory (g_dev_mutex held).
bool status_slots_locked(DeviceInfo* d) {
    if (d->status_host) return true;
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(HostStatus) * STATUS_SLOTS, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return false;
    memset(h, 0, sizeof(HostStatus) * STATUS_SLOTS);
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, h, 0) != hipSuccess) {
        (void)hipHostFree(h);
        return false;
    }
    d->status_host = static_cast<HostStatus*>(h);
    d->status_dev = static_cast<HostStatus*>(dp);
    return true;
}

// A status slot held for the duration of one call.
class StatusSlot {
public:
    explicit StatusSlot(DeviceInfo* d) : d_(d) {
        std::lock_guard<std::mutex> lock(g_dev_mutex);
        if (!status_slots_locked(d_)) return;
        for (int i = 0; i < STATUS_SLOTS; ++i) {
            if (!(d_->slots_used & (1u << i))) {
                d_->slots_used |= 1u << i;
                idx_ = i;
                memset(d_->status_host + i, 0, sizeof(HostStatus));
                break;
            }
        }
    }
    ~StatusSlot() {
        if (idx_ < 0) return;
        std::lock_guard<std::mutex> lock(g_dev_mutex);
        d_->slots_used &= ~(1u << idx_);
    }
    StatusSlot(const StatusSlot&) = delete;
    StatusSlot& operator=(const StatusSlot&) = delete;
    bool ok() const { return idx_ >= 0; }
    HostStatus* host() const { return d_->status_host + idx_; }
    HostStatus* dev() const { return d_->status_dev + idx_; }

private:
    DeviceInfo* d_;
    int idx_ = -1;
};

bool is_fin(double x) { return isfinite(x) != 0; }

#define RPCA_TAKE_SLOT(slot, c)                                       \
    StatusSlot slot((c).dev);                                         \
    if (!slot.ok()) {                                                 \
        g_last_hip_error = (int)hipErrorOutOfMemory;                  \
        return RPCA_EHIP;                                             \
    }                                                                 \
    (c).st_host = slot.host();                                        \
    (c).st_dev = slot.dev()

// ---- measurement: events around every streaming pass ---------------------------
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;                        // free events
    struct Rec {
        hipEvent_t e0, e1;
        int kind;
        int32_t body;   // id of the queued body the record belongs to (0: none)
    };
    std::vector<Rec> pending;
    double ms[RPCA_PROF_KINDS] = {0.0, 0.0, 0.0, 0.0};
    int64_t launches[RPCA_PROF_KINDS] = {0, 0, 0, 0};
};
Profiler g_prof;

hipEvent_t prof_event() {
    if (!g_prof.pool.empty()) {
        hipEvent_t e = g_prof.pool.back();
        g_prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int prof_collect_locked() {
    for (auto& pr : g_prof.pending) {
        HIP_TRY(hipEventSynchronize(pr.e1));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, pr.e0, pr.e1));
        g_prof.ms[pr.kind] += t;
        g_prof.launches[pr.kind] += 1;
        g_prof.pool.push_back(pr.e0);
        g_prof.pool.push_back(pr.e1);
    }
    g_prof.pending.clear();
    return RPCA_OK;
}

// Launch of the streaming pass (mx: products on the matrix cores in BF16),
// bracketed by events when profiling is on.
// events = false: never (rpca_step_noalloc, which creates no runtime objects).
int stream_launch(const StreamArgs& a, int K, int dtype, bool rebuild, bool mx, hipStream_t s, bool events = true,
                  int32_t body_id = 0) {
    if (!events) {
        if (mx) HIP_TRY(launch_stream_mx(a, K, rebuild, s));
        else HIP_TRY(launch_stream(a, K, dtype, rebuild, s));
        return RPCA_OK;
    }
    std::lock_guard<std::mutex> lock(g_prof.mu);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_prof.on) {
        if (g_prof.pending.size() >= 4096) RPCA_TRY(prof_collect_locked());
        e0 = prof_event();
        e1 = prof_event();
        if (!e0 || !e1) return RPCA_EHIP;
        HIP_TRY(hipEventRecord(e0, s));
    }
    if (mx) HIP_TRY(launch_stream_mx(a, K, rebuild, s));
    else HIP_TRY(launch_stream(a, K, dtype, rebuild, s));
    if (g_prof.on) {
        HIP_TRY(hipEventRecord(e1, s));
        g_prof.pending.push_back({e0, e1, mx ? 1 : (rebuild ? 0 : 2), body_id});
    }
    return RPCA_OK;
}

// Event before a loop body (profiling on): the pair is closed by prof_body_end.
int prof_body_begin(hipStream_t s, hipEvent_t* e0) {
    std::lock_guard<std::mutex> lock(g_prof.mu);
    *e0 = nullptr;
    if (!g_prof.on) return RPCA_OK;
    if (g_prof.pending.size() >= 4096) RPCA_TRY(prof_collect_locked());
    *e0 = prof_event();
    if (!*e0) return RPCA_EHIP;
    HIP_TRY(hipEventRecord(*e0, s));
    return RPCA_OK;
}
int prof_body_end(hipStream_t s, hipEvent_t e0, int32_t body_id) {
    if (!e0) return RPCA_OK;
    std::lock_guard<std::mutex> lock(g_prof.mu);
    hipEvent_t e1 = prof_event();
    if (!e1) return RPCA_EHIP;
    HIP_TRY(hipEventRecord(e1, s));
    g_prof.pending.push_back({e0, e1, 3, body_id});
    return RPCA_OK;
}

// The last queued body of a loop ran past the stop and did no work: drop its
// records (its pass and, for a loop body, the body itself).
void prof_drop_last() {
    std::lock_guard<std::mutex> lock(g_prof.mu);
    if (!g_prof.on || g_prof.pending.empty()) return;
    const int32_t body = g_prof.pending.back().body;
    do {
        auto pr = g_prof.pending.back();
        g_prof.pending.pop_back();
        (void)hipEventSynchronize(pr.e1);
        g_prof.pool.push_back(pr.e0);
        g_prof.pool.push_back(pr.e1);
    } while (body != 0 && !g_prof.pending.empty() && g_prof.pending.back().body == body);
}

int init_block_of(const rpca_params* p) {
    if (p->init_block > 0) return p->init_block;
    int q = p->r + 1;   // at m = n = 10^4, r = 5: 5 passes of width 6; the fastest width measured
    if (q > KMAX) q = KMAX;
    const int64_t lim = (p->m < p->n ? p->m : p->n) / 2;
    if (q > lim) q = (int)lim;
    return q < p->r ? p->r : q;
}

int validate(const rpca_params* p) {
    if (!p) return RPCA_EINVAL;
    if (p->m < 1 || p->n < 1 || p->m > (int64_t)INT32_MAX / 2 || p->n > (int64_t)INT32_MAX / 2) return RPCA_EINVAL;
    if (p->ldd < p->n) return RPCA_EINVAL;
    if (p->r < 1 || p->r > KMAX || 2 * (int64_t)p->r > (p->m < p->n ? p->m : p->n)) return RPCA_EINVAL;
    if (p->dtype != RPCA_F64 && p->dtype != RPCA_F32) return RPCA_EINVAL;
    if (!is_fin(p->beta) || !(p->beta > 0) || !is_fin(p->beta_init) || !(p->beta_init > 0)) return RPCA_EINVAL;
    if (!is_fin(p->gamma) || p->gamma < 0 || p->gamma >= 1) return RPCA_EINVAL;
    if (!is_fin(p->tol) || !(p->tol > 0)) return RPCA_EINVAL;
    if (!(p->flags & RPCA_FLAG_NO_TRIM) && (!is_fin(p->mu) || !(p->mu > 0))) return RPCA_EINVAL;
    if (p->max_iter < 0 || p->init_max_passes < 0) return RPCA_EINVAL;
    if (p->flags & ~(RPCA_FLAG_NO_TRIM | RPCA_FLAG_MIXED | RPCA_FLAG_TRAINING | RPCA_FLAG_LEARNED)) return RPCA_EINVAL;
    if ((p->flags & RPCA_FLAG_LEARNED) && !p->zeta_mlp) return RPCA_EINVAL;
    if ((p->flags & RPCA_FLAG_TRAINING) && p->r > RX_KMAX) return RPCA_EINVAL;
    if ((p->flags & RPCA_FLAG_MIXED) && p->dtype != RPCA_F32) return RPCA_EINVAL;
    if (!(p->mixed_err == p->mixed_err) || isinf(p->mixed_err)) return RPCA_EINVAL;
    if (p->init_block != 0) {
        if (p->init_block < p->r || p->init_block > KMAX ||
            2 * (int64_t)p->init_block > (p->m < p->n ? p->m : p->n))
            return RPCA_EINVAL;
    }
    return RPCA_OK;
}

// Workspace layout: every region 256-byte aligned.
struct Layout {
    int K_main, K_init, KW;
    int n_ct, n_rt_max, gU, gV;
    size_t acc;                       // bytes of a partial (4 for FP32, 8 for FP64)
    size_t elt;                       // bytes of an element of D
    size_t off_ctrl, off_small, off_hist, off_P1, off_P2, off_resid, off_gpart;
    size_t off_Y1, off_Y2, off_W1, off_W2, off_Ap, off_Bp, off_Unew, off_Vnew;
    size_t off_Uf, off_Vf, off_AL, off_BL;
    // relaxed iteration (RPCA_FLAG_TRAINING)
    int rx_nct, rx_nrt, rx_TM;
    size_t off_R1, off_R2, off_Rres, off_RY1, off_RY2, off_gpR, off_gram, off_gram2, off_coef, off_rres;
    size_t off_adj;   // reverse mode of unrolled relaxed iterations
    size_t total;
};

// The streaming pass runs one tile per resident workgroup (a single round, no
// tail): the row tiling follows the kernel's occupancy on the device. The
// workspace is sized for the largest tiling any device can ask for.
constexpr int STREAM_MAX_SLOTS = 2048;   // 256 CUs x 8 workgroups of 256 threads
constexpr int STREAM_MIN_TM = 64;

int n_rt_for(int m, int n_ct, int slots) {
    int n_rt = slots / n_ct;
    if (n_rt < 1) n_rt = 1;
    const int cap = (m + STREAM_MIN_TM - 1) / STREAM_MIN_TM;
    return n_rt < cap ? n_rt : cap;
}

Layout make_layout(const rpca_params* p) {
    Layout L;
    L.K_main = p->r;
    L.K_init = init_block_of(p);
    L.KW = L.K_init > L.K_main ? L.K_init : L.K_main;
    L.elt = p->dtype == RPCA_F32 ? 4 : 8;
    L.acc = L.elt;
    const int m = (int)p->m, n = (int)p->n;
    L.n_ct = (n + STREAM_TN - 1) / STREAM_TN;
    L.n_rt_max = n_rt_for(m, L.n_ct, STREAM_MAX_SLOTS);
    L.gU = (m + PANEL_THREADS - 1) / PANEL_THREADS;
    L.gV = (n + PANEL_THREADS - 1) / PANEL_THREADS;
    const int rpb = gather_threads_for(m, n) / GATHER_SPLIT;
    const int g_gather = (m + rpb - 1) / rpb + (n + rpb - 1) / rpb;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    L.off_ctrl = take(sizeof(Ctrl));
    L.off_small = take(sizeof(Small));
    L.off_hist = take(2 * sizeof(double) * (size_t)(p->max_iter + 1));
    L.off_P1 = take((size_t)L.n_ct * m * L.KW * L.acc);
    L.off_P2 = take((size_t)L.n_rt_max * n * L.KW * L.acc);
    // per-tile residual sums, then (init passes) per-tile max |D_ij|
    L.off_resid = take(2 * sizeof(double) * (size_t)L.n_ct * L.n_rt_max);
    L.off_gpart = take(sizeof(double) * (size_t)(g_gather > L.gU + L.gV ? g_gather : L.gU + L.gV) * GPART_STRIDE);
    const size_t pm = sizeof(double) * (size_t)m * L.KW, pn = sizeof(double) * (size_t)n * L.KW;
    L.off_Y1 = take(pm); L.off_Y2 = take(pn);
    L.off_W1 = take(pm); L.off_W2 = take(pn);
    L.off_Ap = take(pm); L.off_Bp = take(pn);
    L.off_Unew = take(pm); L.off_Vnew = take(pn);
    const size_t tm = L.elt * (size_t)m * L.KW, tn = L.elt * (size_t)n * L.KW;
    L.off_Uf = take(tm); L.off_Vf = take(tn);
    L.off_AL = take(tm); L.off_BL = take(tn);
    L.rx_nct = L.rx_nrt = L.rx_TM = 0;
    L.off_R1 = L.off_R2 = L.off_Rres = L.off_RY1 = L.off_RY2 = L.off_gpR = L.off_gram = L.off_gram2 = 0;
    L.off_coef = L.off_rres = L.off_adj = 0;
    if (p->flags & RPCA_FLAG_TRAINING) {
        const int K2 = 2 * p->r;
        L.rx_nct = (n + RX_THREADS - 1) / RX_THREADS;
        int nrt = (m + 63) / 64;
        if (nrt > RX_MAX_RT) nrt = RX_MAX_RT;
        L.rx_TM = (m + nrt - 1) / nrt;
        L.rx_nrt = (m + L.rx_TM - 1) / L.rx_TM;
        const int gp = (m + 255) / 256 + (n + 255) / 256;
        L.off_R1 = take(sizeof(double) * (size_t)L.rx_nct * m * K2);
        L.off_R2 = take(sizeof(double) * (size_t)L.rx_nrt * n * K2);
        L.off_Rres = take(sizeof(double) * (size_t)L.rx_nct * L.rx_nrt);
        L.off_RY1 = take(sizeof(double) * (size_t)m * K2);
        L.off_RY2 = take(sizeof(double) * (size_t)n * K2);
        L.off_gpR = take(sizeof(double) * (size_t)gp * RX_WMAX * RX_WMAX);
        L.off_gram = take(sizeof(double) * 2 * RX_WMAX * RX_WMAX);
        L.off_gram2 = take(sizeof(double) * 2 * RX_WMAX * RX_WMAX);
        L.off_coef = take(sizeof(double) * 6 * KMAX * KMAX);
        L.off_rres = take(sizeof(RelaxResult));
        L.off_adj = take(adjoint_ws_bytes(m, n, p->r, L.rx_nct, L.rx_nrt));
    }
    L.total = off;
    return L;
}

// Everything one call needs: layout plus typed pointers into the workspace.
struct Ctx {
    const rpca_params* p;
    Layout L;
    char* ws;
    hipStream_t s;
    DeviceInfo* dev;
    int dtype;
    bool mixed;          // RPCA_FLAG_MIXED: BF16-product bodies while err_k >= mixed_err
    double mixed_err;
    HostStatus* st_host = nullptr;   // the call's status slot (queues of bodies only)
    HostStatus* st_dev = nullptr;
    bool events = true;              // false: no profiler events (rpca_step_noalloc)
    int32_t batch = 1;               // instances per launch (rpca_solve_batch); all pointers are instance 0's
    int64_t slab = 0;                // bytes between the instances
    Ctrl* ctrl() const { return reinterpret_cast<Ctrl*>(ws + L.off_ctrl); }
    Small* small() const { return reinterpret_cast<Small*>(ws + L.off_small); }
    double* err_hist() const { return reinterpret_cast<double*>(ws + L.off_hist); }
    double* zeta_hist() const { return err_hist() + (p->max_iter + 1); }
    template <typename X> X* at(size_t off) const { return reinterpret_cast<X*>(ws + off); }
};

int make_ctx(const rpca_params* p, void* ws, size_t ws_bytes, void* stream, Ctx* c) {
    RPCA_TRY(validate(p));
    DeviceInfo* dev = nullptr;
    RPCA_TRY(device_info(&dev));
    c->p = p;
    c->L = make_layout(p);
    if (!ws || ((uintptr_t)ws & 255u) != 0 || ws_bytes < c->L.total) return RPCA_EWORKSPACE;
    c->ws = static_cast<char*>(ws);
    c->s = static_cast<hipStream_t>(stream);
    c->dev = dev;
    c->dtype = p->dtype;
    c->mixed = (p->flags & RPCA_FLAG_MIXED) != 0;
    c->mixed_err = p->mixed_err > 0 ? p->mixed_err : DEFAULT_MIXED_ERR;
    return RPCA_OK;
}

Ctrl base_ctrl(const Ctx& c, int stage, double zeta, int k, double normD2, int want_stop,
               const rpca_params* own = nullptr) {
    const rpca_params* p = own ? own : c.p;
    Ctrl t;
    memset(&t, 0, sizeof(t));
    t.stage = stage;
    t.k = k;
    t.max_iter = p->max_iter;
    t.r = p->r;
    t.p = c.L.K_init;
    t.keep = p->r;
    t.init_max_passes = p->init_max_passes > 0 ? p->init_max_passes : DEFAULT_INIT_MAX_PASSES;
    t.trim = (p->flags & RPCA_FLAG_NO_TRIM) ? 0 : 1;
    t.want_stop = want_stop;
    t.active = 1;
    t.zeta = zeta;
    t.normD2 = normD2;
    t.beta = p->beta;
    t.beta_init = p->beta_init;
    t.gamma = p->gamma;
    t.mu = p->mu;
    t.tol = p->tol;
    t.res_prev = 1e300;
    t.tol_res_a = p->dtype == RPCA_F64 ? 1e-9 : 3e-6;
    t.tol_res_b = p->dtype == RPCA_F64 ? 1e-13 : 3e-6;
    // rounding level of the streamed products relative to sigma_1
    t.sigma_dead = p->dtype == RPCA_F64 ? 1e-12 : 1e-5;
    t.single = p->dtype == RPCA_F32 ? 1 : 0;
    t.learned_on = ((p->flags & RPCA_FLAG_LEARNED) && p->zeta_mlp) ? 1 : 0;
    t.err_prev = 1e300;
    return t;
}

// Row tiling of a streaming pass with block width K: one round of tiles.
struct Geo {
    int TM, n_rt;
};
Geo geo_for(const Ctx& c, int K, bool rebuild, bool mx = false) {
    const int m = (int)c.p->m;
    const int occ = mx ? stream_mx_occupancy(K, rebuild) : stream_occupancy(K, c.dtype, rebuild);
    const int slots = occ * c.dev->cus;
    int n_rt;
    if (c.batch > 1) {
        // a batch: at least two rounds of workgroups over all its instances, so
        // that the last, partly filled round is a small part of the pass
        const int64_t per = (int64_t)c.L.n_ct * c.batch;
        const int want = (int)((2 * (int64_t)slots + per - 1) / per);
        n_rt = n_rt_for(m, c.L.n_ct, want * c.L.n_ct);
        if (n_rt > c.L.n_rt_max) n_rt = c.L.n_rt_max;
    } else {
        n_rt = n_rt_for(m, c.L.n_ct, slots < STREAM_MAX_SLOTS ? slots : STREAM_MAX_SLOTS);
    }
    int TM = (m + n_rt - 1) / n_rt;
    TM = (TM + STREAM_WAVES - 1) / STREAM_WAVES * STREAM_WAVES;
    Geo g;
    g.TM = TM;
    g.n_rt = (m + TM - 1) / TM;
    return g;
}

StreamArgs stream_args(const Ctx& c, const void* D, int body, const Geo& g) {
    StreamArgs a;
    memset(&a, 0, sizeof(a));
    a.D = D;
    a.ldd = c.p->ldd;
    a.m = (int)c.p->m;
    a.n = (int)c.p->n;
    a.AL = c.ws + c.L.off_AL;
    a.BL = c.ws + c.L.off_BL;
    a.Uf = c.ws + c.L.off_Uf;
    a.Vf = c.ws + c.L.off_Vf;
    a.ctrl = c.ctrl();
    a.P1 = c.ws + c.L.off_P1;
    a.P2 = c.ws + c.L.off_P2;
    a.resid = c.at<double>(c.L.off_resid);
    a.TM = g.TM;
    a.n_ct = c.L.n_ct;
    a.n_rt = g.n_rt;
    const size_t row_bytes = (size_t)c.p->ldd * c.L.elt;
    a.vec_ok = (((uintptr_t)D & 15u) == 0 && (row_bytes & 15u) == 0 && (c.slab & 15) == 0) ? 1 : 0;
    a.body = body;
    a.batch = c.batch;
    a.slab = c.slab;
    a.post_gpart = c.at<double>(c.L.off_gpart);
    a.post_small = c.small();
    a.post_gU = c.L.gU;
    a.post_gV = c.L.gV;
    return a;
}

PanelArgs panel_args(const Ctx& c, const Geo& g = Geo{0, 1}) {
    PanelArgs a;
    memset(&a, 0, sizeof(a));
    a.m = (int)c.p->m;
    a.n = (int)c.p->n;
    a.gU = c.L.gU;
    a.gV = c.L.gV;
    a.ctrl = c.ctrl();
    a.small = c.small();
    a.gpart = c.at<double>(c.L.off_gpart);
    a.P1 = c.ws + c.L.off_P1;
    a.P2 = c.ws + c.L.off_P2;
    a.n_ct = c.L.n_ct;
    a.n_rt = g.n_rt;
    a.resid = c.at<double>(c.L.off_resid);
    a.n_tiles = c.L.n_ct * g.n_rt;
    a.Y1 = c.at<double>(c.L.off_Y1);
    a.Y2 = c.at<double>(c.L.off_Y2);
    a.W1 = c.at<double>(c.L.off_W1);
    a.W2 = c.at<double>(c.L.off_W2);
    a.Ap = c.at<double>(c.L.off_Ap);
    a.Bp = c.at<double>(c.L.off_Bp);
    a.Uf = c.ws + c.L.off_Uf;
    a.Vf = c.ws + c.L.off_Vf;
    a.AL = c.ws + c.L.off_AL;
    a.BL = c.ws + c.L.off_BL;
    a.host_status = c.st_dev;
    a.body_id = 0;
    a.body = BODY_ANY;
    a.mlp = (c.p->flags & RPCA_FLAG_LEARNED) ? c.p->zeta_mlp : nullptr;
    a.batch = c.batch;
    a.slab = c.slab;
    return a;
}

int setup(const Ctx& c, const Ctrl& t) {
    HIP_TRY(launch_setup(c.ctrl(), t, c.batch, c.slab, c.s));
    return RPCA_OK;
}

// One loop body. FP32: stream pass, gather (with the 2r x 2r step), update.
// FP64: stream pass, gather, complement (explicit W), update.
int enqueue_body(const Ctx& c, const void* D, int K, int body, double* state_U, double* state_V,
                 double* state_sigma, bool with_hist, bool mx = false, int32_t body_id = 0) {
    const bool rebuild = body != BODY_INIT;
    const bool fp32 = c.dtype == RPCA_F32;
    const Geo g = geo_for(c, K, rebuild, mx);
    StreamArgs sa = stream_args(c, D, body, g);
    hipEvent_t eb = nullptr;
    if (body == BODY_MAIN && c.events) RPCA_TRY(prof_body_begin(c.s, &eb));
    RPCA_TRY(stream_launch(sa, K, c.dtype, rebuild, mx, c.s, c.events, body_id));
    PanelArgs pa = panel_args(c, g);
    pa.body = body;
    pa.lcorr = rebuild ? 1 : 0;
    if (with_hist) {
        pa.err_hist = c.err_hist();
        pa.zeta_hist = c.zeta_hist();
        pa.hist_cap = c.p->max_iter + 1;
    }
    pa.mode = fp32 ? GATHER_WITH_SVD : GATHER_ONLY;
    HIP_TRY(launch_gather(pa, K, c.dtype, c.s));
    if (!fp32) HIP_TRY(launch_complement(pa, K, c.dtype, c.s));
    PanelArgs ua = pa;
    ua.mode = UPDATE_FROM_M;
    ua.body_id = body_id;
    ua.S2U = fp32 ? pa.Y1 : pa.W1;
    ua.S2V = fp32 ? pa.Y2 : pa.W2;
    if (body == BODY_INIT) {
        ua.Unew = c.at<double>(c.L.off_Unew);
        ua.Vnew = c.at<double>(c.L.off_Vnew);
    } else {
        ua.Unew = state_U;
        ua.Vnew = state_V;
        ua.sigma_dst = state_sigma;
    }
    HIP_TRY(launch_update(ua, K, c.dtype, c.s));
    RPCA_TRY(prof_body_end(c.s, eb, body_id));
    return RPCA_OK;
}

// Enter the loop from factors src (stride ld_src) with singular values
// src_sigma: rebuild factors, Trim and the bases of the next streaming pass.
int enqueue_enter(const Ctx& c, const double* srcU, const double* srcV, int64_t ld_src,
                  const double* src_sigma, double* dstU, double* dstV, double* dst_sigma) {
    const int K = c.p->r;
    PanelArgs ua = panel_args(c);
    ua.mode = UPDATE_ENTER;
    ua.srcU = srcU;
    ua.srcV = srcV;
    ua.ld_src = ld_src;
    ua.src_sigma = src_sigma;
    ua.Unew = dstU;
    ua.Vnew = dstV;
    ua.sigma_dst = dst_sigma;
    HIP_TRY(launch_update(ua, K, c.dtype, c.s));
    return RPCA_OK;
}

inline void cpu_relax() { __builtin_ia32_pause(); }

// Waits until the completion record of body `id` is in the call's status slot
// (written by the body's last kernel). A stream that drains without it, or
// reports an error, ends the wait with RPCA_EHIP.
int wait_record(const Ctx& c, int32_t id, BodyRecord* out) {
    const volatile BodyRecord* r = &c.st_host->body[id & (BODY_RING - 1)];
    auto last = std::chrono::steady_clock::now();
    for (uint32_t spin = 1; r->id != id; ++spin) {
        cpu_relax();
        if ((spin & 1023u) != 0) continue;
        const auto now = std::chrono::steady_clock::now();
        if (now - last < std::chrono::microseconds(500)) continue;
        last = now;
        const hipError_t e = hipStreamQuery(c.s);
        if (e == hipSuccess) {
            if (r->id == id) break;
            return RPCA_EHIP;   // the queue drained without the record
        }
        if (e != hipErrorNotReady) {
            g_last_hip_error = (int)e;
            return RPCA_EHIP;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    out->id = r->id;
    out->stage = r->stage;
    out->done = r->done;
    out->k = r->k;
    out->err = r->err;
    return RPCA_OK;
}

// Runs queued bodies until `finished(record, b)`, called once body b has
// completed (b = 0, 1, ...; body b has id b + 1); keeps one body queued ahead.
template <typename Enq, typename Fin>
int pipelined_loop(const Ctx& c, int max_bodies, Enq enqueue, Fin finished) {
    int rc = RPCA_OK;
    for (int b = 0; b < max_bodies; ++b) {
        rc = enqueue(b + 1);
        if (rc < 0) break;
        if (b >= 1) {
            BodyRecord rec;
            rc = wait_record(c, b, &rec);
            if (rc < 0) break;
            if (finished(rec, b - 1)) {
                prof_drop_last();   // body b was queued after the stop: a no-op
                break;
            }
        }
    }
    hipError_t e = hipStreamSynchronize(c.s);
    if (e != hipSuccess && rc >= 0) { g_last_hip_error = (int)e; rc = RPCA_EHIP; }
    return rc;
}

int read_ctrl(const Ctx& c, Ctrl* out) {
    HIP_TRY(hipMemcpyAsync(out, c.ctrl(), sizeof(Ctrl), hipMemcpyDeviceToHost, c.s));
    HIP_TRY(hipStreamSynchronize(c.s));
    return RPCA_OK;
}

// Algorithm 3 on the device; leaves the caller's state at L_0 and the
// workspace ready for the first loop body (bases of Trim(L_0), zeta_0).
int run_init(const Ctx& c, const void* D, rpca_state* st, Ctrl* ctrl_out) {
    const int P = c.L.K_init;
    Ctrl t = base_ctrl(c, STAGE_SIGMA_D, INFINITY, 0, 1.0, 0);
    RPCA_TRY(setup(c, t));
    PanelArgs sa = panel_args(c);
    sa.seed = c.p->seed;
    HIP_TRY(launch_start(sa, P, c.dtype, c.s));
    const int max_bodies = 2 * t.init_max_passes + 4;
    int rc = pipelined_loop(
        c, max_bodies,
        [&](int32_t id) { return enqueue_body(c, D, P, BODY_INIT, nullptr, nullptr, nullptr, false, false, id); },
        [&](const BodyRecord& r, int) { return r.stage >= STAGE_INIT_DONE; });
    RPCA_TRY(rc);
    Ctrl now;
    RPCA_TRY(read_ctrl(c, &now));
    if (now.nonfinite) return RPCA_EINVAL;               // ||D||_F = 0 or a non-finite entry
    if (now.stage < STAGE_INIT_DONE) return RPCA_EHIP;   // unreachable: the pass cap forces convergence
    // L_0: the leading r columns of the converged block
    RPCA_TRY(enqueue_enter(c, c.at<double>(c.L.off_Unew), c.at<double>(c.L.off_Vnew), P,
                           c.small()->sigma_new, st->U, st->V, st->sigma));
    *ctrl_out = now;
    return RPCA_OK;
}

// One streaming pass plus gather at the current factors and zeta (rank r):
// residual, err and products for this state.
int threshold_pass(const Ctx& c, const void* D, bool rebuild) {
    const int K = c.p->r;
    const Geo g = geo_for(c, K, rebuild);
    RPCA_TRY(stream_launch(stream_args(c, D, BODY_ANY, g), K, c.dtype, rebuild, false, c.s, c.events));
    PanelArgs pa = panel_args(c, g);
    pa.lcorr = rebuild ? 1 : 0;
    HIP_TRY(launch_gather(pa, K, c.dtype, c.s));
    return RPCA_OK;
}

void fill_state(rpca_state* st, const Ctrl& t) {
    st->zeta = t.zeta;
    st->err = t.err;
    st->k = t.k;
    st->sigma1_pt = t.sig1_pt;
    st->sigma_r1_pt = t.sigr1_pt;
    st->normD = sqrt(t.normD2);
    st->svd_sweeps = t.jacobi_sweeps;
}

int check_state(const rpca_state* st) {
    if (!st || !st->U || !st->V || !st->sigma) return RPCA_EINVAL;
    return RPCA_OK;
}

// Workspace of rpca_step_noalloc: a fixed array in device memory, one copy
// per GPU (the runtime provides it when the library's code is loaded on that
// device, and it stays until the process ends). Host code never passes the
// array's name to a kernel: it is a host-side stand-in for the symbol, not a
// device address. The device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and is kept in DeviceInfo.
static __device__ __align__(256) unsigned char scratch[RPCA_NOALLOC_WS_BYTES];

int noalloc_workspace(DeviceInfo* d, void** out) {
    std::lock_guard<std::mutex> lock(g_dev_mutex);
    if (!d->scratch) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr || ((uintptr_t)ptr & 255u) != 0) {
            g_last_hip_error = (int)(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return RPCA_EHIP;
        }
        d->scratch = ptr;
    }
    *out = d->scratch;
    return RPCA_OK;
}

}  // namespace

extern "C" {

int rpca_version(void) { return 101; }

int rpca_profile_enable(int on) {
    std::lock_guard<std::mutex> lock(g_prof.mu);
    if (!on) RPCA_TRY(prof_collect_locked());
    g_prof.on = on != 0;
    return RPCA_OK;
}

int rpca_profile_read(double* stream_ms, int64_t* stream_launches) {
    if (!stream_ms || !stream_launches) return RPCA_EINVAL;
    std::lock_guard<std::mutex> lock(g_prof.mu);
    RPCA_TRY(prof_collect_locked());
    for (int k = 0; k < RPCA_PROF_KINDS; ++k) {
        stream_ms[k] = g_prof.ms[k];
        stream_launches[k] = g_prof.launches[k];
        g_prof.ms[k] = 0.0;
        g_prof.launches[k] = 0;
    }
    return RPCA_OK;
}

int rpca_last_hip_error(void) { return g_last_hip_error; }

int rpca_read_probe(const void* data, int64_t bytes, float* sink, void* stream) {
    if (!data || !sink || bytes <= 0 || (bytes & 15) != 0 || ((uintptr_t)data & 15u) != 0) return RPCA_EINVAL;
    DeviceInfo* dev = nullptr;
    RPCA_TRY(device_info(&dev));
    int blocks = 8 * dev->cus;
    if (blocks > RPCA_PROBE_SINK) blocks = RPCA_PROBE_SINK;
    HIP_TRY(launch_read_probe(data, bytes, sink, blocks, static_cast<hipStream_t>(stream)));
    return RPCA_OK;
}

const char* rpca_strerror(int status) {
    switch (status) {
        case RPCA_OK: return "success";
        case RPCA_MAXITER: return "iteration cap reached before err < tol";
        case RPCA_EINVAL: return "invalid argument";
        case RPCA_EWORKSPACE: return "workspace missing, misaligned or too small";
        case RPCA_EHIP: return "HIP runtime error";
        case RPCA_ENODEV: return "current device is not a gfx950 GPU";
        case RPCA_EBREAKDOWN: return "non-finite residual inside the iteration (numerical breakdown)";
        default: return "unknown status";
    }
}

int rpca_workspace_size(const rpca_params* p, size_t* bytes) {
    RPCA_TRY(validate(p));
    if (!bytes) return RPCA_EINVAL;
    *bytes = make_layout(p).total;
    return RPCA_OK;
}

int rpca_init(const void* D, const rpca_params* p, rpca_state* st, void* ws, size_t ws_bytes, void* stream) {
    if (!D) return RPCA_EINVAL;
    RPCA_TRY(check_state(st));
    Ctx c;
    RPCA_TRY(make_ctx(p, ws, ws_bytes, stream, &c));
    RPCA_TAKE_SLOT(slot, c);
    Ctrl ic;
    RPCA_TRY(run_init(c, D, st, &ic));
    // err_0 from one threshold pass: S_0 = T_zeta_0(D - L_0)
    RPCA_TRY(threshold_pass(c, D, true));
    Ctrl t;
    RPCA_TRY(read_ctrl(c, &t));
    if (t.nonfinite) return RPCA_EBREAKDOWN;
    fill_state(st, t);
    st->init_passes = ic.total_passes;
    return RPCA_OK;
}

// RPCA_TRACE: unset or "0" off; "1" JSON lines on stderr; anything else is a
// file that the lines are appended to. One line per state k of a finished solve
// (err_k, zeta_k) and a summary line; written after the device work is done.
std::mutex g_trace_mutex;

void trace_solve(const char* call, int instance, int status, const Ctrl& fin, const double* err, const double* zeta,
                 int cnt, const rpca_params* p) {
    const char* where = getenv("RPCA_TRACE");
    if (!where || !*where || strcmp(where, "0") == 0) return;
    std::lock_guard<std::mutex> lock(g_trace_mutex);
    FILE* f = strcmp(where, "1") == 0 ? stderr : fopen(where, "a");
    if (!f) return;
    for (int k = 0; err && zeta && k < cnt; ++k)
        fprintf(f, "{\"call\": \"%s\", \"instance\": %d, \"k\": %d, \"err\": %.17g, \"zeta\": %.17g}\n", call,
                instance, k, err[k], zeta[k]);
    fprintf(f,
            "{\"call\": \"%s\", \"instance\": %d, \"status\": %d, \"iterations\": %d, \"init_passes\": %d, "
            "\"err\": %.17g, \"zeta\": %.17g, \"sigma1\": %.17g, \"sigma_r1\": %.17g, \"m\": %lld, \"n\": %lld, "
            "\"r\": %d, \"dtype\": \"%s\", \"flags\": %u}\n",
            call, instance, status, fin.k, fin.total_passes, fin.err, fin.zeta, fin.sig1_pt, fin.sigr1_pt,
            (long long)p->m, (long long)p->n, p->r, p->dtype == RPCA_F32 ? "f32" : "f64", p->flags);
    if (f != stderr) fclose(f);
}

bool trace_on() {
    const char* where = getenv("RPCA_TRACE");
    return where && *where && strcmp(where, "0") != 0;
}

// One solve (Algorithm 3, then Algorithm 1) as a queue of bodies that the host
// advances step by step, so that several solves can share one host thread.
// Bodies are queued one ahead of the host: initialisation bodies until a
// completed one reports the stage INIT_DONE (the body queued meanwhile is a
// no-op), then the entry update, the switch of the control block (both on the
// device) and loop bodies until the stopping rule fires. Body b has id b + 1;
// the host reads the completion record of body b - 1 (written by its last
// kernel into mapped host memory) after queueing body b, instead of queueing
// events, which would add a marker between the bodies.
// Mixed form: loop body k + 1 is queued once loop body k - 1 has completed, so
// it takes BF16 products while err_{k-1} >= mixed_err (bodies 0 and 1 always
// do); the first body with err below the level switches every later body to
// the FP32 pass. The decision reads err of a fixed body (its completion
// record), so it does not depend on timing.
class SolveJob {
public:
    int start(const void* D, const rpca_params* p, rpca_state* st, double* err_hist, double* zeta_hist,
              int32_t hist_cap, void* ws, size_t ws_bytes, void* stream) {
        if (!D || hist_cap < 0) return RPCA_EINVAL;
        RPCA_TRY(check_state(st));
        RPCA_TRY(make_ctx(p, ws, ws_bytes, stream, &c_));
        slot_.reset(new StatusSlot(c_.dev));
        if (!slot_->ok()) {
            g_last_hip_error = (int)hipErrorOutOfMemory;
            return RPCA_EHIP;
        }
        c_.st_host = slot_->host();
        c_.st_dev = slot_->dev();
        D_ = D;
        p_ = p;
        st_ = st;
        err_hist_ = err_hist;
        zeta_hist_ = zeta_hist;
        hist_cap_ = hist_cap;
        P_ = c_.L.K_init;
        const Ctrl t = base_ctrl(c_, STAGE_SIGMA_D, INFINITY, 0, 1.0, 0);
        RPCA_TRY(setup(c_, t));
        PanelArgs sa = panel_args(c_);
        sa.seed = p->seed;
        HIP_TRY(launch_start(sa, P_, c_.dtype, c_.s));
        max_bodies_ = 2 * t.init_max_passes + 4 + p->max_iter + 3;
        use_mx_ = c_.mixed;
        b_ = 0;
        return enqueue_current();
    }

    // Queues bodies while the records they depend on are there. Returns 1 once
    // the last body is queued, 0 if the record of body b - 1 is not there yet
    // (block = false), a negative status on failure.
    int step(bool block) {
        while (!queued_all_) {
            if (b_ >= 1) {
                BodyRecord hs;
                if (block) {
                    const int e = wait_record(c_, b_, &hs);
                    if (e < 0) return fail(e);
                } else if (!try_record(b_, &hs)) {
                    return 0;
                }
                const int e = on_record(hs);
                if (e < 0) return fail(e);
                if (stopped_) {
                    queued_all_ = true;
                    break;
                }
            }
            if (b_ + 1 >= max_bodies_) {
                queued_all_ = true;
                break;
            }
            ++b_;
            const int e = enqueue_current();
            if (e < 0) return fail(e);
        }
        return rc_ < 0 ? rc_ : 1;
    }

    bool queued_all() const { return queued_all_; }
    hipStream_t stream() const { return c_.s; }

    // After the last body: waits for the stream, then fills the state and the
    // histories. Returns rpca_solve's status.
    int finish() {
        // the last kernel copies the control block and the histories' leading
        // entries into the status slot: one synchronisation reads them all
        if (rc_ >= 0) {
            const hipError_t le =
                launch_publish(c_.ctrl(), c_.err_hist(), c_.zeta_hist(), p_->max_iter + 1, c_.st_dev, c_.s);
            if (le != hipSuccess) {
                g_last_hip_error = (int)le;
                rc_ = RPCA_EHIP;
            }
        }
        hipError_t e = hipStreamSynchronize(c_.s);
        if (e != hipSuccess && rc_ >= 0) {
            g_last_hip_error = (int)e;
            rc_ = RPCA_EHIP;
        }
        RPCA_TRY(rc_);
        const volatile HostStatus* hs = c_.st_host;
        std::atomic_thread_fence(std::memory_order_acquire);
        Ctrl fin;
        memcpy(&fin, const_cast<const Ctrl*>(&hs->fin), sizeof(Ctrl));
        if (fin.nonfinite == 1) return RPCA_EINVAL;       // ||D||_F = 0 or a non-finite entry of D
        if (fin.nonfinite) return RPCA_EBREAKDOWN;        // a non-finite residual inside the loop
        if (fin.stage != STAGE_MAIN) return RPCA_EHIP;   // unreachable: the pass cap forces convergence
        fill_state(st_, fin);
        st_->init_passes = fin.total_passes;
        const int n = fin.k + 1;
        const int cnt = n < hist_cap_ ? n : hist_cap_;
        if (cnt > 0 && cnt <= PUBLISH_HIST) {
            for (int i = 0; i < cnt; ++i) {
                if (err_hist_) err_hist_[i] = hs->hist[0][i];
                if (zeta_hist_) zeta_hist_[i] = hs->hist[1][i];
            }
        } else if (cnt > 0) {
            if (err_hist_)
                HIP_TRY(hipMemcpyAsync(err_hist_, c_.err_hist(), sizeof(double) * cnt, hipMemcpyDeviceToHost, c_.s));
            if (zeta_hist_)
                HIP_TRY(hipMemcpyAsync(zeta_hist_, c_.zeta_hist(), sizeof(double) * cnt, hipMemcpyDeviceToHost, c_.s));
            HIP_TRY(hipStreamSynchronize(c_.s));
        }
        const int status = fin.stopped_by_tol ? RPCA_OK : RPCA_MAXITER;
        if (trace_on()) {
            std::vector<double> eh((size_t)n), zh((size_t)n);
            HIP_TRY(hipMemcpyAsync(eh.data(), c_.err_hist(), sizeof(double) * n, hipMemcpyDeviceToHost, c_.s));
            HIP_TRY(hipMemcpyAsync(zh.data(), c_.zeta_hist(), sizeof(double) * n, hipMemcpyDeviceToHost, c_.s));
            HIP_TRY(hipStreamSynchronize(c_.s));
            trace_solve("rpca_solve", 0, status, fin, eh.data(), zh.data(), n, p_);
        }
        return status;
    }

private:
    int fail(int e) {
        rc_ = e;
        queued_all_ = true;
        return e;
    }

    int enqueue_current() {
        return in_loop_ ? enqueue_body(c_, D_, p_->r, BODY_MAIN, st_->U, st_->V, st_->sigma, true, use_mx_, b_ + 1)
                        : enqueue_body(c_, D_, P_, BODY_INIT, nullptr, nullptr, nullptr, false, false, b_ + 1);
    }

    bool try_record(int32_t id, BodyRecord* out) const {
        const volatile BodyRecord* r = &c_.st_host->body[id & (BODY_RING - 1)];
        if (r->id != id) return false;
        std::atomic_thread_fence(std::memory_order_acquire);
        out->id = r->id;
        out->stage = r->stage;
        out->done = r->done;
        out->k = r->k;
        out->err = r->err;
        return true;
    }

    // The record of body b - 1 (queued before body b).
    int on_record(const BodyRecord& hs) {
        if (!in_loop_) {
            if (hs.stage == STAGE_FAILED) {
                prof_drop_last();   // body b ran after the failed pass: a no-op
                stopped_ = true;
            } else if (hs.stage >= STAGE_INIT_DONE) {
                prof_drop_last();   // body b ran after the stage changed: a no-op
                // L_0: the leading r columns of the converged block; Trim and bases
                RPCA_TRY(enqueue_enter(c_, c_.at<double>(c_.L.off_Unew), c_.at<double>(c_.L.off_Vnew), P_,
                                       c_.small()->sigma_new, st_->U, st_->V, st_->sigma));
                HIP_TRY(launch_enter_loop(c_.ctrl(), 1, 0, c_.s));
                in_loop_ = true;
                loop_first_ = b_ + 1;
            }
        } else if (b_ - 1 >= loop_first_) {
            if (use_mx_ && hs.err < c_.mixed_err) use_mx_ = false;   // hs.err = err of loop body b - 1 - loop_first
            if (hs.done) {
                prof_drop_last();   // body b was queued after the stop: a no-op
                stopped_ = true;
            }
        }
        return RPCA_OK;
    }

    Ctx c_;
    std::unique_ptr<StatusSlot> slot_;
    const void* D_ = nullptr;
    const rpca_params* p_ = nullptr;
    rpca_state* st_ = nullptr;
    double* err_hist_ = nullptr;
    double* zeta_hist_ = nullptr;
    int32_t hist_cap_ = 0;
    int P_ = 0, max_bodies_ = 0, b_ = 0, loop_first_ = -1;
    bool in_loop_ = false, use_mx_ = false, stopped_ = false, queued_all_ = false;
    int rc_ = RPCA_OK;
};

int rpca_solve(const void* D, const rpca_params* p, rpca_state* st, double* err_hist, double* zeta_hist,
               int32_t hist_cap, void* ws, size_t ws_bytes, void* stream) {
    SolveJob job;
    const int e = job.start(D, p, st, err_hist, zeta_hist, hist_cap, ws, ws_bytes, stream);
    if (e < 0) {
        (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));   // nothing queued stays in flight
        return e;
    }
    (void)job.step(true);
    return job.finish();
}

int rpca_solve_many(int32_t count, const void* const* D, const rpca_params* const* p, rpca_state* const* st,
                    double* const* err_hist, double* const* zeta_hist, int32_t hist_cap, void* const* ws,
                    const size_t* ws_bytes, void* const* streams, int32_t n_streams, int32_t* status) {
    if (count < 0 || !status || (count > 0 && (!D || !p || !st || !ws || !ws_bytes || !streams)) ||
        n_streams < 1 || n_streams > RPCA_MANY_MAX_STREAMS || hist_cap < 0)
        return RPCA_EINVAL;
    for (int32_t i = 0; i < count; ++i) {
        status[i] = RPCA_EINVAL;
        if (!D[i] || !p[i] || !st[i]) return RPCA_EINVAL;
        RPCA_TRY(validate(p[i]));
        RPCA_TRY(check_state(st[i]));
    }
    // Up to n_streams solves in flight, instance i on streams[i % n_streams];
    // a new one starts once an earlier one has queued its last body and its
    // stream has drained.
    std::vector<std::unique_ptr<SolveJob>> live(n_streams);
    std::vector<int32_t> who(n_streams, -1);
    int32_t next = 0, done = 0;
    int first_err = RPCA_OK;
    auto t_idle = std::chrono::steady_clock::now();
    while (done < count) {
        bool moved = false;
        for (int32_t k = 0; k < n_streams; ++k) {
            if (!live[k] && next < count && next % n_streams == k) {
                const int32_t i = next++;
                live[k].reset(new SolveJob());
                who[k] = i;
                const int e = live[k]->start(D[i], p[i], st[i], err_hist ? err_hist[i] : nullptr,
                                             zeta_hist ? zeta_hist[i] : nullptr, hist_cap, ws[i], ws_bytes[i],
                                             streams[k]);
                if (e < 0) {
                    (void)hipStreamSynchronize(static_cast<hipStream_t>(streams[k]));
                    status[i] = e;
                    if (first_err == RPCA_OK) first_err = e;
                    live[k].reset();
                    ++done;
                }
                moved = true;
                continue;
            }
            if (!live[k]) continue;
            SolveJob& j = *live[k];
            if (!j.queued_all()) {
                if (j.step(false) != 0) moved = true;
                continue;
            }
            const hipError_t q = hipStreamQuery(j.stream());
            if (q == hipErrorNotReady) continue;
            status[who[k]] = j.finish();
            if (status[who[k]] < 0 && first_err == RPCA_OK) first_err = status[who[k]];
            live[k].reset();
            ++done;
            moved = true;
        }
        if (moved) {
            t_idle = std::chrono::steady_clock::now();
            continue;
        }
        cpu_relax();
        // Nothing advanced for a while: take the oldest live solve's next step
        // blocking, which also reports a failed or drained stream.
        if (std::chrono::steady_clock::now() - t_idle > std::chrono::microseconds(500)) {
            for (int32_t k = 0; k < n_streams; ++k) {
                if (live[k] && !live[k]->queued_all()) {
                    (void)live[k]->step(true);
                    break;
                }
            }
            t_idle = std::chrono::steady_clock::now();
        }
    }
    return first_err;
}

int rpca_batch_layout_of(const rpca_params* p, rpca_batch_layout* out) {
    if (!out) return RPCA_EINVAL;
    RPCA_TRY(validate(p));
    const Layout L = make_layout(p);
    const size_t elt = p->dtype == RPCA_F32 ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
    out->off_D = take(elt * (size_t)p->m * (size_t)p->ldd);
    out->off_U = take(sizeof(double) * (size_t)p->m * p->r);
    out->off_V = take(sizeof(double) * (size_t)p->n * p->r);
    out->off_sigma = take(sizeof(double) * p->r);
    out->off_ws = take(L.total);
    out->slab_bytes = off;
    return RPCA_OK;
}

// Every launch of the solve covers all instances (grid y); each instance's
// control block gates its own work, so instances that have finished a stage
// turn the later launches into no-ops. The host queues bodies a few at a time
// and reads all control blocks in between (one strided copy).
static_assert(sizeof(Ctrl) % 8 == 0, "control blocks are copied in 4-byte words, rows stay 8-byte aligned");

// One of the device's mapped, coherent host buffers for batched calls, locked
// for the caller: the first one free, else (every one in use) the first, once
// its call has ended.
std::unique_lock<std::mutex> take_batch_buffer(DeviceInfo* d, BatchBuf** out) {
    for (int i = 0; i < BATCH_BUFS; ++i) {
        std::unique_lock<std::mutex> lock(d->batch[i].mutex, std::try_to_lock);
        if (lock.owns_lock()) {
            *out = &d->batch[i];
            return lock;
        }
    }
    *out = &d->batch[0];
    return std::unique_lock<std::mutex>(d->batch[0].mutex);
}

// Grows a batch buffer (its mutex held by the caller) to at least `bytes`.
// Returns false if it cannot be allocated.
bool batch_buffer(BatchBuf* b, size_t bytes) {
    if (b->bytes >= bytes) return true;
    if (b->host) {
        (void)hipHostFree(b->host);
        b->host = b->dev = nullptr;
        b->bytes = 0;
    }
    void* h = nullptr;
    const size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
    if (hipHostMalloc(&h, want, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return false;
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, h, 0) != hipSuccess) {
        (void)hipHostFree(h);
        return false;
    }
    b->host = h;
    b->dev = dp;
    b->bytes = want;
    return true;
}

// Fields that every instance of a batch must share (one launch shape).
bool same_shape(const rpca_params* a, const rpca_params* b) {
    return a->m == b->m && a->n == b->n && a->ldd == b->ldd && a->r == b->r && a->dtype == b->dtype &&
           a->max_iter == b->max_iter && a->init_block == b->init_block &&
           a->init_max_passes == b->init_max_passes && a->flags == b->flags && a->seed == b->seed &&
           a->mixed_err == b->mixed_err && a->zeta_mlp == b->zeta_mlp;
}

int rpca_solve_batch(int32_t count, void* slabs, const rpca_params* params, rpca_state* st, double* err_hist,
                     double* zeta_hist, int32_t hist_cap, int32_t* status, void* stream) {
    if (count < 1 || !slabs || !params || !st || !status || hist_cap < 0 || ((uintptr_t)slabs & 255u) != 0)
        return RPCA_EINVAL;
    if (count > RPCA_BATCH_MAX) return RPCA_EINVAL;
    for (int32_t i = 0; i < count; ++i) status[i] = RPCA_EINVAL;
    const rpca_params* p = &params[0];
    for (int32_t i = 0; i < count; ++i) {
        RPCA_TRY(validate(&params[i]));
        if (!same_shape(p, &params[i])) return RPCA_EINVAL;
    }
    if ((p->flags & RPCA_FLAG_MIXED) && p->mixed_err > 0) return RPCA_EINVAL;
    rpca_batch_layout bl;
    RPCA_TRY(rpca_batch_layout_of(p, &bl));
    char* base = static_cast<char*>(slabs);
    Ctx c;
    RPCA_TRY(make_ctx(p, base + bl.off_ws, make_layout(p).total, stream, &c));
    c.batch = count;
    c.slab = (int64_t)bl.slab_bytes;
    c.events = false;
    const void* D0 = base + bl.off_D;
    double* U0 = reinterpret_cast<double*>(base + bl.off_U);
    double* V0 = reinterpret_cast<double*>(base + bl.off_V);
    double* s0 = reinterpret_cast<double*>(base + bl.off_sigma);
    // Control blocks and histories pass through mapped host memory, moved by a
    // kernel (one row per instance)
    const int cnt_h = hist_cap < p->max_iter + 1 ? hist_cap : p->max_iter + 1;
    const size_t row = sizeof(Ctrl) + 2 * sizeof(double) * (size_t)(cnt_h > 0 ? cnt_h : 0);
    BatchBuf* bb = nullptr;
    const std::unique_lock<std::mutex> hold = take_batch_buffer(c.dev, &bb);
    if (!batch_buffer(bb, row * (size_t)count)) {
        g_last_hip_error = (int)hipErrorOutOfMemory;
        return RPCA_EHIP;
    }
    void* const hb_dev = bb->dev;
    Ctrl* ctl = reinterpret_cast<Ctrl*>(bb->host);
    // (the host spins on the stream instead of a blocking wait, which can put
    // the thread to sleep for much longer than a few bodies take)
    auto read_all = [&]() -> int {
        HIP_TRY(launch_slab_copy(c.ctrl(), c.slab, hb_dev, (int64_t)row, sizeof(Ctrl), count, 0, c.s));
        hipError_t q;
        while ((q = hipStreamQuery(c.s)) == hipErrorNotReady) cpu_relax();
        HIP_TRY(q);
        std::atomic_thread_fence(std::memory_order_acquire);
        return RPCA_OK;
    };
    auto at = [&](int32_t i) -> Ctrl& { return *reinterpret_cast<Ctrl*>(reinterpret_cast<char*>(ctl) + row * i); };
    // Algorithm 3. Each instance's control block carries its own beta,
    // beta_init, gamma, mu and tol.
    const int P = c.L.K_init;
    const Ctrl t = base_ctrl(c, STAGE_SIGMA_D, INFINITY, 0, 1.0, 0);
    for (int32_t i = 0; i < count; ++i) at(i) = base_ctrl(c, STAGE_SIGMA_D, INFINITY, 0, 1.0, 0, &params[i]);
    std::atomic_thread_fence(std::memory_order_release);
    HIP_TRY(launch_slab_copy(c.ctrl(), c.slab, hb_dev, (int64_t)row, sizeof(Ctrl), count, 1, c.s));
    HIP_TRY(hipStreamSynchronize(c.s));
    PanelArgs sa = panel_args(c);
    sa.seed = p->seed;
    HIP_TRY(launch_start(sa, P, c.dtype, c.s));
    const int max_init = 2 * t.init_max_passes + 4;
    for (int b = 0; b < max_init;) {
        const int chunk = b == 0 ? 4 : 2;
        for (int j = 0; j < chunk && b < max_init; ++j, ++b)
            RPCA_TRY(enqueue_body(c, D0, P, BODY_INIT, nullptr, nullptr, nullptr, false, false, 0));
        RPCA_TRY(read_all());
        bool all = true;
        for (int32_t i = 0; i < count; ++i) all = all && at(i).stage >= STAGE_INIT_DONE;
        if (all) break;
    }
    RPCA_TRY(enqueue_enter(c, c.at<double>(c.L.off_Unew), c.at<double>(c.L.off_Vnew), P, c.small()->sigma_new, U0,
                           V0, s0));
    HIP_TRY(launch_enter_loop(c.ctrl(), c.batch, c.slab, c.s));
    // Algorithm 1 (the device's stopping rule ends each instance)
    const int max_main = p->max_iter + 3;
    for (int b = 0; b < max_main;) {
        const int chunk = b < 4 ? 4 : 2;
        for (int j = 0; j < chunk && b < max_main; ++j, ++b)
            RPCA_TRY(enqueue_body(c, D0, p->r, BODY_MAIN, U0, V0, s0, true, c.mixed, 0));
        RPCA_TRY(read_all());
        bool all = true;
        for (int32_t i = 0; i < count; ++i) all = all && at(i).done != 0;
        if (all) break;
    }
    RPCA_TRY(read_all());
    int first_err = RPCA_OK;
    for (int32_t i = 0; i < count; ++i) {
        const Ctrl f = at(i);
        char* bi = base + (size_t)i * bl.slab_bytes;
        int si;
        if (f.nonfinite == 1) si = RPCA_EINVAL;
        else if (f.nonfinite) si = RPCA_EBREAKDOWN;
        else if (f.stage != STAGE_MAIN || !f.done) si = RPCA_EHIP;
        else si = f.stopped_by_tol ? RPCA_OK : RPCA_MAXITER;
        status[i] = si;
        if (si < 0 && first_err == RPCA_OK) first_err = si;
        st[i].U = reinterpret_cast<double*>(bi + bl.off_U);
        st[i].V = reinterpret_cast<double*>(bi + bl.off_V);
        st[i].sigma = reinterpret_cast<double*>(bi + bl.off_sigma);
        fill_state(&st[i], f);
        st[i].init_passes = f.total_passes;
        st[i].reserved = 0;
    }
    if (cnt_h > 0 && (err_hist || zeta_hist)) {
        // err and zeta histories are adjacent in the workspace: one row each
        char* h0 = static_cast<char*>(hb_dev) + sizeof(Ctrl);
        HIP_TRY(launch_slab_copy(c.err_hist(), c.slab, h0, (int64_t)row, sizeof(double) * cnt_h, count, 0, c.s));
        HIP_TRY(launch_slab_copy(c.zeta_hist(), c.slab, h0 + sizeof(double) * cnt_h, (int64_t)row,
                                 sizeof(double) * cnt_h, count, 0, c.s));
        HIP_TRY(hipStreamSynchronize(c.s));
        std::atomic_thread_fence(std::memory_order_acquire);
        for (int32_t i = 0; i < count; ++i) {
            const double* hr = reinterpret_cast<const double*>(reinterpret_cast<char*>(ctl) + row * i + sizeof(Ctrl));
            if (err_hist) memcpy(err_hist + (size_t)i * hist_cap, hr, sizeof(double) * cnt_h);
            if (zeta_hist) memcpy(zeta_hist + (size_t)i * hist_cap, hr + cnt_h, sizeof(double) * cnt_h);
        }
    }
    if (trace_on()) {
        const bool h = cnt_h > 0 && (err_hist || zeta_hist);
        for (int32_t i = 0; i < count; ++i) {
            const double* hr = reinterpret_cast<const double*>(reinterpret_cast<char*>(ctl) + row * i + sizeof(Ctrl));
            const int n = at(i).k + 1 < cnt_h ? at(i).k + 1 : cnt_h;
            trace_solve("rpca_solve_batch", i, status[i], at(i), h ? hr : nullptr, h ? hr + cnt_h : nullptr, n,
                        &params[i]);
        }
    }
    return first_err;
}

int rpca_trim(const rpca_params* p, const rpca_state* st, double* U_tilde, double* V_tilde, void* ws,
              size_t ws_bytes, void* stream) {
    RPCA_TRY(check_state(st));
    if (!U_tilde || !V_tilde) return RPCA_EINVAL;
    Ctx c;
    RPCA_TRY(make_ctx(p, ws, ws_bytes, stream, &c));
    RPCA_TRY(setup(c, base_ctrl(c, STAGE_MAIN, st->zeta, st->k, 1.0, 0)));
    PanelArgs ua = panel_args(c);
    ua.mode = UPDATE_ENTER_EXACT;
    ua.srcU = st->U;
    ua.srcV = st->V;
    ua.ld_src = p->r;
    ua.src_sigma = st->sigma;
    HIP_TRY(launch_update(ua, p->r, c.dtype, c.s));
    PanelArgs ba = panel_args(c);
    ba.outU = U_tilde;
    ba.outV = V_tilde;
    HIP_TRY(launch_basis(ba, p->r, c.dtype, c.s));
    HIP_TRY(hipStreamSynchronize(c.s));
    return RPCA_OK;
}

namespace {
// ||D||_F^2 by one pass with zeta = +inf (every entry counts in the residual).
int compute_normD2(const Ctx& c, const void* D, double* out) {
    RPCA_TRY(setup(c, base_ctrl(c, STAGE_SIGMA_D, INFINITY, 0, 1.0, 0)));
    RPCA_TRY(threshold_pass(c, D, false));
    Ctrl t;
    RPCA_TRY(read_ctrl(c, &t));
    if (t.nonfinite) return RPCA_EINVAL;
    *out = t.normD2;
    return RPCA_OK;
}
}  // namespace

namespace {
int step_impl(const void* D, const rpca_params* p, rpca_state* st, void* ws, size_t ws_bytes, void* stream,
              bool events) {
    if (!D) return RPCA_EINVAL;
    RPCA_TRY(check_state(st));
    if (!is_fin(st->zeta) || st->k < 0) return RPCA_EINVAL;
    Ctx c;
    RPCA_TRY(make_ctx(p, ws, ws_bytes, stream, &c));
    c.events = events;
    double nd2 = st->normD > 0 ? st->normD * st->normD : 0.0;
    if (!(nd2 > 0)) RPCA_TRY(compute_normD2(c, D, &nd2));
    RPCA_TRY(setup(c, base_ctrl(c, STAGE_MAIN, st->zeta, st->k, nd2, 0)));
    const int K = p->r;
    // Trim(L_k) and its orthonormal bases
    RPCA_TRY(enqueue_enter(c, st->U, st->V, K, st->sigma, nullptr, nullptr, nullptr));
    // products with Z_k, the 2r x 2r update, zeta_{k+1}; L_{k+1} overwrites the state
    const bool mx = c.mixed && !(st->err > 0 && st->err < c.mixed_err);
    RPCA_TRY(enqueue_body(c, D, K, BODY_ANY, st->U, st->V, st->sigma, false, mx));
    // err_{k+1}: threshold pass at (L_{k+1}, zeta_{k+1})
    RPCA_TRY(threshold_pass(c, D, true));
    Ctrl t;
    RPCA_TRY(read_ctrl(c, &t));
    // a non-finite residual of the pass at L_k (D or the given state) stopped
    // the body before its update: the state is untouched
    if (t.nonfinite) return RPCA_EINVAL;
    fill_state(st, t);
    return RPCA_OK;
}
}  // namespace

int rpca_step(const void* D, const rpca_params* p, rpca_state* st, void* ws, size_t ws_bytes, void* stream) {
    return step_impl(D, p, st, ws, ws_bytes, stream, true);
}

int rpca_step_noalloc(const void* D, const rpca_params* p, rpca_state* st, void* stream) {
    RPCA_TRY(validate(p));
    if (make_layout(p).total > RPCA_NOALLOC_WS_BYTES) return RPCA_EWORKSPACE;
    DeviceInfo* dev = nullptr;
    RPCA_TRY(device_info(&dev));
    void* ws = nullptr;
    RPCA_TRY(noalloc_workspace(dev, &ws));
    return step_impl(D, p, st, ws, RPCA_NOALLOC_WS_BYTES, stream, false);
}

int rpca_relaxed_step(const void* D, const rpca_params* p, rpca_state* st, double zeta, double tau,
                      const double* P_true, const double* Q_true, int32_t r_true, rpca_relax_result* out, void* ws,
                      size_t ws_bytes, void* stream) {
    if (!D || !P_true || !Q_true || !out) return RPCA_EINVAL;
    RPCA_TRY(check_state(st));
    if (!p || !(p->flags & RPCA_FLAG_TRAINING)) return RPCA_EINVAL;
    if (r_true < 1 || r_true > RX_TRUE_MAX) return RPCA_EINVAL;
    if (!is_fin(zeta) || !(zeta > 0) || !is_fin(tau) || !(tau > 0)) return RPCA_EINVAL;
    Ctx c;
    RPCA_TRY(make_ctx(p, ws, ws_bytes, stream, &c));
    double nd2 = st->normD > 0 ? st->normD * st->normD : 0.0;
    if (!(nd2 > 0)) RPCA_TRY(compute_normD2(c, D, &nd2));
    RPCA_TRY(setup(c, base_ctrl(c, STAGE_MAIN, zeta, st->k, nd2, 0)));
    const int K = p->r;
    // Trim(L_k): bases U_f, V_f (with R_U, R_V) and the rebuild factors of L_k
    RPCA_TRY(enqueue_enter(c, st->U, st->V, K, st->sigma, nullptr, nullptr, nullptr));
    const Layout& L = c.L;
    RelaxArgs a;
    memset(&a, 0, sizeof(a));
    a.D = D;
    a.ldd = p->ldd;
    a.m = (int)p->m;
    a.n = (int)p->n;
    a.K = K;
    a.rt_true = r_true;
    a.AL = c.ws + L.off_AL;
    a.BL = c.ws + L.off_BL;
    a.Uf = c.ws + L.off_Uf;
    a.Vf = c.ws + L.off_Vf;
    a.zeta = zeta;
    a.tau = tau;
    a.normD2 = nd2;
    a.TM = L.rx_TM;
    a.n_ct = L.rx_nct;
    a.n_rt = L.rx_nrt;
    a.n_tiles = L.rx_nct * L.rx_nrt;
    a.gU = (a.m + 255) / 256;
    a.gV = (a.n + 255) / 256;
    a.R1 = c.at<double>(L.off_R1);
    a.R2 = c.at<double>(L.off_R2);
    a.Rres = c.at<double>(L.off_Rres);
    a.RY1 = c.at<double>(L.off_RY1);
    a.RY2 = c.at<double>(L.off_RY2);
    a.gpartR = c.at<double>(L.off_gpR);
    a.gram = c.at<double>(L.off_gram);
    a.gram2 = c.at<double>(L.off_gram2);
    a.P = P_true;
    a.Q = Q_true;
    a.RUinv = c.small()->RUinv;
    a.RVinv = c.small()->RVinv;
    a.coef = c.at<double>(L.off_coef);
    a.sigma_out = st->sigma;
    a.Uout = st->U;
    a.Vout = st->V;
    a.result = c.at<RelaxResult>(L.off_rres);
    a.ctrl = c.ctrl();
    HIP_TRY(launch_relax(a, c.dtype, c.s));
    RelaxResult r;
    HIP_TRY(hipMemcpyAsync(&r, a.result, sizeof(r), hipMemcpyDeviceToHost, c.s));
    HIP_TRY(hipStreamSynchronize(c.s));
    out->loss = r.loss;
    out->dloss_dzeta = r.dloss_dzeta;
    out->err = r.err;
    out->sigma1 = r.sigma1;
    out->sigma_r1 = r.sigma_r1;
    out->svd_sweeps = r.sweeps;
    out->reserved = 0;
    st->zeta = zeta;
    st->err = r.err;
    st->k += 1;
    st->sigma1_pt = r.sigma1;
    st->sigma_r1_pt = r.sigma_r1;
    st->normD = sqrt(nd2);
    return RPCA_OK;
}

int rpca_unrolled_adjoint(const void* D, const rpca_params* p, int32_t K, const double* const* U_ck,
                          const double* const* sigma_ck, const double* const* V_ck, const double* zeta,
                          const double* tau, const double* weight, const double* P_true, const double* Q_true,
                          int32_t r_true, double* zeta_bar, double* U_bar, double* sigma_bar, double* V_bar, void* ws,
                          size_t ws_bytes, void* stream) {
    if (!D || !U_ck || !sigma_ck || !V_ck || !zeta || !tau || !weight || !P_true || !Q_true || !zeta_bar || !U_bar ||
        !sigma_bar || !V_bar)
        return RPCA_EINVAL;
    if (!p || !(p->flags & RPCA_FLAG_TRAINING)) return RPCA_EINVAL;
    if (K < 1 || K > RPCA_MAX_UNROLL || r_true < 1 || r_true > RX_TRUE_MAX) return RPCA_EINVAL;
    for (int k = 0; k <= K; ++k)
        if (!U_ck[k] || !sigma_ck[k] || !V_ck[k]) return RPCA_EINVAL;
    for (int k = 0; k < K; ++k)
        if (!is_fin(zeta[k]) || !(zeta[k] > 0) || !is_fin(tau[k]) || !(tau[k] > 0) || !is_fin(weight[k]))
            return RPCA_EINVAL;
    Ctx c;
    RPCA_TRY(make_ctx(p, ws, ws_bytes, stream, &c));
    const Layout& L = c.L;
    AdjointBufs B;
    HIP_TRY(adjoint_carve(c.ws + L.off_adj, p->m, p->n, p->r, L.rx_nct, L.rx_nrt, &B));
    AdjointProblem P;
    memset(&P, 0, sizeof(P));
    P.D = D;
    P.ldd = p->ldd;
    P.m = p->m;
    P.n = p->n;
    P.dtype = c.dtype;
    P.K = p->r;
    P.Kt = K;
    P.rt = r_true;
    P.P = P_true;
    P.Q = Q_true;
    P.U = U_ck;
    P.sigma = sigma_ck;
    P.V = V_ck;
    P.zeta = zeta;
    P.tau = tau;
    P.weight = weight;
    const bool trim = !(p->flags & RPCA_FLAG_NO_TRIM);
    P.cU = trim ? sqrt(p->mu * (double)p->r / (double)p->m) : 0.0;
    P.cV = trim ? sqrt(p->mu * (double)p->r / (double)p->n) : 0.0;
    P.TM = L.rx_TM;
    P.n_ct = L.rx_nct;
    P.n_rt = L.rx_nrt;
    P.zeta_bar_dev = B.zbar;
    P.U_bar = U_bar;
    P.sigma_bar = sigma_bar;
    P.V_bar = V_bar;
    HIP_TRY(adjoint_run(P, B, c.s));
    std::vector<double> zb((size_t)K);
    HIP_TRY(hipMemcpyAsync(zb.data(), B.zbar, sizeof(double) * (size_t)K, hipMemcpyDeviceToHost, c.s));
    HIP_TRY(hipStreamSynchronize(c.s));
    for (int k = 0; k < K; ++k) zeta_bar[k] = zb[(size_t)k];
    return RPCA_OK;
}

int rpca_mlp_forward(const float* theta, const float* phi, int32_t batch, float* o, void* stream) {
    if (!theta || !phi || !o || batch < 0) return RPCA_EINVAL;
    DeviceInfo* dev = nullptr;
    RPCA_TRY(device_info(&dev));
    HIP_TRY(launch_mlp_forward(theta, phi, o, batch, static_cast<hipStream_t>(stream)));
    return RPCA_OK;
}

int rpca_mlp_backward(const float* theta, const float* phi, const float* grad_o, int32_t batch, float* grad_theta,
                      void* stream) {
    if (!theta || !phi || !grad_o || !grad_theta || batch < 0) return RPCA_EINVAL;
    DeviceInfo* dev = nullptr;
    RPCA_TRY(device_info(&dev));
    HIP_TRY(launch_mlp_backward(theta, phi, grad_o, batch, grad_theta, static_cast<hipStream_t>(stream)));
    return RPCA_OK;
}

int rpca_mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t t, float lr, float beta1, float beta2,
                  float eps, void* stream) {
    if (!theta || !m || !v || !grad || t < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return RPCA_EINVAL;
    DeviceInfo* dev = nullptr;
    RPCA_TRY(device_info(&dev));
    HIP_TRY(launch_mlp_adam(theta, m, v, grad, t, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream)));
    return RPCA_OK;
}

int rpca_materialize(const void* D, const rpca_params* p, const rpca_state* st, void* L_out, int64_t ldl,
                     void* S_out, int64_t lds, void* ws, size_t ws_bytes, void* stream) {
    if (!D) return RPCA_EINVAL;
    RPCA_TRY(check_state(st));
    if ((L_out && ldl < p->n) || (S_out && lds < p->n)) return RPCA_EINVAL;
    Ctx c;
    RPCA_TRY(make_ctx(p, ws, ws_bytes, stream, &c));
    RPCA_TRY(setup(c, base_ctrl(c, STAGE_MAIN, st->zeta, st->k, 1.0, 0)));
    const int K = p->r;
    HIP_TRY(launch_convert(st->U, c.ws + c.L.off_AL, p->m * K, st->sigma, K, c.dtype, c.s));
    HIP_TRY(launch_convert(st->V, c.ws + c.L.off_BL, p->n * K, nullptr, K, c.dtype, c.s));
    MaterializeArgs a;
    a.D = D;
    a.ldd = p->ldd;
    a.m = (int)p->m;
    a.n = (int)p->n;
    a.AL = c.ws + c.L.off_AL;
    a.BL = c.ws + c.L.off_BL;
    a.ctrl = c.ctrl();
    a.L_out = L_out;
    a.ldl = ldl;
    a.S_out = S_out;
    a.lds = lds;
    if (L_out || S_out) HIP_TRY(launch_materialize(a, K, c.dtype, c.s));
    HIP_TRY(hipStreamSynchronize(c.s));
    return RPCA_OK;
}

int rpca_tangent_products(const void* D, const rpca_params* p, const double* A_L, const double* B_L,
                          double zeta, const double* U_t, const double* V_t, double* Y1, double* Y2,
                          double* resid2, void* ws, size_t ws_bytes, void* stream) {
    if (!D || !A_L || !B_L || !U_t || !V_t || !Y1 || !Y2 || !resid2 || isnan(zeta)) return RPCA_EINVAL;
    Ctx c;
    RPCA_TRY(make_ctx(p, ws, ws_bytes, stream, &c));
    const int K = p->r;
    RPCA_TRY(setup(c, base_ctrl(c, STAGE_MAIN, zeta, 0, 1.0, 0)));
    HIP_TRY(launch_convert(A_L, c.ws + c.L.off_AL, p->m * K, nullptr, K, c.dtype, c.s));
    HIP_TRY(launch_convert(B_L, c.ws + c.L.off_BL, p->n * K, nullptr, K, c.dtype, c.s));
    HIP_TRY(launch_convert(U_t, c.ws + c.L.off_Uf, p->m * K, nullptr, K, c.dtype, c.s));
    HIP_TRY(launch_convert(V_t, c.ws + c.L.off_Vf, p->n * K, nullptr, K, c.dtype, c.s));
    HIP_TRY(launch_cross(panel_args(c), K, c.dtype, c.s));   // AL^T U_f, BL^T V_f for the gather
    const Geo g = geo_for(c, K, true, c.mixed);
    RPCA_TRY(stream_launch(stream_args(c, D, BODY_ANY, g), K, c.dtype, true, c.mixed, c.s));
    PanelArgs pa = panel_args(c, g);
    pa.Y1 = Y1;
    pa.Y2 = Y2;
    pa.lcorr = 1;
    HIP_TRY(launch_gather(pa, K, c.dtype, c.s));
    Ctrl t;
    RPCA_TRY(read_ctrl(c, &t));
    *resid2 = t.resid2;
    return RPCA_OK;
}

}  // extern "C"
