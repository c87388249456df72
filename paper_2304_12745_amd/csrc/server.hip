// Serving runtime: continuous batching of power-map queries on one GPU.
//
// A query names a resident deployment (antenna positions uploaded once by
// dmimo_server_add_deployment) and brings K user positions, a precoder, a
// grid and two caller-owned output maps.  A worker thread owns the device
// and runs a loop:
//   * admission: pending queries are admitted while a slot is free and
//     their HBM footprint (server scratch + output maps) fits the budget.
//     The scratch comes from one arena allocated at creation; nothing is
//     allocated afterwards.  An admitted query gets its user channel and
//     precoder on the server stream: for MR and ZF one launch of the
//     one-pass beamform kernel, which synthesises the channel itself (ZF
//     with its Gram and FP64 inverse), for other shapes the channel kernel
//     and then the beamform kernels; for DMIMO_PA the channel kernel and
//     the PA-aware precoder.
//   * ticks: each tick is one launch of serve_kernel, a fixed grid that
//     loops over a list of (query, 128- or 256-point tile) work items.  The
//     items come from every active query, smallest remaining work first,
//     up to a budget of channel terms per tick.  Queries that arrive while
//     others run join at the next tick, so their work overlaps on the device.
//     Two ticks may be in flight; each work list lives in pinned memory and
//     is reused only after its tick completed.
//   * completion: a query is done when the tick holding its last tile has
//     completed (one event per tick).  Its slot and memory are released.
// A point's value is reduced by one workgroup in a fixed antenna order, so a
// query's maps are bitwise the same whether it runs alone or in a mix.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "kernels.h"
#include "powermap_body.h"
#include "server_arena.h"

namespace dmimo {

namespace {

constexpr int kServeWaves = 8;
constexpr int kServeThreads = 64 * kServeWaves;

// item modes: precision x stream-count bucket
enum : int32_t {
    kF32Nt1 = 0, kF32Nt2, kF32Nt4, kF16Nt1, kF16Nt2, kF16Nt4, kBf16Nt1, kBf16Nt2, kBf16Nt4,
    kF32K1, kF32K2   // FP32, one or two streams: the VALU map, as in dmimo_powermap
};

struct ServeItem {
    int32_t slot;
    int32_t mode;
    int64_t first;   // first point of the tile
};

// split-precision modes with more than 8 streams run the many-stream body
// (map_x3w_wg) with kServeX3wPt tiles per wave
constexpr int kServeX3wPt = 2;

bool x3w_mode(int mode) {
    return mode == kF16Nt2 || mode == kF16Nt4 || mode == kBf16Nt2 || mode == kBf16Nt4;
}

// points of one work item: 16 PT points per wave (one point per lane for VALU)
int tile_points(int mode) {
    if (mode >= kF32K1) return kServeThreads;
    if (x3w_mode(mode)) return 16 * kServeX3wPt * kServeWaves;
    return mode < kF16Nt1 ? 16 * 2 * kServeWaves : 16 * kServeWaves;
}

// One launch per mode present in a tick: a fixed grid looping over that
// mode's items (each mode keeps the register budget of its own map body).
template <int KT>
__global__ __launch_bounds__(kServeThreads) void serve_valu_kernel(
    const PmMapDev* __restrict__ slots, const ServeItem* __restrict__ items, int n_items) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const ServeItem w = items[it];
        const PmMapDev a = slots[w.slot];
        map_valu_wg<KT>(a, w.first);
    }
}

template <int MODE>
__global__ __launch_bounds__(kServeThreads) __attribute__((amdgpu_waves_per_eu(4)))
void serve_kernel(const PmMapDev* __restrict__ slots, const ServeItem* __restrict__ items,
                  int n_items) {
    constexpr int NT = MODE % 3 == 0 ? 1 : (MODE % 3 == 1 ? 2 : 4);
    constexpr bool X3 = MODE >= kF16Nt1;
    constexpr bool BF16 = MODE >= kBf16Nt1;
    constexpr int PT = X3 ? 1 : 2;   // one 16-point tile per wave keeps x3 within 128 VGPRs
    constexpr int LDS = X3 ? x3_lds_bytes<NT, PT, kServeWaves>() : f32_lds_bytes<NT, PT, kServeWaves>();
    __shared__ __attribute__((aligned(16))) char smem[LDS];
    __shared__ float s_red[kServeWaves];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const ServeItem w = items[it];
        const PmMapDev a = slots[w.slot];
        if constexpr (X3) map_x3_wg<NT, PT, BF16, kServeWaves, false>(a, w.first, smem, s_red);
        else map_f32_wg<NT, PT, kServeWaves>(a, w.first, smem);
        __syncthreads();   // LDS is reused by the next item
    }
}

// The many-stream split-precision modes: the body of the one-shot map kernel
// (the same bits per point for any workgroup shape), two waves per SIMD.
template <int NT, bool BF16>
__global__ __launch_bounds__(kServeThreads) __attribute__((amdgpu_waves_per_eu(2)))
void serve_x3w_kernel(const PmMapDev* __restrict__ slots, const ServeItem* __restrict__ items,
                      int n_items) {
    __shared__ __attribute__((aligned(16))) char smem[x3w_lds_bytes<NT, kServeX3wPt, kServeWaves>()];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const ServeItem w = items[it];
        const PmMapDev a = slots[w.slot];
        map_x3w_wg<NT, kServeX3wPt, BF16, kServeWaves>(a, w.first, smem);
        __syncthreads();   // LDS is reused by the next item
    }
}

using ServeKernel = void (*)(const PmMapDev*, const ServeItem*, int);
const ServeKernel kServeKernels[11] = {serve_kernel<0>, serve_kernel<1>, serve_kernel<2>,
                                       serve_kernel<3>, serve_x3w_kernel<2, false>,
                                       serve_x3w_kernel<4, false>, serve_kernel<6>,
                                       serve_x3w_kernel<2, true>, serve_x3w_kernel<4, true>,
                                       serve_valu_kernel<1>, serve_valu_kernel<2>};

double now_s() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct Deployment {
    WaveConst w;
    int M;
    size_t off;   // arena offset of FP64 [M][3]
};

enum QState : int32_t { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3, kCancelled = 4,
                         kTimedOut = 5 };

struct Query {
    uint64_t ticket = 0;
    int dep = 0;
    int K = 0;
    double users[DMIMO_K_MAX * 3];
    int precoder = 0;
    PointsDev P;
    double sigma2 = 0, p_total = 0;
    int prec = DMIMO_F32;
    float* power = nullptr;
    float* sinr = nullptr;
    // runtime
    int mode = 0;
    int64_t tile = 0, n_items = 0, next_item = 0;
    double item_terms = 0;   // channel terms of one tile (tile points x M)
    int slot = -1;
    size_t off = 0, bytes = 0, footprint = 0;
    int64_t last_tick = -1;
    std::atomic<int32_t> state{kQueued};
    double t_submit = 0, t_done = 0;
    int64_t terms = 0;
    int32_t info = 0;    // ZF: the failed pivot (copied from the device at retirement)
};

}  // namespace

struct ServerImpl {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0, in_use = 0, geom_bytes = 0;
    int max_inflight = 0;
    char* arena_base = nullptr;
    Arena arena;
    std::vector<Deployment> deps;
    // slot table: device array + pinned host mirror + per-slot pinned user staging
    PmMapDev* d_slots = nullptr;
    PmMapDev* h_slots = nullptr;
    double* h_users = nullptr;
    int32_t* h_info = nullptr;   // pinned: each slot's precoder info word, copied back
    std::vector<int> free_slots;
    double queue_timeout = 0.0;   // seconds a query may wait for admission; 0 = no limit
    // work lists (double buffered)
    int item_cap = 0;
    ServeItem* h_items[2] = {nullptr, nullptr};
    ServeItem* d_items[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    int64_t tick_of_buf[2] = {-1, -1};
    int64_t ticks_issued = 0, ticks_done = 0;
    // channel terms per tick (about 0.4 ms of map work): at 2000 queries/s of
    // the serving mix with two workgroups per CU, 6e7 gave p50 / p99 0.17 /
    // 1.68 ms, 3e7 0.15 / 2.09, 1.2e8 0.16 / 1.53, 2.4e8 0.15 / 1.33, 4.8e8
    // 0.15 / 1.40, 1e9 0.14 / 1.48; with three (grid below), 1.6e8 0.16 /
    // 1.36, 2.4e8 0.15 / 1.35, 3.2e8 0.14 / 1.29, 4.8e8 0.14 / 1.38, 6.4e8
    // 0.14 / 1.44
    double tick_terms = 3.2e8;
    int grid = 512;
    // schedule of DMIMO_PA queries (device FP64 [2][layers] in the arena)
    int pa_layers = -1;
    const double* pa_lam = nullptr;
    const double* pa_eta = nullptr;
    double pa_gamma[DMIMO_K_MAX];
    // queries
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Query*> pending;
    std::vector<Query*> active;
    std::map<uint64_t, Query*> all;
    uint64_t next_ticket = 1;
    std::atomic<bool> stop{false};
    std::thread worker;
    std::string err;
    // stats
    std::atomic<int64_t> n_done{0}, terms_done{0};

    void loop();
    // 1 = admitted (or failed at once), 0 = not now, -1 = can never be admitted
    int admit_one(Query* q);
    void retire_ticks(bool block);
    void finish(Query* q, bool ok);
};

static bool hip_ok(hipError_t e, ServerImpl* s, const char* what) {
    if (e == hipSuccess) return true;
    s->err = std::string(what) + ": " + hipGetErrorString(e);
    return false;
}

int ServerImpl::admit_one(Query* q) {
    const Deployment& d = deps[q->dep];
    const int K = q->K;
    const size_t M = (size_t)d.M;
    const size_t users_b = align256((size_t)K * 3 * 8);
    const size_t h_b = align256((size_t)K * M * 8);
    const size_t w_b = align256((size_t)K * M * 8);
    const size_t g_b = align256(beamform_workspace_bytes(q->precoder, 1, K, M, q->prec));
    const size_t pa_b = q->precoder == DMIMO_PA ? align256(2 * sizeof(double)) : 0;
    const size_t info_b = 256;
    q->bytes = users_b + h_b + w_b + g_b + pa_b + info_b;
    if (in_use + q->footprint > budget) return active.empty() ? -1 : 0;
    if (free_slots.empty()) return 0;
    size_t off;
    // with no query running, the space below the resident data is one block:
    // a query that does not fit then never will
    if (!arena.alloc_low(q->bytes, &off)) return active.empty() ? -1 : 0;
    q->off = off;
    q->slot = free_slots.back();
    free_slots.pop_back();
    in_use += q->footprint;
    char* base = arena_base + off;
    double* d_users = reinterpret_cast<double*>(base);
    void* H = base + users_b;
    void* W = base + users_b + h_b;
    void* G = base + users_b + h_b + w_b;
    int32_t* d_info = reinterpret_cast<int32_t*>(base + users_b + h_b + w_b + g_b + pa_b);
    h_info[q->slot] = 0;
    // user positions: pinned staging of this slot -> device
    double* stage = h_users + (size_t)q->slot * DMIMO_K_MAX * 3;
    std::memcpy(stage, q->users, sizeof(double) * 3 * K);
    bool ok = hip_ok(hipMemcpyAsync(d_users, stage, sizeof(double) * 3 * K, hipMemcpyHostToDevice,
                                    stream), this, "users upload");
    PointsDev up;
    std::memset(&up, 0, sizeof(up));
    up.kind = DMIMO_PTS_LIST;
    up.xyz = d_users;
    up.n = K;
    const double* ap = reinterpret_cast<const double*>(arena_base + d.off);
    if (q->precoder == DMIMO_PA) {
        ok = ok && launch_channel(d.w, up, false, 1, d.M, ap, nullptr, false, H, stream) == DMIMO_OK;
        void* pa_ws = base + users_b + h_b + w_b + g_b;
        ok = ok && launch_pa_precoder(1, K, d.M, H, pa_gamma, q->sigma2, pa_layers, pa_lam, pa_eta,
                                      W, nullptr, nullptr, nullptr, nullptr, pa_ws, DMIMO_F32,
                                      stream) == DMIMO_OK;
    } else {
        BeamformArgs ba;
        std::memset(&ba, 0, sizeof(ba));
        ba.precoder = q->precoder;
        ba.B = 1;
        ba.K = K;
        ba.M = d.M;
        ba.H = H;
        for (int k = 0; k < DMIMO_K_MAX; ++k) ba.gamma[k] = 1.0;
        ba.sigma2 = q->sigma2;
        ba.p_total = q->p_total;
        ba.prec = q->prec;
        ba.W = W;
        ba.ws = G;
        ba.info = d_info;   // a failed ZF pivot fails the query (read back at retirement)
        const int pc = q->precoder;
        ok = ok && launch_beamform_users(ba, 1, &pc, d.w, ap, d_users, stream) == DMIMO_OK;
        ok = ok && hip_ok(hipMemcpyAsync(h_info + q->slot, d_info, sizeof(int32_t),
                                         hipMemcpyDeviceToHost, stream), this, "info copy");
    }
    // map descriptor of the slot
    PmMapDev& m = h_slots[q->slot];
    m.P = q->P;
    m.M = d.M;
    m.K = K;
    m.G = K;
    m.inv_lam = d.w.inv_lam;
    m.amp_rev = (float)(1.0 / (4.0 * kPi));
    m.inv_dmin_rev = (float)(d.w.inv_dmin / d.w.inv_lam);
    m.hexp = fp16_h_exponent(m.amp_rev, m.inv_dmin_rev);
    m.ap = ap;
    m.W = reinterpret_cast<const float2*>(W);
    m.sigma2 = (float)q->sigma2;
    m.power = q->power;
    m.sinr = q->sinr;
    m.best_k = nullptr;
    m.per_stream = nullptr;
    ok = ok && hip_ok(hipMemcpyAsync(d_slots + q->slot, &m, sizeof(PmMapDev), hipMemcpyHostToDevice,
                                     stream), this, "slot upload");
    const int nt = K <= 8 ? 0 : (K <= 16 ? 1 : 2);
    q->mode = (q->prec == DMIMO_F32 ? kF32Nt1 : (q->prec == DMIMO_MIX_F16X3 ? kF16Nt1 : kBf16Nt1)) + nt;
    if (q->prec == DMIMO_F32 && K <= 2) q->mode = K == 1 ? kF32K1 : kF32K2;
    q->tile = tile_points(q->mode);
    q->n_items = ceil_div(q->P.n, q->tile);
    q->item_terms = (double)q->tile * (double)d.M;
    q->next_item = 0;
    q->state.store(kRunning);
    if (!ok) {
        finish(q, false);
        return true;
    }
    active.push_back(q);
    return true;
}

void ServerImpl::finish(Query* q, bool ok) {
    q->t_done = now_s();
    if (q->slot >= 0) {
        arena.release(q->off, q->bytes);
        free_slots.push_back(q->slot);
        in_use -= q->footprint;
        q->slot = -1;
    }
    if (ok) {
        n_done++;
        terms_done += q->terms;
    }
    q->state.store(ok ? kDone : kFailed);
}

// Retire completed ticks: queries whose last tile ran in a completed tick are done.
void ServerImpl::retire_ticks(bool block) {
    while (ticks_done < ticks_issued) {
        const int buf = (int)(ticks_done & 1);
        if (block) {
            hipEventSynchronize(ev[buf]);
            block = false;
        } else if (hipEventQuery(ev[buf]) != hipSuccess) {
            break;
        }
        const int64_t t = ticks_done++;
        std::lock_guard<std::mutex> lk(mu);
        for (auto it = active.begin(); it != active.end();) {
            Query* q = *it;
            if (q->next_item == q->n_items && q->last_tick <= t) {
                // the tick ran after the precoder on the same stream, so the
                // precoder's info word has been copied back
                q->info = h_info[q->slot];
                finish(q, q->info == 0);
                it = active.erase(it);
            } else {
                ++it;
            }
        }
        cv.notify_all();
    }
}

void ServerImpl::loop() {
    hipSetDevice(device);
    while (true) {
        retire_ticks(false);
        {
            std::unique_lock<std::mutex> lk(mu);
            bool admitted = false;
            const double now = now_s();
            while (!pending.empty()) {
                Query* q = pending.front();
                if (queue_timeout > 0.0 && now - q->t_submit > queue_timeout) {
                    pending.pop_front();
                    q->t_done = now;
                    q->state.store(kTimedOut);
                    admitted = true;
                    continue;
                }
                const int r = admit_one(q);
                if (r == 0) break;
                pending.pop_front();
                if (r < 0) {   // nothing is running and it still does not fit
                    q->t_done = now;
                    q->state.store(kFailed);
                }
                admitted = true;
            }
            if (admitted) cv.notify_all();
            bool work = false;
            for (Query* q : active) work |= q->next_item < q->n_items;
            if (!work) {
                if (ticks_done < ticks_issued) {
                    lk.unlock();
                    retire_ticks(true);
                    continue;
                }
                if (stop.load() && pending.empty()) break;
                cv.wait_for(lk, std::chrono::microseconds(200));
                continue;
            }
        }
        if (ticks_issued - ticks_done >= 2) {
            retire_ticks(true);
            continue;
        }
        // build the next tick: smallest remaining work first
        const int buf = (int)(ticks_issued & 1);
        int n = 0;
        {
            std::lock_guard<std::mutex> lk(mu);
            std::vector<Query*> order;
            for (Query* q : active)
                if (q->next_item < q->n_items) order.push_back(q);
            // remaining channel terms, ascending; ties by arrival (ticket)
            std::sort(order.begin(), order.end(), [](const Query* x, const Query* y) {
                const double rx = (double)(x->n_items - x->next_item) * x->item_terms;
                const double ry = (double)(y->n_items - y->next_item) * y->item_terms;
                return rx < ry || (rx == ry && x->ticket < y->ticket);
            });
            double left = tick_terms;
            for (Query* q : order) {
                if (left <= 0 || n >= item_cap) break;
                const double per = q->item_terms;
                int64_t take = std::max<int64_t>(1, (int64_t)(left / per));
                take = std::min<int64_t>(take, q->n_items - q->next_item);
                take = std::min<int64_t>(take, item_cap - n);
                for (int64_t i = 0; i < take; ++i) {
                    ServeItem& it = h_items[buf][n++];
                    it.slot = q->slot;
                    it.mode = q->mode;
                    it.first = (q->next_item + i) * q->tile;
                }
                q->next_item += take;
                if (q->next_item == q->n_items) q->last_tick = ticks_issued;
                left -= per * (double)take;
            }
        }
        if (n == 0) continue;
        // group the items by mode (stable: each query's tiles keep their order)
        std::stable_sort(h_items[buf], h_items[buf] + n,
                         [](const ServeItem& x, const ServeItem& y) { return x.mode < y.mode; });
        hipMemcpyAsync(d_items[buf], h_items[buf], sizeof(ServeItem) * n, hipMemcpyHostToDevice, stream);
        for (int i0 = 0; i0 < n;) {
            int i1 = i0;
            while (i1 < n && h_items[buf][i1].mode == h_items[buf][i0].mode) ++i1;
            kServeKernels[h_items[buf][i0].mode]<<<dim3((unsigned)std::min(i1 - i0, grid)),
                                                   dim3(kServeThreads), 0, stream>>>(
                d_slots, d_items[buf] + i0, i1 - i0);
            i0 = i1;
        }
        hipEventRecord(ev[buf], stream);
        tick_of_buf[buf] = ticks_issued;
        ticks_issued++;
    }
    hipStreamSynchronize(stream);
}

}  // namespace dmimo

using namespace dmimo;

struct dmimo_server {
    ServerImpl impl;
};

extern "C" {

dmimo_status dmimo_server_create(int32_t device, size_t hbm_budget_bytes, int32_t max_inflight,
                                 dmimo_server** srv) {
    clear_error();
    if (!srv) return fail(DMIMO_E_ARG, "server_create: srv is NULL");
    if (hbm_budget_bytes < (1u << 20)) return fail(DMIMO_E_ARG, "server_create: budget below 1 MiB");
    if (max_inflight < 1 || max_inflight > 4096)
        return fail(DMIMO_E_ARG, "server_create: max_inflight must be in [1, 4096]");
    if (device < 0) return fail(DMIMO_E_ARG, "server_create: bad device");
    auto* s = new dmimo_server();
    ServerImpl& S = s->impl;
    S.device = device;
    S.budget = hbm_budget_bytes;
    S.max_inflight = max_inflight;
    S.item_cap = 1 << 16;
    bool ok = hip_ok(hipSetDevice(device), &S, "hipSetDevice") &&
              hip_ok(hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking), &S, "stream") &&
              hip_ok(hipMalloc(&S.arena_base, hbm_budget_bytes), &S, "arena") &&
              hip_ok(hipMalloc(&S.d_slots, sizeof(PmMapDev) * max_inflight), &S, "slots") &&
              hip_ok(hipHostMalloc(&S.h_slots, sizeof(PmMapDev) * max_inflight), &S, "pinned slots") &&
              hip_ok(hipHostMalloc(&S.h_users, sizeof(double) * DMIMO_K_MAX * 3 * max_inflight), &S,
                     "pinned users") &&
              hip_ok(hipHostMalloc(&S.h_info, sizeof(int32_t) * max_inflight), &S, "pinned info");
    for (int i = 0; ok && i < 2; ++i)
        ok = hip_ok(hipHostMalloc(&S.h_items[i], sizeof(ServeItem) * S.item_cap), &S, "pinned items") &&
             hip_ok(hipMalloc(&S.d_items[i], sizeof(ServeItem) * S.item_cap), &S, "items") &&
             hip_ok(hipEventCreateWithFlags(&S.ev[i], hipEventDisableTiming), &S, "event");
    if (ok) {
        int cus = 0;
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
        // three workgroups per CU per mode launch (each loops over its
        // mode's items): p50 / p99 0.15 / 1.32 ms against 0.16 / 1.34 with two
        // and 0.18 / 1.68 with one (2000 queries/s, 2.4e8 terms per tick)
        S.grid = std::max(1, cus) * 3;
    }
    if (!ok) {
        set_error("%s", S.err.c_str());
        dmimo_server_destroy(s);
        return DMIMO_E_HIP;
    }
    S.arena.init(hbm_budget_bytes);
    for (int i = max_inflight - 1; i >= 0; --i) S.free_slots.push_back(i);
    S.worker = std::thread([&S] { S.loop(); });
    *srv = s;
    return DMIMO_OK;
}

dmimo_status dmimo_server_add_deployment(dmimo_server* srv, const dmimo_channel_params* params,
                                         int32_t M, const double* ap_xyz_host, int32_t* dep_id) {
    clear_error();
    if (!srv || !ap_xyz_host || !dep_id) return fail(DMIMO_E_ARG, "add_deployment: NULL argument");
    WaveConst w;
    dmimo_status st = make_wave_const(params, &w);
    if (st) return st;
    if (params->model != DMIMO_CH_LOS)
        return fail(DMIMO_E_UNSUPPORTED, "add_deployment: maps use the LoS model");
    if (M < 1) return fail(DMIMO_E_SHAPE, "add_deployment: M must be >= 1");
    ServerImpl& S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    const size_t bytes = (size_t)M * 3 * sizeof(double);
    size_t off;
    // resident data comes from the top of the arena, query scratch from the bottom
    if (S.in_use + align256(bytes) > S.budget || !S.arena.alloc_high(bytes, &off))
        return fail(DMIMO_E_NOMEM, "add_deployment: geometry does not fit the budget (or the "
                                   "space not used by running queries)");
    S.in_use += align256(bytes);
    S.geom_bytes += align256(bytes);
    if (hipMemcpy(S.arena_base + off, ap_xyz_host, bytes, hipMemcpyHostToDevice) != hipSuccess) {
        S.arena.release(off, bytes);
        S.in_use -= align256(bytes);
        S.geom_bytes -= align256(bytes);
        return fail(DMIMO_E_HIP, "add_deployment: upload failed");
    }
    Deployment d;
    d.w = w;
    d.M = M;
    d.off = off;
    S.deps.push_back(d);
    *dep_id = (int32_t)S.deps.size() - 1;
    return DMIMO_OK;
}

dmimo_status dmimo_server_submit(dmimo_server* srv, int32_t dep_id, int32_t K,
                                 const double* user_xyz_host, int32_t precoder,
                                 const dmimo_points* pts, double sigma2, double p_total, int32_t prec,
                                 float* power_out_dev, float* sinr_out_dev, uint64_t* ticket) {
    clear_error();
    if (!srv || !user_xyz_host || !pts || !power_out_dev || !ticket)
        return fail(DMIMO_E_ARG, "submit: NULL argument");
    ServerImpl& S = srv->impl;
    PointsDev P;
    dmimo_status st = make_points(pts, &P);
    if (st) return st;
    if (P.n < 1) return fail(DMIMO_E_SHAPE, "submit: empty point set");
    if (precoder != DMIMO_MR && precoder != DMIMO_ZF && precoder != DMIMO_MR_PHASE &&
        precoder != DMIMO_PA)
        return fail(DMIMO_E_DTYPE, "submit: unknown precoder");
    if (precoder == DMIMO_PA && !(sigma2 > 0.0))
        return fail(DMIMO_E_ARG, "submit: DMIMO_PA needs sigma2 > 0");
    if (prec != DMIMO_F32 && prec != DMIMO_MIX_F16X3 && prec != DMIMO_MIX_BF16X3)
        return fail(DMIMO_E_UNSUPPORTED, "submit: serving runs FP32 or mixed precision");
    if (!(sigma2 >= 0.0) || (sinr_out_dev && !(sigma2 > 0.0)))
        return fail(DMIMO_E_ARG, "submit: bad sigma2");
    auto* q = new Query();
    {
        std::lock_guard<std::mutex> lk(S.mu);
        if (dep_id < 0 || dep_id >= (int)S.deps.size()) {
            delete q;
            return fail(DMIMO_E_NOTFOUND, "submit: unknown deployment");
        }
        const int M = S.deps[dep_id].M;
        if (K < 1 || K > DMIMO_K_MAX || (precoder == DMIMO_ZF && K > M)) {
            delete q;
            return fail(DMIMO_E_SHAPE, "submit: K must be in [1, min(32, M)] (ZF)");
        }
        if (precoder == DMIMO_PA && (K > 16 || M > 256)) {
            delete q;
            return fail(DMIMO_E_SHAPE, "submit: DMIMO_PA needs K <= 16 and M <= 256");
        }
        if (precoder == DMIMO_PA && S.pa_layers < 0) {
            delete q;
            return fail(DMIMO_E_ARG, "submit: no DMIMO_PA schedule (dmimo_server_set_pa_schedule)");
        }
        if (S.pending.size() >= (size_t)(S.max_inflight) * 64) {
            delete q;
            return fail(DMIMO_E_BUSY, "submit: pending queue full");
        }
        q->dep = dep_id;
        q->K = K;
        std::memcpy(q->users, user_xyz_host, sizeof(double) * 3 * K);
        q->precoder = precoder;
        q->P = P;
        q->sigma2 = sigma2;
        q->p_total = p_total;
        q->prec = prec;
        q->power = power_out_dev;
        q->sinr = sinr_out_dev;
        q->terms = P.n * (int64_t)M;
        const size_t scratch = align256((size_t)K * 24) + 2 * align256((size_t)K * M * 8) +
                               align256(beamform_workspace_bytes(precoder, 1, K, M, prec)) +
                               (precoder == DMIMO_PA ? align256(2 * sizeof(double)) : 0);
        q->footprint = scratch + (size_t)P.n * 4 * (sinr_out_dev ? 2 : 1);
        if (q->footprint > S.budget - S.geom_bytes) {
            delete q;
            return fail(DMIMO_E_NOMEM, "submit: query footprint exceeds the HBM budget");
        }
        q->ticket = S.next_ticket++;
        q->t_submit = now_s();
        S.all[q->ticket] = q;
        S.pending.push_back(q);
        *ticket = q->ticket;
    }
    S.cv.notify_all();
    return DMIMO_OK;
}

dmimo_status dmimo_server_set_pa_schedule(dmimo_server* srv, int32_t layers,
                                          const double* lambdas, const double* eta_rel,
                                          double gamma_lin) {
    clear_error();
    if (!srv) return fail(DMIMO_E_ARG, "set_pa_schedule: NULL server");
    if (layers < 0) return fail(DMIMO_E_SHAPE, "set_pa_schedule: layers must be >= 0");
    if (layers > 0 && (!lambdas || !eta_rel)) return fail(DMIMO_E_ARG, "set_pa_schedule: NULL schedule");
    if (!(gamma_lin > 0.0) || !std::isfinite(gamma_lin))
        return fail(DMIMO_E_ARG, "set_pa_schedule: gamma_lin must be > 0");
    ServerImpl& S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.pa_layers >= 0) return fail(DMIMO_E_BUSY, "set_pa_schedule: already set");
    const size_t bytes = sizeof(double) * 2 * (size_t)std::max(layers, 1);
    size_t off;
    if (S.in_use + align256(bytes) > S.budget || !S.arena.alloc_high(bytes, &off))
        return fail(DMIMO_E_NOMEM, "set_pa_schedule: schedule does not fit the budget");
    double* dev = reinterpret_cast<double*>(S.arena_base + off);
    if (layers > 0 &&
        (hipMemcpy(dev, lambdas, sizeof(double) * layers, hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy(dev + layers, eta_rel, sizeof(double) * layers, hipMemcpyHostToDevice) != hipSuccess)) {
        S.arena.release(off, bytes);
        return fail(DMIMO_E_HIP, "set_pa_schedule: upload failed");
    }
    S.in_use += align256(bytes);
    S.geom_bytes += align256(bytes);
    for (int k = 0; k < DMIMO_K_MAX; ++k) S.pa_gamma[k] = gamma_lin;
    S.pa_lam = dev;
    S.pa_eta = dev + layers;
    S.pa_layers = layers;
    return DMIMO_OK;
}

dmimo_status dmimo_server_poll(dmimo_server* srv, uint64_t ticket, int32_t* state,
                               double* t_submit, double* t_done) {
    clear_error();
    if (!srv || !state) return fail(DMIMO_E_ARG, "poll: NULL argument");
    ServerImpl& S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return fail(DMIMO_E_NOTFOUND, "poll: unknown ticket");
    *state = it->second->state.load();
    if (t_submit) *t_submit = it->second->t_submit;
    if (t_done) *t_done = it->second->t_done;
    return DMIMO_OK;
}

dmimo_status dmimo_server_wait(dmimo_server* srv, uint64_t ticket, double timeout_s,
                               int32_t* state) {
    clear_error();
    if (!srv || !state) return fail(DMIMO_E_ARG, "wait: NULL argument");
    ServerImpl& S = srv->impl;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return fail(DMIMO_E_NOTFOUND, "wait: unknown ticket");
    Query* q = it->second;
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::microseconds((int64_t)(std::max(0.0, timeout_s) * 1e6));
    S.cv.wait_until(lk, until, [q] { return q->state.load() >= kDone; });
    *state = q->state.load();
    return DMIMO_OK;
}

dmimo_status dmimo_server_cancel(dmimo_server* srv, uint64_t ticket) {
    clear_error();
    if (!srv) return fail(DMIMO_E_ARG, "cancel: NULL server");
    ServerImpl& S = srv->impl;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        auto it = S.all.find(ticket);
        if (it == S.all.end()) return fail(DMIMO_E_NOTFOUND, "cancel: unknown ticket");
        Query* q = it->second;
        auto pos = std::find(S.pending.begin(), S.pending.end(), q);
        if (pos == S.pending.end())
            return fail(DMIMO_E_BUSY, "cancel: the query was admitted already (or is finished)");
        S.pending.erase(pos);
        q->t_done = now_s();
        q->state.store(kCancelled);
    }
    S.cv.notify_all();
    return DMIMO_OK;
}

dmimo_status dmimo_server_set_queue_timeout(dmimo_server* srv, double seconds) {
    clear_error();
    if (!srv) return fail(DMIMO_E_ARG, "set_queue_timeout: NULL server");
    if (!(seconds >= 0.0) || !std::isfinite(seconds))
        return fail(DMIMO_E_ARG, "set_queue_timeout: seconds must be >= 0");
    ServerImpl& S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    S.queue_timeout = seconds;
    return DMIMO_OK;
}

dmimo_status dmimo_server_query_info(dmimo_server* srv, uint64_t ticket, int32_t* info) {
    clear_error();
    if (!srv || !info) return fail(DMIMO_E_ARG, "query_info: NULL argument");
    ServerImpl& S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return fail(DMIMO_E_NOTFOUND, "query_info: unknown ticket");
    *info = it->second->state.load() >= kDone ? it->second->info : 0;
    return DMIMO_OK;
}

dmimo_status dmimo_server_release(dmimo_server* srv, uint64_t ticket) {
    clear_error();
    if (!srv) return fail(DMIMO_E_ARG, "release: NULL server");
    ServerImpl& S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.all.find(ticket);
    if (it == S.all.end()) return fail(DMIMO_E_NOTFOUND, "release: unknown ticket");
    if (it->second->state.load() < kDone) return fail(DMIMO_E_BUSY, "release: query not finished");
    delete it->second;
    S.all.erase(it);
    return DMIMO_OK;
}

dmimo_status dmimo_server_stats(dmimo_server* srv, int64_t* completed, int64_t* terms,
                                int64_t* ticks, int32_t* queued, int32_t* running) {
    clear_error();
    if (!srv) return fail(DMIMO_E_ARG, "stats: NULL server");
    ServerImpl& S = srv->impl;
    std::lock_guard<std::mutex> lk(S.mu);
    if (completed) *completed = S.n_done.load();
    if (terms) *terms = S.terms_done.load();
    if (ticks) *ticks = S.ticks_issued;
    if (queued) *queued = (int32_t)S.pending.size();
    if (running) *running = (int32_t)S.active.size();
    return DMIMO_OK;
}

dmimo_status dmimo_server_destroy(dmimo_server* srv) {
    clear_error();
    if (!srv) return DMIMO_OK;
    ServerImpl& S = srv->impl;
    if (S.worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S.mu);
            S.stop.store(true);
        }
        S.cv.notify_all();
        S.worker.join();
    }
    if (S.stream) hipStreamSynchronize(S.stream);
    for (int i = 0; i < 2; ++i) {
        if (S.ev[i]) hipEventDestroy(S.ev[i]);
        if (S.d_items[i]) hipFree(S.d_items[i]);
        if (S.h_items[i]) hipHostFree(S.h_items[i]);
    }
    if (S.h_users) hipHostFree(S.h_users);
    if (S.h_info) hipHostFree(S.h_info);
    if (S.h_slots) hipHostFree(S.h_slots);
    if (S.d_slots) hipFree(S.d_slots);
    if (S.arena_base) hipFree(S.arena_base);
    if (S.stream) hipStreamDestroy(S.stream);
    for (auto& kv : S.all) delete kv.second;   // pending and active queries are in `all`
    delete srv;
    return DMIMO_OK;
}

}  // extern "C"
