// Host side of the C ABI: argument validation, error state and dispatch.
// Every check here runs before the first HIP runtime call of an entry point,
// so argument errors are reported without touching the GPU.
#include <cmath>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <mutex>

#include "dmimo_internal.h"
#include "kernels.h"

namespace dmimo {

static thread_local char g_last_error[512] = {0};

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_last_error[0] = 0; }

dmimo_status check_launch(const char* kernel) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", kernel, hipGetErrorString(e));
        return DMIMO_E_HIP;
    }
    return DMIMO_OK;
}

dmimo_status make_wave_const(const dmimo_channel_params* p, WaveConst* out) {
    if (!p) return fail(DMIMO_E_ARG, "channel params: NULL");
    if (!(p->freq_hz > 0.0) || !std::isfinite(p->freq_hz))
        return fail(DMIMO_E_ARG, "channel params: freq_hz must be > 0");
    if (p->model != DMIMO_CH_LOS && p->model != DMIMO_CH_RICIAN)
        return fail(DMIMO_E_DTYPE, "channel params: unknown channel model");
    if (p->model == DMIMO_CH_RICIAN && !(p->kappa_lin >= 0.0))
        return fail(DMIMO_E_ARG, "channel params: kappa_lin must be >= 0");
    const double lam = kSpeedOfLight / p->freq_hz;
    const double dmin = p->d_min_m > 0.0 ? p->d_min_m : lam / (4.0 * kPi);
    out->inv_lam = 1.0 / lam;
    out->amp_c = lam / (4.0 * kPi);
    out->inv_dmin = 1.0 / dmin;
    if (p->model == DMIMO_CH_RICIAN) {
        const double k = p->kappa_lin;
        out->a_los = std::sqrt(k / (1.0 + k));
        out->a_nlos = std::sqrt(1.0 / (1.0 + k));
    } else {
        out->a_los = 1.0;
        out->a_nlos = 0.0;
    }
    return DMIMO_OK;
}

dmimo_status make_points(const dmimo_points* p, PointsDev* out) {
    if (!p) return fail(DMIMO_E_ARG, "points: NULL descriptor");
    out->kind = p->kind;
    out->nx = p->nx;
    out->ny = p->ny;
    out->x0 = p->x0;
    out->y0 = p->y0;
    out->dx = p->dx;
    out->dy = p->dy;
    out->z = p->z;
    out->xyz = p->xyz;
    if (p->kind == DMIMO_PTS_GRID) {
        if (p->nx < 0 || p->ny < 0) return fail(DMIMO_E_SHAPE, "points: grid nx, ny must be >= 0");
        if (!std::isfinite(p->x0) || !std::isfinite(p->y0) || !std::isfinite(p->dx) ||
            !std::isfinite(p->dy) || !std::isfinite(p->z))
            return fail(DMIMO_E_ARG, "points: grid origin / pitch / height must be finite");
        out->n = (int64_t)p->nx * (int64_t)p->ny;
        out->xyz = nullptr;
    } else if (p->kind == DMIMO_PTS_LIST) {
        if (p->n < 0) return fail(DMIMO_E_SHAPE, "points: list n must be >= 0");
        if (p->n > 0 && !p->xyz) return fail(DMIMO_E_ARG, "points: list xyz is NULL");
        out->n = p->n;
    } else {
        return fail(DMIMO_E_DTYPE, "points: unknown kind");
    }
    return DMIMO_OK;
}

static bool valid_prec(int32_t p) { return p >= DMIMO_F64 && p <= DMIMO_MIX_BF16X3; }

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static dmimo_status check_ufpgd_common(const char* who, int32_t K, int32_t M, int32_t layers,
                                const double* gamma_lin, double sigma2, double lam_c, int32_t prec) {
    char msg[160];
    if (K < 1 || M < 1 || layers < 0) {
        std::snprintf(msg, sizeof msg, "%s: K, M must be >= 1 and layers >= 0", who);
        return fail(DMIMO_E_SHAPE, msg);
    }
    if (M > 256 || K > 16) {
        std::snprintf(msg, sizeof msg, "%s: K <= 8 and M <= 256", who);
        return fail(DMIMO_E_SHAPE, msg);
    }
    if (K > 8) {
        std::snprintf(msg, sizeof msg, "%s: training is provided for K <= 8", who);
        return fail(DMIMO_E_UNSUPPORTED, msg);
    }
    if (!valid_prec(prec)) {
        std::snprintf(msg, sizeof msg, "%s: unknown precision", who);
        return fail(DMIMO_E_DTYPE, msg);
    }
    if (prec != DMIMO_F32) {
        std::snprintf(msg, sizeof msg, "%s: FP32 only", who);
        return fail(DMIMO_E_UNSUPPORTED, msg);
    }
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2) || !(lam_c >= 0.0) || !std::isfinite(lam_c)) {
        std::snprintf(msg, sizeof msg, "%s: sigma2 and lam_c must be finite and >= 0", who);
        return fail(DMIMO_E_ARG, msg);
    }
    for (int k = 0; gamma_lin && k < K; ++k)
        if (!(gamma_lin[k] >= 0.0) || !std::isfinite(gamma_lin[k])) {
            std::snprintf(msg, sizeof msg, "%s: gamma_lin must be finite and >= 0", who);
            return fail(DMIMO_E_ARG, msg);
        }
    return DMIMO_OK;
}

}  // namespace dmimo

using namespace dmimo;

extern "C" {

const char* dmimo_version(void) { return "dmimo 0.1 (gfx950)"; }

const char* dmimo_status_string(int32_t s) {
    switch (s) {
        case DMIMO_OK: return "ok";
        case DMIMO_E_ARG: return "invalid argument";
        case DMIMO_E_SHAPE: return "invalid shape";
        case DMIMO_E_DTYPE: return "invalid precision / model / kind";
        case DMIMO_E_WORKSPACE: return "workspace too small";
        case DMIMO_E_HIP: return "HIP runtime error";
        case DMIMO_E_UNSUPPORTED: return "unsupported combination";
        case DMIMO_E_BUSY: return "busy";
        case DMIMO_E_NOMEM: return "does not fit the memory budget";
        case DMIMO_E_NOTFOUND: return "not found";
        default: return "unknown status";
    }
}

const char* dmimo_last_error(void) { return g_last_error; }

size_t dmimo_workspace_size(int32_t call, int32_t B, int32_t K, int32_t M, int32_t N,
                            int32_t prec) {
    (void)M;
    (void)N;
    if (B <= 0 || K <= 0) return 0;
    switch (call) {
        case DMIMO_CALL_BEAMFORM_ZF:
            return beamform_workspace_bytes(DMIMO_ZF, B, K, M, prec);
        case DMIMO_CALL_BEAMFORM_MR:
            return beamform_workspace_bytes(DMIMO_MR, B, K, M, prec);
        case DMIMO_CALL_PA_PRECODER: {
            if (K > 32 || M < 1 || M > 4096) return 0;
            const size_t f = align256((size_t)B * 2 * sizeof(double));
            return (K > 16 || M > 256) ? f + align256(pa_large_workspace_bytes(B, K, M)) : f;
        }
        default:
            return 0;
    }
}

dmimo_status dmimo_channel(const dmimo_channel_params* params, int32_t B, int32_t M,
                           const double* ap_xyz, const dmimo_points* pts, const void* nlos,
                           int32_t out, void* H, void* stream) {
    clear_error();
    WaveConst w;
    dmimo_status st = make_wave_const(params, &w);
    if (st) return st;
    PointsDev P;
    if ((st = make_points(pts, &P))) return st;
    if (B < 0) return fail(DMIMO_E_SHAPE, "channel: B must be >= 0");
    if (M < 1) return fail(DMIMO_E_SHAPE, "channel: M must be >= 1");
    if (!valid_prec(out)) return fail(DMIMO_E_DTYPE, "channel: unknown precision");
    if (out != DMIMO_F64 && out != DMIMO_F32)
        return fail(DMIMO_E_UNSUPPORTED, "channel: output must be DMIMO_F64 or DMIMO_F32");
    if (params->model == DMIMO_CH_RICIAN && !nlos && B > 0 && P.n > 0)
        return fail(DMIMO_E_ARG, "channel: Rician model needs the nlos draws");
    if (B == 0 || P.n == 0) return DMIMO_OK;
    if (!ap_xyz || !H) return fail(DMIMO_E_ARG, "channel: NULL ap_xyz or H");
    return launch_channel(w, P, params->model == DMIMO_CH_RICIAN, B, M, ap_xyz,
                          nlos, out == DMIMO_F64, H, as_stream(stream));
}

dmimo_status dmimo_gram(int32_t B, int32_t K, int32_t M, const void* H, int32_t prec,
                        void* G, void* stream) {
    clear_error();
    if (B < 0) return fail(DMIMO_E_SHAPE, "gram: B must be >= 0");
    if (K < 1 || M < 1) return fail(DMIMO_E_SHAPE, "gram: K and M must be >= 1");
    if (K > DMIMO_K_MAX) return fail(DMIMO_E_SHAPE, "gram: K exceeds DMIMO_K_MAX");
    if (!valid_prec(prec)) return fail(DMIMO_E_DTYPE, "gram: unknown precision");
    if (B == 0) return DMIMO_OK;
    if (!H || !G) return fail(DMIMO_E_ARG, "gram: NULL H or G");
    return launch_gram(B, K, M, H, prec, G, as_stream(stream));
}

namespace {

// Argument checks shared by the beamform calls; fills gam with the targets.
dmimo_status check_beamform(int32_t precoder, int32_t B, int32_t K, int32_t M, double sigma2,
                            double p_total, int32_t prec, const double* sinr_or_rsum,
                            const double* gamma_lin, double* gam) {
    if (precoder != DMIMO_MR && precoder != DMIMO_ZF && precoder != DMIMO_MR_PHASE)
        return fail(DMIMO_E_DTYPE, "beamform: unknown precoder");
    if (B < 0) return fail(DMIMO_E_SHAPE, "beamform: B must be >= 0");
    if (K < 1 || M < 1) return fail(DMIMO_E_SHAPE, "beamform: K and M must be >= 1");
    if (K > DMIMO_K_MAX) return fail(DMIMO_E_SHAPE, "beamform: K exceeds DMIMO_K_MAX");
    if (precoder == DMIMO_ZF && K > M)
        return fail(DMIMO_E_SHAPE, "beamform: ZF needs K <= M");
    if (!valid_prec(prec)) return fail(DMIMO_E_DTYPE, "beamform: unknown precision");
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2))
        return fail(DMIMO_E_ARG, "beamform: sigma2 must be >= 0");
    if (!std::isfinite(p_total)) return fail(DMIMO_E_ARG, "beamform: p_total must be finite");
    if (sinr_or_rsum && !(sigma2 > 0.0))
        return fail(DMIMO_E_ARG, "beamform: SINR outputs need sigma2 > 0");
    for (int k = 0; k < K; ++k) {
        gam[k] = gamma_lin ? gamma_lin[k] : 1.0;
        if (!(gam[k] >= 0.0) || !std::isfinite(gam[k]))
            return fail(DMIMO_E_ARG, "beamform: gamma_lin must be finite and >= 0");
    }
    return DMIMO_OK;
}

BeamformArgs beamform_args(int32_t precoder, int32_t B, int32_t K, int32_t M, const void* H,
                           const double* gam, double sigma2, double p_total, int32_t prec,
                           void* W, double* p_ant, double* l21, double* sinr, double* rsum,
                           int32_t* info, void* ws) {
    BeamformArgs a;
    a.precoder = precoder;
    a.B = B;
    a.K = K;
    a.M = M;
    a.H = H;
    for (int k = 0; k < DMIMO_K_MAX; ++k) a.gamma[k] = k < K ? gam[k] : 0.0;
    a.sigma2 = sigma2;
    a.p_total = p_total;
    a.prec = prec;
    a.W = W;
    a.p_ant = p_ant;
    a.l21 = l21;
    a.sinr = sinr;
    a.rsum = rsum;
    a.info = info;
    a.ws = ws;
    return a;
}

}  // namespace

dmimo_status dmimo_beamform(int32_t precoder, int32_t B, int32_t K, int32_t M, const void* H,
                            const double* gamma_lin, double sigma2, double p_total,
                            int32_t prec, void* W, double* p_ant, double* l21, double* sinr,
                            double* rsum, int32_t* info, void* ws, size_t ws_bytes,
                            void* stream) {
    clear_error();
    double gam[DMIMO_K_MAX];
    dmimo_status st = check_beamform(precoder, B, K, M, sigma2, p_total, prec,
                                     sinr ? sinr : rsum, gamma_lin, gam);
    if (st) return st;
    const size_t need = dmimo_workspace_size(
        precoder == DMIMO_ZF ? DMIMO_CALL_BEAMFORM_ZF : DMIMO_CALL_BEAMFORM_MR, B, K, M, 0, prec);
    if (B == 0) return DMIMO_OK;
    if (!H || !W) return fail(DMIMO_E_ARG, "beamform: NULL H or W");
    if (need > 0 && (!ws || ws_bytes < need)) {
        set_error("beamform: workspace needs %zu bytes, got %zu", need, ws ? ws_bytes : 0);
        return DMIMO_E_WORKSPACE;
    }
    return launch_beamform(beamform_args(precoder, B, K, M, H, gam, sigma2, p_total, prec, W, p_ant,
                                         l21, sinr, rsum, info, ws),
                           as_stream(stream));
}

dmimo_status dmimo_beamform_batched(int32_t precoder, const dmimo_channel_params* params,
                                    int32_t B, int32_t K, int32_t M, const double* ap_xyz,
                                    const double* user_xyz, const void* nlos,
                                    const double* gamma_lin, double sigma2, double p_total,
                                    int32_t prec, void* H, void* W, double* p_ant, double* l21,
                                    double* sinr, double* rsum, int32_t* info, void* stream) {
    clear_error();
    WaveConst w;
    dmimo_status st = make_wave_const(params, &w);
    if (st) return st;
    if (precoder != DMIMO_MR && precoder != DMIMO_ZF)
        return fail(DMIMO_E_UNSUPPORTED, "beamform_batched: MR or ZF");
    if ((params->model == DMIMO_CH_RICIAN) != (nlos != nullptr))
        return fail(DMIMO_E_ARG, "beamform_batched: nlos is required for Rician and only for it");
    double gam[DMIMO_K_MAX];
    st = check_beamform(precoder, B, K, M, sigma2, p_total, prec, sinr ? sinr : rsum, gamma_lin, gam);
    if (st) return st;
    if (prec == DMIMO_F64) return fail(DMIMO_E_UNSUPPORTED, "beamform_batched: FP32 or MIX precision");
    if (K > 16 || M > 256)
        return fail(DMIMO_E_UNSUPPORTED, "beamform_batched: K <= 16 and M <= 256 "
                                         "(dmimo_channel + dmimo_beamform serve larger deployments)");
    if (B == 0) return DMIMO_OK;
    if (!ap_xyz || !user_xyz) return fail(DMIMO_E_ARG, "beamform_batched: NULL positions");
    return launch_beamform_batched(beamform_args(precoder, B, K, M, nullptr, gam, sigma2, p_total,
                                                 prec, W, p_ant, l21, sinr, rsum, info, nullptr),
                                   w, ap_xyz, user_xyz, nlos, H, as_stream(stream));
}

// ---------------------------------------------------------------------------
// dmimo_beamform_noalloc: the scratch of dmimo_beamform in a static device array
// ---------------------------------------------------------------------------
//
// Each GPU that runs the library holds its own copy of `scratch` until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it only stands for the symbol): its device address is looked up once
// per device with hipGetSymbolAddress, with that device current, and that
// address is what the kernels receive.  Every call on a device shares the
// array, so calls that overlap on one device (different streams, or threads)
// race; the kernels write every byte of the scratch they read, so no call
// depends on what an earlier one left there.

static __device__ __align__(256) char scratch[DMIMO_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the device that `stream` belongs to (the
// current device for the NULL stream).
dmimo_status scratch_address(hipStream_t stream, void** out) {
    int dev = 0;
    hipError_t e = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("beamform_noalloc: device of the stream: %s", hipGetErrorString(e));
        return DMIMO_E_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(DMIMO_E_UNSUPPORTED, "beamform_noalloc: device index");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        if ((e = hipGetDevice(&cur)) == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess || !p) {
            set_error("beamform_noalloc: scratch address: %s", hipGetErrorString(e));
            return DMIMO_E_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return DMIMO_OK;
}

}  // namespace

dmimo_status dmimo_beamform_noalloc(int32_t precoder, int32_t B, int32_t K, int32_t M,
                                    const void* H, const double* gamma_lin, double sigma2,
                                    double p_total, int32_t prec, void* W, double* p_ant,
                                    double* l21, double* sinr, double* rsum, int32_t* info,
                                    void* stream) {
    clear_error();
    double gam[DMIMO_K_MAX];
    dmimo_status st = check_beamform(precoder, B, K, M, sigma2, p_total, prec,
                                     sinr ? sinr : rsum, gamma_lin, gam);
    if (st) return st;
    const size_t need = dmimo_workspace_size(
        precoder == DMIMO_ZF ? DMIMO_CALL_BEAMFORM_ZF : DMIMO_CALL_BEAMFORM_MR, B, K, M, 0, prec);
    if (need > (size_t)DMIMO_NOALLOC_SCRATCH_BYTES) {
        set_error("beamform_noalloc: the call needs %zu bytes of scratch, more than the %d bytes "
                  "of the static array (use dmimo_beamform with a workspace)",
                  need, DMIMO_NOALLOC_SCRATCH_BYTES);
        return DMIMO_E_WORKSPACE;
    }
    if (B == 0) return DMIMO_OK;
    if (!H || !W) return fail(DMIMO_E_ARG, "beamform_noalloc: NULL H or W");
    void* ws = nullptr;
    if (need > 0 && (st = scratch_address(as_stream(stream), &ws))) return st;
    return launch_beamform(beamform_args(precoder, B, K, M, H, gam, sigma2, p_total, prec, W, p_ant,
                                         l21, sinr, rsum, info, ws),
                           as_stream(stream));
}

dmimo_status dmimo_beamform_multi(int32_t P, const int32_t* precoders, int32_t B, int32_t K,
                                  int32_t M, const void* H, const double* gamma_lin,
                                  double sigma2, double p_total, int32_t prec, void* W,
                                  double* p_ant, double* l21, double* sinr, double* rsum,
                                  int32_t* info, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (P < 0 || P > 8) return fail(DMIMO_E_SHAPE, "beamform_multi: 0 <= P <= 8");
    if (P > 0 && !precoders) return fail(DMIMO_E_ARG, "beamform_multi: NULL precoders");
    double gam[DMIMO_K_MAX];
    for (int i = 0; i < P; ++i) {
        dmimo_status st = check_beamform(precoders[i], B, K, M, sigma2, p_total, prec,
                                         sinr ? sinr : rsum, gamma_lin, gam);
        if (st) return st;
    }
    if (P == 0 || B == 0) return DMIMO_OK;
    if (!H || !W) return fail(DMIMO_E_ARG, "beamform_multi: NULL H or W");
    const size_t need = dmimo_beamform_multi_workspace_size(P, precoders, B, K, M, prec);
    if (need > 0 && (!ws || ws_bytes < need)) {
        set_error("beamform_multi: workspace needs %zu bytes, got %zu", need, ws ? ws_bytes : 0);
        return DMIMO_E_WORKSPACE;
    }
    return launch_beamform_multi(beamform_args(precoders[0], B, K, M, H, gam, sigma2, p_total,
                                               prec, W, p_ant, l21, sinr, rsum, info, ws),
                                 P, precoders, as_stream(stream));
}

dmimo_status dmimo_beamform_users(int32_t P, const int32_t* precoders,
                                  const dmimo_channel_params* params, int32_t B, int32_t K,
                                  int32_t M, const double* ap_xyz, const double* user_xyz,
                                  const double* gamma_lin, double sigma2, double p_total,
                                  int32_t prec, void* H, void* W, double* p_ant, double* l21,
                                  double* sinr, double* rsum, int32_t* info, void* ws,
                                  size_t ws_bytes, void* stream) {
    clear_error();
    WaveConst w;
    dmimo_status st = make_wave_const(params, &w);
    if (st) return st;
    if (params->model != DMIMO_CH_LOS)
        return fail(DMIMO_E_UNSUPPORTED, "beamform_users: LoS channel model only");
    if (P < 0 || P > 8) return fail(DMIMO_E_SHAPE, "beamform_users: 0 <= P <= 8");
    if (P > 0 && !precoders) return fail(DMIMO_E_ARG, "beamform_users: NULL precoders");
    double gam[DMIMO_K_MAX];
    for (int i = 0; i < P; ++i) {
        st = check_beamform(precoders[i], B, K, M, sigma2, p_total, prec, sinr ? sinr : rsum,
                            gamma_lin, gam);
        if (st) return st;
    }
    if (P == 0 || B == 0) return DMIMO_OK;
    if (!ap_xyz || !user_xyz) return fail(DMIMO_E_ARG, "beamform_users: NULL ap_xyz or user_xyz");
    if (!H || !W) return fail(DMIMO_E_ARG, "beamform_users: NULL H or W");
    const size_t need = dmimo_beamform_multi_workspace_size(P, precoders, B, K, M, prec);
    if (need > 0 && (!ws || ws_bytes < need)) {
        set_error("beamform_users: workspace needs %zu bytes, got %zu", need, ws ? ws_bytes : 0);
        return DMIMO_E_WORKSPACE;
    }
    return launch_beamform_users(beamform_args(precoders[0], B, K, M, H, gam, sigma2, p_total,
                                               prec, W, p_ant, l21, sinr, rsum, info, ws),
                                 P, precoders, w, ap_xyz, user_xyz, as_stream(stream));
}

size_t dmimo_beamform_multi_workspace_size(int32_t P, const int32_t* precoders, int32_t B,
                                           int32_t K, int32_t M, int32_t prec) {
    if (P < 1 || P > 8 || !precoders || B <= 0 || K <= 0 || M <= 0) return 0;
    for (int i = 0; i < P; ++i)
        if (precoders[i] != DMIMO_MR && precoders[i] != DMIMO_ZF && precoders[i] != DMIMO_MR_PHASE)
            return 0;
    return beamform_multi_workspace_bytes(P, precoders, B, K, M, prec);
}

namespace {

dmimo_status powermap_maps(const dmimo_channel_params* params, int32_t M, const double* ap_xyz,
                           int32_t maps, int32_t K, const void* W, const dmimo_points* pts,
                           double sigma2, int32_t prec, void* power, void* sinr, int32_t* best_k,
                           void* per_stream, void* stream) {
    clear_error();
    WaveConst w;
    dmimo_status st = make_wave_const(params, &w);
    if (st) return st;
    if (params->model != DMIMO_CH_LOS)
        return fail(DMIMO_E_UNSUPPORTED, "powermap: only the LoS model is mapped");
    PointsDev P;
    if ((st = make_points(pts, &P))) return st;
    if (maps < 0 || maps > 65535) return fail(DMIMO_E_SHAPE, "powermap: 0 <= maps <= 65535");
    if (M < 1 || K < 1) return fail(DMIMO_E_SHAPE, "powermap: K and M must be >= 1");
    if (K > DMIMO_K_MAX) return fail(DMIMO_E_SHAPE, "powermap: K exceeds DMIMO_K_MAX");
    if (!valid_prec(prec)) return fail(DMIMO_E_DTYPE, "powermap: unknown precision");
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2))
        return fail(DMIMO_E_ARG, "powermap: sigma2 must be >= 0");
    if (sinr && !(sigma2 > 0.0)) return fail(DMIMO_E_ARG, "powermap: SINR map needs sigma2 > 0");
    if (P.n > (int64_t)INT32_MAX * 8) return fail(DMIMO_E_SHAPE, "powermap: too many points");
    if (P.n == 0 || maps == 0) return DMIMO_OK;
    if (!ap_xyz || !W || !power) return fail(DMIMO_E_ARG, "powermap: NULL ap_xyz, W or power");
    PowermapArgs a;
    a.w = w;
    a.P = P;
    a.M = M;
    a.K = K;
    a.maps = maps;
    a.ap = ap_xyz;
    a.W = W;
    a.sigma2 = sigma2;
    a.prec = prec;
    a.power = power;
    a.sinr = sinr;
    a.best_k = best_k;
    a.per_stream = per_stream;
    return launch_powermap(a, as_stream(stream));
}

}  // namespace

dmimo_status dmimo_powermap(const dmimo_channel_params* params, int32_t M, const double* ap_xyz,
                            int32_t K, const void* W, const dmimo_points* pts, double sigma2,
                            int32_t prec, void* power, void* sinr, int32_t* best_k,
                            void* per_stream, void* stream) {
    return powermap_maps(params, M, ap_xyz, 1, K, W, pts, sigma2, prec, power, sinr, best_k,
                         per_stream, stream);
}

dmimo_status dmimo_powermap_batch(const dmimo_channel_params* params, int32_t M,
                                  const double* ap_xyz, int32_t maps, int32_t K, const void* W,
                                  const dmimo_points* pts, double sigma2, int32_t prec,
                                  void* power, void* sinr, int32_t* best_k, void* per_stream,
                                  void* stream) {
    return powermap_maps(params, M, ap_xyz, maps, K, W, pts, sigma2, prec, power, sinr, best_k,
                         per_stream, stream);
}

dmimo_status dmimo_pgd(int32_t B, int32_t K, int32_t M, const void* H, const double* gamma_lin,
                       double sigma2, int32_t layers, const double* lambdas, const double* etas,
                       const void* W0, int32_t prec, void* W, double* l21, double* rsum,
                       void* stream) {
    clear_error();
    if (B < 0 || layers < 0) return fail(DMIMO_E_SHAPE, "pgd: B and layers must be >= 0");
    if (K < 1 || M < 1) return fail(DMIMO_E_SHAPE, "pgd: K and M must be >= 1");
    if (K > 16 || M > 256) return fail(DMIMO_E_SHAPE, "pgd: K <= 16 and M <= 256");
    if (!valid_prec(prec)) return fail(DMIMO_E_DTYPE, "pgd: unknown precision");
    if (prec != DMIMO_F32 && !(prec == DMIMO_MIX_BF16X3 && K <= 8))
        return fail(DMIMO_E_UNSUPPORTED, "pgd: FP32, or BF16x3 for K <= 8");
    if (!(sigma2 >= 0.0) || !std::isfinite(sigma2)) return fail(DMIMO_E_ARG, "pgd: sigma2 must be >= 0");
    if (rsum && !(sigma2 > 0.0)) return fail(DMIMO_E_ARG, "pgd: the sum rate needs sigma2 > 0");
    for (int k = 0; gamma_lin && k < K; ++k)
        if (!(gamma_lin[k] >= 0.0) || !std::isfinite(gamma_lin[k]))
            return fail(DMIMO_E_ARG, "pgd: gamma_lin must be finite and >= 0");
    if (B == 0) return DMIMO_OK;
    if (!H || !W) return fail(DMIMO_E_ARG, "pgd: NULL H or W");
    if (layers > 0 && (!lambdas || !etas)) return fail(DMIMO_E_ARG, "pgd: NULL lambdas or etas");
    return launch_pgd(B, K, M, H, gamma_lin, sigma2, layers, lambdas, etas, W0, W, l21, rsum, prec,
                      as_stream(stream));
}

dmimo_status dmimo_pa_precoder(int32_t B, int32_t K, int32_t M, const void* H,
                               const double* gamma_lin, double sigma2, int32_t layers,
                               const double* lambdas, const double* eta_rel, int32_t prec,
                               void* W, double* p_ant, double* l21, double* sinr, double* rsum,
                               void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (B < 0 || layers < 0) return fail(DMIMO_E_SHAPE, "pa_precoder: B and layers must be >= 0");
    if (K < 1 || M < 1) return fail(DMIMO_E_SHAPE, "pa_precoder: K and M must be >= 1");
    if (K > 32 || M > 4096) return fail(DMIMO_E_SHAPE, "pa_precoder: K <= 32 and M <= 4096");
    if (!valid_prec(prec)) return fail(DMIMO_E_DTYPE, "pa_precoder: unknown precision");
    if (prec != DMIMO_F32 && !(prec == DMIMO_MIX_BF16X3 && K <= 8 && M <= 256))
        return fail(DMIMO_E_UNSUPPORTED, "pa_precoder: FP32, or BF16x3 for K <= 8 and M <= 256");
    if (!(sigma2 > 0.0) || !std::isfinite(sigma2)) return fail(DMIMO_E_ARG, "pa_precoder: sigma2 must be > 0");
    for (int k = 0; gamma_lin && k < K; ++k)
        if (!(gamma_lin[k] >= 0.0) || !std::isfinite(gamma_lin[k]))
            return fail(DMIMO_E_ARG, "pa_precoder: gamma_lin must be finite and >= 0");
    if (B == 0) return DMIMO_OK;
    if (!H || !W) return fail(DMIMO_E_ARG, "pa_precoder: NULL H or W");
    if (layers > 0 && (!lambdas || !eta_rel)) return fail(DMIMO_E_ARG, "pa_precoder: NULL lambdas or eta_rel");
    if (!ws || ws_bytes < dmimo_workspace_size(DMIMO_CALL_PA_PRECODER, B, K, M, 0, prec))
        return fail(DMIMO_E_WORKSPACE, "pa_precoder: workspace smaller than dmimo_workspace_size()");
    if (K > 16 || M > 256)
        return launch_pa_large(B, K, M, H, gamma_lin, sigma2, layers, lambdas, eta_rel, W, p_ant,
                               l21, sinr, rsum, ws, align256((size_t)B * 2 * sizeof(double)),
                               as_stream(stream));
    return launch_pa_precoder(B, K, M, H, gamma_lin, sigma2, layers, lambdas, eta_rel, W, p_ant,
                              l21, sinr, rsum, ws, prec, as_stream(stream));
}

size_t dmimo_ufpgd_workspace_size(int32_t B, int32_t K, int32_t M, int32_t layers) {
    if (B < 1 || K < 1 || K > 8 || M < 1 || M > 256 || layers < 0) return 0;
    return ufpgd_workspace_bytes(B, M, layers);
}

dmimo_status dmimo_ufpgd_grad(int32_t B, int32_t n_channels, int32_t K, int32_t M, const void* H,
                              const int32_t* idx, const double* gamma_lin, double sigma2,
                              double lam_c, int32_t layers, const double* lambdas,
                              const double* etas, int32_t prec, double* cost, double* dlam,
                              double* deta, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (B < 0 || n_channels < 0) return fail(DMIMO_E_SHAPE, "ufpgd_grad: B and n_channels must be >= 0");
    dmimo_status st = check_ufpgd_common("ufpgd_grad", K, M, layers, gamma_lin, sigma2, lam_c, prec);
    if (st) return st;
    if (!idx && n_channels < B) return fail(DMIMO_E_SHAPE, "ufpgd_grad: without idx, n_channels >= B");
    if ((dlam == nullptr) != (deta == nullptr))
        return fail(DMIMO_E_ARG, "ufpgd_grad: give both dlam and deta, or neither");
    if (B == 0) return DMIMO_OK;
    if (!H) return fail(DMIMO_E_ARG, "ufpgd_grad: NULL H");
    if (!cost && !dlam) return fail(DMIMO_E_ARG, "ufpgd_grad: nothing to compute");
    if (layers > 0 && (!lambdas || !etas)) return fail(DMIMO_E_ARG, "ufpgd_grad: NULL lambdas or etas");
    if (dlam && (!ws || ws_bytes < ufpgd_workspace_bytes(B, M, layers)))
        return fail(DMIMO_E_WORKSPACE, "ufpgd_grad: workspace smaller than dmimo_ufpgd_workspace_size()");
    UfpgdArgs g{B, K, M, layers, n_channels, H, idx, gamma_lin, sigma2, lam_c, lambdas, etas};
    return launch_ufpgd_grad(g, cost, dlam, deta, ws, as_stream(stream));
}

dmimo_status dmimo_ufpgd_train(int32_t n_channels, int32_t K, int32_t M, const void* H,
                               const double* gamma_lin, double sigma2, double lam_c,
                               int32_t layers, double* lambdas, double* etas, double* adam_m,
                               double* adam_v, int64_t t0, const dmimo_adam_params* opt,
                               int32_t batch, int32_t steps, const int32_t* idx,
                               double* batch_cost, int32_t prec, void* ws, size_t ws_bytes,
                               void* stream) {
    clear_error();
    dmimo_status st = check_ufpgd_common("ufpgd_train", K, M, layers, gamma_lin, sigma2, lam_c, prec);
    if (st) return st;
    if (n_channels < 1 || batch < 1 || steps < 0 || layers < 1 || t0 < 0)
        return fail(DMIMO_E_SHAPE, "ufpgd_train: n_channels, batch, layers >= 1; steps, t0 >= 0");
    if (!opt) return fail(DMIMO_E_ARG, "ufpgd_train: NULL optimiser parameters");
    if (!(opt->lr > 0.0) || !std::isfinite(opt->lr) || !(opt->beta1 >= 0.0 && opt->beta1 < 1.0) ||
        !(opt->beta2 >= 0.0 && opt->beta2 < 1.0) || !(opt->eps > 0.0) || !std::isfinite(opt->eps))
        return fail(DMIMO_E_ARG, "ufpgd_train: lr > 0, 0 <= beta < 1, eps > 0");
    if (steps == 0) return DMIMO_OK;
    if (!H || !lambdas || !etas || !adam_m || !adam_v || !idx)
        return fail(DMIMO_E_ARG, "ufpgd_train: NULL H, parameters, Adam moments or idx");
    if (!ws || ws_bytes < ufpgd_workspace_bytes(batch, M, layers))
        return fail(DMIMO_E_WORKSPACE, "ufpgd_train: workspace smaller than dmimo_ufpgd_workspace_size()");
    UfpgdArgs g{batch, K, M, layers, n_channels, H, nullptr, gamma_lin, sigma2, lam_c, lambdas, etas};
    UfpgdTrainArgs t{lambdas, etas, adam_m, adam_v, t0, opt->lr, opt->beta1, opt->beta2, opt->eps,
                     steps, idx, batch_cost};
    return launch_ufpgd_train(g, t, ws, as_stream(stream));
}

}  // extern "C"
