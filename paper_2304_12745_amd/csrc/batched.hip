// Users' channels, precoder and epilogues of many small deployments in one
// launch (K <= 16 users, M <= 256 antennas): the batched workload of
// independent rooms with LoS or Rician channels.  Persistent 256-thread
// workgroups (four waves, three per CU) take the deployments in turn, with
// the next deployment's positions and NLoS draws loaded into registers while
// the current one runs; everything else is in LDS:
//
//  1. H: thread m synthesises antenna m's terms for every user with the
//     channel kernel's term arithmetic (FP64 distance and phase, the same
//     bits as dmimo_channel), reading the Rician NLoS draws once, coalesced
//     along m.  H goes to LDS ([K][M], rows padded) and, if asked, to HBM.
//  2. G = H H^H on the matrix cores, wave w over antennas 64 w .. 64 w + 63:
//     FP32 16x16x4 products (DMIMO_F32), or 16x16x32 FP16 / BF16 products of
//     hi/lo splits, three per real product (MIX modes; FP16 with a power-of-
//     two scale of H).  Real form: Gr = Hr Hr^T + Hi Hi^T,
//     Gi = Hi Hr^T - Hr Hi^T, with one register feeding both MFMA operands.
//     The four partial sums are added in wave order in FP64, and the upper
//     triangle is mirrored (G exactly Hermitian).
//  3. ZF: G^-1 by FP64 Gauss-Jordan without pivoting, one entry per thread;
//     the pivot test of dmimo_beamform (info = failed step).  MR: none.
//  4. X = G^-1 H by FP32 16x16x4 products (the FP64 inverse rounded to FP32;
//     Xr = Ar Hr - Ai Hi, Xi = Ar Hi + Ai Hr), or X = H for MR; then
//     W = c conj(X) to HBM (optional), p_m = sum_k |w_km|^2 and sum_m sqrt(p_m)
//     in FP64.
//  5. The gains A = H W^T.  With W = conj(G^-1 H) D_c and G = H H^H this is
//     A = G G^-1 D_c for ZF and A = c G for MR (exact identities), formed in
//     FP64 from the same G; SINR_k and the sum rate follow (Sec. VI-B).
// A deployment reads its NLoS draws (8 B per term) and positions and writes
// W (8 B per term, optional) and the epilogues: nothing else touches HBM.
#include <algorithm>
#include <atomic>
#include <cmath>

#include "kernels.h"
#include "split16.h"

namespace dmimo {

namespace {

constexpr int kBbThreads = 256;
constexpr int kBbK = 16;         // users: the rows of every product tile
constexpr int kBbM = 256;        // antennas: four waves of 64
constexpr int kBbP = kBbM + 1;   // LDS row stride of H (complex entries): distinct banks per row

struct BbDev {
    WaveConst w;
    int64_t B;
    int K, M;
    int precoder;          // DMIMO_MR or DMIMO_ZF
    int prec;              // DMIMO_F32, DMIMO_MIX_F16X3, DMIMO_MIX_BF16X3
    const double* ap;      // [B][M][3]
    const double* users;   // [B][K][3]
    const float2* nlos;    // [B][K][M] CN(0,1) draws, or null (LoS)
    double cpaper[kBbK];   // ZF at p_total <= 0: the row scales sigma sqrt(gamma_k)
    double sigma2, p_total, pivot_tol;
    float2* H;             // [B][K][M] or null
    float2* W;             // [B][K][M] or null
    double* p_ant;         // [B][M] or null
    double* l21;           // [B] or null
    double* sinr;          // [B][K] or null
    double* rsum;          // [B] or null
    int32_t* info;         // [B] or null
};

struct BbShared {
    float2 h[kBbK][kBbP];                    // the channel, FP32
    union {
        float part[4][2][kBbK][kBbK + 1];    // per-wave Gram partials (Gr, Gi)
        double2 A[kBbK][kBbK + 1];           // the gains, at the end
    } u;
    double2 g0[kBbK][kBbK + 1];              // G (FP64)
    double2 gi[kBbK][kBbK + 1];              // G^-1
    double user[kBbK][3];
    double d0[kBbK];
    double c[kBbK];                          // scale of W's row k
    double cpaper[kBbK];                     // the row scales of ZF at p_total <= 0
    double red[4];
    float hmax[4];
    int fail;
};

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Gauss-Jordan elimination without pivoting of the K x K matrix g in LDS, in
// place, by one wave with no barrier: lane l holds row l / 4 and columns
// 4 (l % 4) .. 4 (l % 4) + 3.  In every step each lane reads the pivot, its
// row's pivot-column entry and the pivot row's entries of its columns before
// any lane writes (a wave's LDS accesses run in program order).  The pivot of
// step p is the diagonal entry of the Schur complement (L_pp^2 of the
// Cholesky factor); one not above tol * d0[p] stops the elimination.
// Returns 0 or the failed step p + 1 (the same in every lane).
__device__ int bb_invert_wave(double2 (*g)[kBbK + 1], const double* d0, int K, double tol,
                              int lane) {
    const int r = lane >> 2, c0 = 4 * (lane & 3);
    for (int p = 0; p < K; ++p) {
        const double piv = g[p][p].x;
        if (!(piv > tol * d0[p])) return p + 1;
        const double inv = 1.0 / piv;
        const double2 gip = g[r][p];
        double2 prow[4], mine[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            prow[e] = g[p][c0 + e];
            mine[e] = g[r][c0 + e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = c0 + e;
            const double2 rv = j == p ? make_double2(inv, 0.0)
                                      : make_double2(prow[e].x * inv, prow[e].y * inv);
            double2 nv;
            if (r == p) {
                nv = rv;
            } else {
                const double2 x = j == p ? make_double2(0.0, 0.0) : mine[e];
                nv = make_double2(fma(-gip.x, rv.x, fma(gip.y, rv.y, x.x)),
                                  fma(-gip.x, rv.y, fma(-gip.y, rv.x, x.y)));
            }
            if (r < K && j < K) g[r][j] = nv;
        }
    }
    return 0;
}

// The Gram partial of wave `wave` (antennas 64 wave .. 64 wave + 63) into part[wave].
template <int MODE>   // 0: FP32, 1: FP16 x3, 2: BF16 x3
__device__ __forceinline__ void bb_gram(BbShared& S, int wave, int lane, int hexp) {
    f32x4 gr = {0.f, 0.f, 0.f, 0.f}, gim = {0.f, 0.f, 0.f, 0.f};
    if constexpr (MODE == 0) {
        // lane (k, i): H[i][64 wave + 4 s + k]; the same value is A[i][k] and B[k][i]
        const int k = lane >> 4, i = lane & 15;
#pragma unroll 4
        for (int s = 0; s < 16; ++s) {
            const float2 v = S.h[i][64 * wave + 4 * s + k];
            gr = mfma4(v.x, v.x, gr);
            gr = mfma4(v.y, v.y, gr);
            gim = mfma4(v.y, v.x, gim);
            gim = mfma4(-v.x, v.y, gim);
        }
    } else {
        constexpr bool BF16 = MODE == 2;
        // lane (g, i): H[i][64 wave + 32 s + 8 g .. + 7], hi/lo split
        const int g = lane >> 4, i = lane & 15;
        const u32x4 sgn = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float2* row = &S.h[i][64 * wave + 32 * s + 8 * g];
            u32x4 rh, rl, ih, il;
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
                const float2 v0 = row[e], v1 = row[e + 1];
                float r0, r1, q0, q1;
                rh[e >> 1] = pack_hi<BF16>(ldexpf(v0.x, hexp), ldexpf(v1.x, hexp), r0, r1);
                ih[e >> 1] = pack_hi<BF16>(ldexpf(v0.y, hexp), ldexpf(v1.y, hexp), q0, q1);
                rl[e >> 1] = pack_lo<BF16>(r0, r1);
                il[e >> 1] = pack_lo<BF16>(q0, q1);
            }
            const u32x4 nrh = rh ^ sgn, nrl = rl ^ sgn;
            gr = mfma16<BF16>(rh, rh, gr);
            gr = mfma16<BF16>(rl, rh, gr);
            gr = mfma16<BF16>(rh, rl, gr);
            gr = mfma16<BF16>(ih, ih, gr);
            gr = mfma16<BF16>(il, ih, gr);
            gr = mfma16<BF16>(ih, il, gr);
            gim = mfma16<BF16>(ih, rh, gim);
            gim = mfma16<BF16>(il, rh, gim);
            gim = mfma16<BF16>(ih, rl, gim);
            gim = mfma16<BF16>(nrh, ih, gim);
            gim = mfma16<BF16>(nrl, ih, gim);
            gim = mfma16<BF16>(nrh, il, gim);
        }
    }
    // lane (g, j) holds D[4 g + r][j]
    const int g = lane >> 4, j = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        S.u.part[wave][0][4 * g + r][j] = gr[r];
        S.u.part[wave][1][4 * g + r][j] = gim[r];
    }
}

// Inputs of one deployment held in registers: thread m's antenna position
// and NLoS draws (16 users), and one coordinate of the users.
struct BbIn {
    double ax, ay, az, u;
    float2 g[kBbK];
};

__device__ __forceinline__ void bb_fetch(const BbDev& a, int64_t b, int tid, BbIn& in) {
    const int K = a.K, M = a.M;
    // clamped indices: every lane loads a valid address, unused values are never read
    const int m = tid < M ? tid : M - 1;
    const double* q = a.ap + (b * M + m) * 3;
    in.ax = q[0];
    in.ay = q[1];
    in.az = q[2];
    if (a.nlos) {
        const float2* gb = a.nlos + b * K * M + m;
#pragma unroll
        for (int i = 0; i < kBbK; ++i) in.g[i] = gb[(i < K ? i : K - 1) * M];
    }
    if (tid < 3 * K) in.u = a.users[b * K * 3 + tid];
}

// 1. the users' channels of deployment b, from the inputs in registers
template <int MODE>
__device__ __forceinline__ void bb_deployment(const BbDev& a, int64_t b, BbShared& S, const BbIn& in) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int K = a.K, M = a.M;
    const bool live = tid < M;
    const double ax = in.ax, ay = in.ay, az = in.az;
    const bool rician = a.nlos != nullptr;
    float2* const Hb = a.H ? a.H + b * K * M + tid : nullptr;
    float mx = 0.0f;
    // all 16 rows are computed (rows k >= K from user 0's position) and the
    // unused ones zeroed: no per-row lane masks
#pragma unroll
    for (int i = 0; i < kBbK; ++i) {
        const int iu = i < K ? i : 0;
        const TermF32 t = wave_term_f32(S.user[iu][0] - ax, S.user[iu][1] - ay, S.user[iu][2] - az,
                                        a.w.inv_lam, (float)a.w.amp_c, (float)a.w.inv_dmin);
        float2 h;
        if (rician) {
            const float2 g = in.g[i];
            h.x = t.amp * fmaf((float)a.w.a_los, t.c, (float)a.w.a_nlos * g.x);
            h.y = t.amp * fmaf(-(float)a.w.a_los, t.s, (float)a.w.a_nlos * g.y);
        } else {
            h.x = t.amp * t.c;
            h.y = -t.amp * t.s;
        }
        const bool use = live && i < K;
        h = use ? h : make_float2(0.f, 0.f);
        if (Hb && use) Hb[i * M] = h;
        if (MODE == 1) mx = fmaxf(mx, fmaxf(fabsf(h.x), fabsf(h.y)));
        S.h[i][tid] = h;    // zero rows and columns pad H to 16 x 256
    }
    if constexpr (MODE == 1) {
        for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        if (lane == 0) S.hmax[wave] = mx;
    }
    (void)lane;
    (void)wave;
    (void)mx;
}

// 2 - 5: the Gram, the precoder and the epilogues of deployment b
template <int MODE>
__device__ __forceinline__ void bb_rest(const BbDev& a, int64_t b, BbShared& S) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int K = a.K, M = a.M;
    __syncthreads();
    int hexp = 0;
    if constexpr (MODE == 1) {
        // FP16: largest |h| of the deployment scaled into [2^13, 2^14)
        const float m4 = fmaxf(fmaxf(S.hmax[0], S.hmax[1]), fmaxf(S.hmax[2], S.hmax[3]));
        hexp = m4 > 0.0f ? 14 - (ilogbf(m4) + 1) : 0;
    }

    // 2. the Gram, per wave, then added in wave order in FP64
    if (64 * wave < M) {
        bb_gram<MODE>(S, wave, lane, hexp);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            S.u.part[wave][0][4 * (lane >> 4) + r][lane & 15] = 0.0f;
            S.u.part[wave][1][4 * (lane >> 4) + r][lane & 15] = 0.0f;
        }
    }
    __syncthreads();
    {
        const int i = tid >> 4, j = tid & 15;
        const int ii = i <= j ? i : j, jj = i <= j ? j : i;   // upper triangle, mirrored
        double gr = 0.0, gim = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            gr += (double)S.u.part[w][0][ii][jj];
            gim += (double)S.u.part[w][1][ii][jj];
        }
        if (MODE == 1) {
            gr = ldexp(gr, -2 * hexp);
            gim = ldexp(gim, -2 * hexp);
        }
        if (i == j) gim = 0.0;
        if (i > j) gim = -gim;
        const double2 v = make_double2(gr, gim);
        S.g0[i][j] = v;
        S.gi[i][j] = v;
        if (i == j) S.d0[i] = gr;
    }
    __syncthreads();

    // 3. ZF: the inverse (wave 0); the scale of every row of W
    const bool zf = a.precoder == DMIMO_ZF;
    if (zf && wave == 0) {
        const int f = bb_invert_wave(S.gi, S.d0, K, a.pivot_tol, lane);
        if (lane == 0) S.fail = f;
    }
    __syncthreads();
    const int fail = S.fail;
    if (tid < K) {
        double c;
        if (a.p_total > 0.0) {
            double tr = 0.0;
            for (int k = 0; k < K; ++k) tr += zf ? S.gi[k][k].x : S.g0[k][k].x;
            c = tr > 0.0 ? sqrt(a.p_total / tr) : 0.0;
        } else {
            c = zf ? S.cpaper[tid] : 1.0;
        }
        S.c[tid] = fail ? 0.0 : c;
    }
    __syncthreads();

    // 4. X = G^-1 H (or H), W = c conj(X), p_m; wave w takes antenna tiles
    //    4 w .. 4 w + 3 of 16 antennas
    double l21_part = 0.0;
    {
        const int kq = lane >> 4, col = lane & 15;    // operand lane (k', i) / output lane (g, c)
        float ar[4], ai[4];
        if (zf) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double2 v = S.gi[col][4 * t + kq];
                const bool in = col < K && 4 * t + kq < K;
                ar[t] = in ? (float)v.x : 0.0f;
                ai[t] = in ? (float)v.y : 0.0f;
            }
        }
        float cs[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) cs[r] = 4 * kq + r < K ? (float)S.c[4 * kq + r] : 0.0f;
        for (int n = 4 * wave; n < 4 * wave + 4 && 16 * n < M; ++n) {
            const int m0 = 16 * n;
            f32x4 xr = {0.f, 0.f, 0.f, 0.f}, xi = {0.f, 0.f, 0.f, 0.f};
            if (zf) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float2 hv = S.h[4 * t + kq][m0 + col];
                    xr = mfma4(ar[t], hv.x, xr);
                    xr = mfma4(-ai[t], hv.y, xr);
                    xi = mfma4(ar[t], hv.y, xi);
                    xi = mfma4(ai[t], hv.x, xi);
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float2 hv = S.h[4 * kq + r][m0 + col];
                    xr[r] = hv.x;
                    xi[r] = hv.y;
                }
            }
            // lane (g, c) holds X[4 g + r][m0 + c]
            const int m = m0 + col;
            double pm = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k = 4 * kq + r;
                const float wr = cs[r] * xr[r], wi = -cs[r] * xi[r];
                if (a.W && k < K && m < M) a.W[(b * K + k) * M + m] = make_float2(wr, wi);
                pm += (double)wr * (double)wr + (double)wi * (double)wi;
            }
            pm += __shfl_xor(pm, 16, 64);
            pm += __shfl_xor(pm, 32, 64);
            if (m < M) {
                if (a.p_ant && kq == 0) a.p_ant[b * M + m] = pm;
                if (kq == 0) l21_part += sqrt(pm);
            }
        }
    }
    for (int off = 8; off > 0; off >>= 1) l21_part += __shfl_xor(l21_part, off, 64);
    if (lane == 0) S.red[wave] = l21_part;

    // 5. gains A = G G^-1 D_c (ZF) or c G (MR), SINR_k, sum rate
    {
        const int k = tid >> 4, j = tid & 15;
        double2 acc = make_double2(0.0, 0.0);
        if (k < K && j < K && !fail) {
            if (zf) {
                for (int l = 0; l < K; ++l) {
                    const double2 x = S.g0[k][l], y = S.gi[l][j];
                    acc.x = fma(x.x, y.x, fma(-x.y, y.y, acc.x));
                    acc.y = fma(x.x, y.y, fma(x.y, y.x, acc.y));
                }
            } else {
                acc = S.g0[k][j];
            }
            acc.x *= S.c[j];
            acc.y *= S.c[j];
        }
        __syncthreads();   // the Gram partials are dead; A reuses their bytes
        S.u.A[k][j] = acc;
    }
    __syncthreads();
    if (tid < K) {
        double sig = 0.0, intf = 0.0;
        for (int j = 0; j < K; ++j) {
            const double2 v = S.u.A[tid][j];
            const double p = v.x * v.x + v.y * v.y;
            if (j == tid) sig = p;
            else intf += p;
        }
        const double s = fail ? 0.0 : sig / (intf + a.sigma2);
        if (a.sinr) a.sinr[b * K + tid] = s;
        S.d0[tid] = log2(1.0 + s);
    }
    __syncthreads();
    if (tid == 0) {
        double rs = 0.0;
        for (int k = 0; k < K; ++k) rs += S.d0[k];
        if (a.rsum) a.rsum[b] = fail ? 0.0 : rs;
        if (a.l21) a.l21[b] = fail ? 0.0 : ((S.red[0] + S.red[1]) + S.red[2]) + S.red[3];
        if (a.info) a.info[b] = fail;
    }
}

// Persistent: workgroup w takes deployments w, w + gridDim.x, ...; the next
// deployment's inputs are loaded into registers while the current one runs.
template <int MODE>
__global__ __launch_bounds__(kBbThreads) __attribute__((amdgpu_waves_per_eu(3)))
void beamform_batched_kernel(BbDev a) {
    __shared__ BbShared S;
    const int tid = threadIdx.x;
    const int K = a.K;
    BbIn in;
    if (tid < kBbK) S.cpaper[tid] = a.cpaper[tid];
    if ((int64_t)blockIdx.x < a.B) bb_fetch(a, blockIdx.x, tid, in);
    for (int64_t b = blockIdx.x; b < a.B; b += gridDim.x) {
        if (tid < 3 * K) S.user[tid / 3][tid - 3 * (tid / 3)] = in.u;
        if (tid == 0) S.fail = 0;
        __syncthreads();
        bb_deployment<MODE>(a, b, S, in);
        if (b + gridDim.x < a.B) bb_fetch(a, b + gridDim.x, tid, in);   // in flight meanwhile
        bb_rest<MODE>(a, b, S);
        __syncthreads();   // LDS is rewritten for the next deployment
    }
}

// Compute units of the current device (cached per device).
int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int c = cache[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
            c = 256;
        cache[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

}  // namespace

dmimo_status launch_beamform_batched(const BeamformArgs& ba, const WaveConst& w,
                                     const double* ap_xyz, const double* user_xyz,
                                     const void* nlos, void* H, hipStream_t s) {
    if (ba.K < 1 || ba.K > kBbK || ba.M < 1 || ba.M > kBbM)
        return fail(DMIMO_E_SHAPE, "beamform_batched: K <= 16 and M <= 256");
    if (ba.B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "beamform_batched: B too large");
    if (ba.B == 0) return DMIMO_OK;
    BbDev d;
    d.w = w;
    d.B = ba.B;
    d.K = ba.K;
    d.M = (int)ba.M;
    d.precoder = ba.precoder;
    d.prec = ba.prec;
    d.ap = ap_xyz;
    d.users = user_xyz;
    d.nlos = reinterpret_cast<const float2*>(nlos);
    for (int k = 0; k < kBbK; ++k) d.cpaper[k] = std::sqrt(ba.sigma2) * std::sqrt(ba.gamma[k]);
    d.sigma2 = ba.sigma2;
    d.p_total = ba.p_total;
    d.pivot_tol = ba.prec == DMIMO_MIX_BF16X3 ? 1e-4 : 1e-6;
    d.H = reinterpret_cast<float2*>(H);
    d.W = reinterpret_cast<float2*>(ba.W);
    d.p_ant = ba.p_ant;
    d.l21 = ba.l21;
    d.sinr = ba.sinr;
    d.rsum = ba.rsum;
    d.info = ba.info;
    // persistent workgroups: three per CU fit the 51 KB of LDS
    const int64_t wgs = 3 * (int64_t)device_cus();
    const dim3 grid((unsigned)std::min<int64_t>(ba.B, wgs)), block(kBbThreads);
    if (ba.prec == DMIMO_MIX_F16X3)
        beamform_batched_kernel<1><<<grid, block, 0, s>>>(d);
    else if (ba.prec == DMIMO_MIX_BF16X3)
        beamform_batched_kernel<2><<<grid, block, 0, s>>>(d);
    else
        beamform_batched_kernel<0><<<grid, block, 0, s>>>(d);
    return check_launch("beamform_batched_kernel");
}

}  // namespace dmimo
