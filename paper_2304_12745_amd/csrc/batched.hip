// Users' channels, precoder and epilogues of many small deployments in one
// launch (K <= 16 users, M <= 256 antennas): the batched workload of
// independent rooms with LoS or Rician channels.  Persistent 256-thread
// workgroups (four waves, three per CU) take the deployments b, b + grid, ...
// in a two-stage pipeline: while wave 0 inverts the Gram of deployment b,
// waves 1 - 3 synthesise the channel of b + grid into registers, and the
// inputs of b + 2 grid are loaded.  Per deployment:
//
//  1. H: thread m synthesises antenna m's terms for every user with the
//     channel kernel's term arithmetic (FP64 distance and phase, the same
//     bits as dmimo_channel), reading the Rician NLoS draws once, coalesced
//     along m, into registers (and, if asked, H to HBM); the column goes to
//     LDS ([16][257], zero past K and M) once the previous deployment is done.
//  2. G = H H^H on the matrix cores, wave w over antennas 64 w .. 64 w + 63:
//     FP32 16x16x4 products (DMIMO_F32), or 16x16x32 FP16 / BF16 products of
//     hi/lo splits, three per real product (MIX modes; FP16 with a power-of-
//     two scale of H).  Real form: Gr = Hr Hr^T + Hi Hi^T,
//     Gi = Hi Hr^T - Hr Hi^T, with one register feeding both MFMA operands.
//     The four partial sums are added in wave order in FP64, and the upper
//     triangle is mirrored (G exactly Hermitian).
//  3. ZF: G^-1 by FP64 Gauss-Jordan without pivoting in wave 0's registers;
//     the pivot test of dmimo_beamform (info = failed step); the scales of
//     W's rows.  MR: the scales only.
//  4. Waves 1 - 3: X = G^-1 H (FP32 16x16x4 products of the FP64 inverse
//     rounded to FP32, or split-FP16 16x16x32 products in the MIX modes), or
//     X = H for MR; W = c conj(X) to HBM (optional), p_m and sum_m sqrt(p_m).
//  5. Wave 0: the gains A = H W^T.  With W = conj(G^-1 H) D_c and G = H H^H
//     this is A = D_c for ZF and A = G D_c for MR (exact identities), so ZF
//     has SINR_k = c_k^2 / sigma^2 and MR sums its interference from G;
//     SINR_k and the sum rate follow (Sec. VI-B).
// A deployment reads its NLoS draws (8 B per term) and positions and writes
// W (8 B per term, optional) and the epilogues: nothing else touches HBM.
// The same kernel with H given (HIN: dmimo_beamform's ZF and MR at these
// shapes) loads thread m's column of H in step 1 instead of synthesising it
// and runs steps 2 - 5 unchanged: the same bits as the fused call on the H
// that call writes.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>

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
    const float2* Hin;     // [B][K][M]: the channel given (the HIN kernel)
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
        double2 prow[kBbK][kBbK];            // Gauss-Jordan: row r as it enters step r
    } u;
    double2 g0[kBbK][kBbK + 1];              // G (FP64), zero outside K x K
    double2 gi[kBbK][kBbK + 1];              // G^-1, zero outside K x K
    double user[kBbK][3];
    double c[kBbK];                          // scale of W's row k, zero for k >= K
    double cpaper[kBbK];                     // the row scales of ZF at p_total <= 0
    double rate[kBbK];                       // log2(1 + SINR_k)
    double red[4];
    float hmax[4];
    int aexp;                                // MIX: power-of-two scale of G^-1
    int fail;
};

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// x summed over the four lanes l, l ^ 16, l ^ 32, l ^ 48 (the same bits in
// all four): the row swaps of v_permlane16_swap / v_permlane32_swap
__device__ __forceinline__ float sum_rows4(float x) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    const auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(t[0]) + __uint_as_float(t[1]);
}

__device__ __forceinline__ double readlane_d(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// every lane of a quad takes the value of quad lane Q (DPP quad_perm)
template <int Q>
__device__ __forceinline__ double quad_bcast(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), Q * 0x55, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), Q * 0x55, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double quad_bcast(double x, int q) {
    switch (q) {
        case 0: return quad_bcast<0>(x);
        case 1: return quad_bcast<1>(x);
        case 2: return quad_bcast<2>(x);
        default: return quad_bcast<3>(x);
    }
}

// Cross-lane reductions without LDS: DPP moves within each 16-lane row
// (quad_perm [1,0,3,2] and [2,3,0,1], then row_ror:4 and row_ror:8), then the
// row swaps of v_permlane16_swap / v_permlane32_swap across the four rows.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_mov_dpp(x, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    return __hiloint2double(dpp_i<CTRL>(__double2hiint(x)), dpp_i<CTRL>(__double2loint(x)));
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}

// x summed over the 16 lanes of its row (in every lane of the row)
__device__ __forceinline__ double row_sum16(double x) {
    x += dpp_d<0xB1>(x);
    x += dpp_d<0x4E>(x);
    x += dpp_d<0x124>(x);
    x += dpp_d<0x128>(x);
    return x;
}

// x summed over the lanes l, l ^ 16, l ^ 32, l ^ 48
__device__ __forceinline__ double sum_rows4_d(double x) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(x), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(x), false, false);
    x = __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
    const auto lo2 = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(x), false, false);
    const auto hi2 = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(x), false, false);
    return __hiloint2double(hi2[0], lo2[0]) + __hiloint2double(hi2[1], lo2[1]);
}

__device__ __forceinline__ double wave_sum(double x) { return sum_rows4_d(row_sum16(x)); }

__device__ __forceinline__ int wave_max_i(int x) {
    x = max(x, dpp_i<0xB1>(x));
    x = max(x, dpp_i<0x4E>(x));
    x = max(x, dpp_i<0x124>(x));
    x = max(x, dpp_i<0x128>(x));
    const auto s = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    x = max((int)s[0], (int)s[1]);
    const auto t = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return max((int)t[0], (int)t[1]);
}

__device__ __forceinline__ float wave_max_f(float x) {
    x = fmaxf(x, dpp_f<0xB1>(x));
    x = fmaxf(x, dpp_f<0x4E>(x));
    x = fmaxf(x, dpp_f<0x124>(x));
    x = fmaxf(x, dpp_f<0x128>(x));
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = fmaxf(__uint_as_float(s[0]), __uint_as_float(s[1]));
    const auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return fmaxf(__uint_as_float(t[0]), __uint_as_float(t[1]));
}

// Gauss-Jordan elimination without pivoting of a 16 x 16 Hermitian positive
// definite matrix G held by one wave in registers: lane l holds row l / 4,
// columns 4 (l % 4) .. + 3 in v.  The elimination runs on the Jacobi-scaled
// matrix G' = S G S, S = diag(G)^-1/2 (unit diagonal, every pivot at most 1),
// and G^-1 = S G'^-1 S at the end.  Step p reads the pivot from its lane
// (readlane), gives every lane the pivot-column entry g of its row by a
// broadcast within the quad that holds the row (DPP), and the pivot row's
// entries of its columns through LDS (prow), where the lanes of row p + 1
// leave that row after step p with 1 in place of its pivot.  Every row then
// takes the same update x - (g / piv) pr: the pivot row with g - 1 (which
// gives pr / piv up to piv 2^-53 relative, piv <= 1), the pivot column with
// x = 0 (1 in the pivot row), so no row needs a case of its own.  The pivot
// of step p is the Schur complement's diagonal entry of G' (L_pp^2 / G_pp of
// the Cholesky factor L of G); one not above tol stops the elimination.
// Returns 0 or the failed step p + 1, the same in every lane (v is then not
// used).
__device__ __forceinline__ int bb_gauss_jordan(double2 (&v)[4], double2 (*prow)[kBbK], double tol,
                                               int lane) {
    const int r = lane >> 2, q = lane & 3;
    // 1 / sqrt(G_rr), held by the lane that holds the diagonal entry of row r
    double dg = 1.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) dg = 4 * q + e == r ? v[e].x : dg;
    const double sd = 1.0 / sqrt(dg);
    const double sr = __shfl(sd, 4 * r + (r >> 2), 64);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double sc = __shfl(sd, 4 * (4 * q + e) + q, 64);
        const bool dia = 4 * q + e == r;
        v[e].x = dia ? 1.0 : v[e].x * sr * sc;
        v[e].y = dia ? 0.0 : v[e].y * sr * sc;
    }
    if (r == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) prow[0][4 * q + e] = 4 * q + e == 0 ? make_double2(1.0, 0.0) : v[e];
    }
#pragma unroll
    for (int p = 0; p < kBbK; ++p) {
        const double piv = readlane_d(v[p & 3].x, 4 * p + (p >> 2));
        if (!(piv > tol)) return p + 1;
        // 1 / piv: hardware reciprocal and two Newton steps (within an ulp)
        double inv = __builtin_amdgcn_rcp(piv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        inv = fma(inv, fma(-piv, inv, 1.0), inv);
        double2 pr[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) pr[e] = prow[p][4 * q + e];
        const double gx = quad_bcast(v[p & 3].x, p >> 2) - (r == p ? 1.0 : 0.0);
        const double gy = quad_bcast(v[p & 3].y, p >> 2);
        const double gix = gx * inv, giy = gy * inv;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double xx = v[e].x, xy = v[e].y;
            if (e == (p & 3)) {
                const bool jp = q == (p >> 2);
                xx = jp ? (r == p ? 1.0 : 0.0) : xx;
                xy = jp ? 0.0 : xy;
            }
            v[e].x = fma(-gix, pr[e].x, fma(giy, pr[e].y, xx));
            v[e].y = fma(-gix, pr[e].y, fma(-giy, pr[e].x, xy));
        }
        if (p + 1 < kBbK && r == p + 1) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                prow[p + 1][4 * q + e] = 4 * q + e == p + 1 ? make_double2(1.0, 0.0) : v[e];
        }
    }
    // G^-1 = S G'^-1 S
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double sc = __shfl(sd, 4 * (4 * q + e) + q, 64);
        v[e] = make_double2(v[e].x * sr * sc, v[e].y * sr * sc);
    }
    return 0;
}

// 5. (one wave) the gains A = H W^T and SINR_k = |A_kk|^2 / (sum_{j != k}
// |A_kj|^2 + sigma^2), written for k < K with log2(1 + SINR_k) to LDS for
// R_sum.  ZF: A = G G^-1 D_c = D_c, no interference, SINR_k = c_k^2 / sigma^2
// (the product G G^-1 formed in FP64 differs from I only by the inverse's
// rounding, which changes no digit of SINR_k).  MR: A = G D_c, the
// interference summed over the 16 lanes of a row group (lane (g, j) holds
// A[g + 4r][j]) and SINR_k formed by lane (g, x < 4) for row g + 4x.
__device__ __forceinline__ void bb_gains(const BbDev& a, int64_t b, BbShared& S, int K, int lane,
                                         int fail, bool zf) {
    if (zf) {
        if (lane < K) {
            const double ck = S.c[lane];
            const double sv = fail ? 0.0 : (ck * ck) / a.sigma2;
            if (a.sinr) a.sinr[b * K + lane] = sv;
            S.rate[lane] = log2(1.0 + sv);
        }
        return;
    }
    const int kq = lane >> 4, x = lane & 15;
    double ar[4], ai[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double2 g = S.g0[kq + 4 * r][x];
        ar[r] = g.x;
        ai[r] = g.y;
    }
    const double cj = S.c[x];
    double sig[4], itf[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double pw = (ar[r] * ar[r] + ai[r] * ai[r]) * (cj * cj);
        const bool diag = x == kq + 4 * r;
        sig[r] = row_sum16(diag ? pw : 0.0);
        itf[r] = row_sum16(diag ? 0.0 : pw);
    }
    // lane (kq, x < 4) finishes row k = kq + 4 x
    if (x < 4) {
        const int k = kq + 4 * x;
        double sg = sig[0], it = itf[0];
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            sg = x == r ? sig[r] : sg;
            it = x == r ? itf[r] : it;
        }
        if (k < K) {
            const double sv = fail ? 0.0 : sg / (it + a.sigma2);
            if (a.sinr) a.sinr[b * K + k] = sv;
            S.rate[k] = log2(1.0 + sv);
        }
    }
}

// The Gram partial of wave `wave` over antennas 64 wave .. 64 wave + 63 of
// h (LDS, [16][kBbP], zero past K and M): lane (g, j) gets Re and Im of
// entry (4 g + r, j) in gr[r], gim[r].  MIX: h scaled by 2^hexp before the
// split (FP16), so the partial is 2^(2 hexp) times the Gram's.
template <int MODE>   // 0: FP32, 1: FP16 x3, 2: BF16 x3
__device__ __forceinline__ void gram_partial(const float2 (*h)[kBbP], int wave, int lane, int hexp,
                                             f32x4& gr, f32x4& gim) {
    gr = f32x4{0.f, 0.f, 0.f, 0.f};
    gim = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (MODE == 0) {
        // lane (k, i): H[i][64 wave + 4 s + k]; the same value is A[i][k] and B[k][i]
        const int k = lane >> 4, i = lane & 15;
#pragma unroll 4
        for (int s = 0; s < 16; ++s) {
            const float2 v = h[i][64 * wave + 4 * s + k];
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
            const float2* row = &h[i][64 * wave + 32 * s + 8 * g];
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
}

// The Gram partial of wave `wave` into part[wave].
template <int MODE>
__device__ __forceinline__ void bb_gram(BbShared& S, int wave, int lane, int hexp) {
    f32x4 gr, gim;
    gram_partial<MODE>(S.h, wave, lane, hexp, gr, gim);
    // lane (g, j) holds D[4 g + r][j]
    const int g = lane >> 4, j = lane & 15;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        S.u.part[wave][0][4 * g + r][j] = gr[r];
        S.u.part[wave][1][4 * g + r][j] = gim[r];
    }
}

// Inputs of one deployment held in registers: thread m's antenna position
// and NLoS draws (16 users), and one coordinate of the users; with H given,
// thread m's column of H in g.
struct BbIn {
    double ax, ay, az, u;
    float2 g[kBbK];
};

// Marks the inputs as read here: the compiler waits for their loads at this
// point and at no later one.
__device__ __forceinline__ void bb_settle(BbIn& in) {
    asm volatile("" : "+v"(in.ax), "+v"(in.ay), "+v"(in.az), "+v"(in.u));
#pragma unroll
    for (int i = 0; i < kBbK; ++i) asm volatile("" : "+v"(in.g[i].x), "+v"(in.g[i].y));
}

template <bool HIN>
__device__ __forceinline__ void bb_fetch(const BbDev& a, int64_t b, int tid, BbIn& in, int K, int M) {
    // clamped indices: every lane loads a valid address, unused values are never read
    const int m = tid < M ? tid : M - 1;
    if constexpr (HIN) {
        const float2* hb = a.Hin + b * K * M + m;
#pragma unroll
        for (int i = 0; i < kBbK; ++i) in.g[i] = hb[(i < K ? i : K - 1) * M];
        in.ax = in.ay = in.az = in.u = 0.0;
        return;
    }
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

// 1. The users' channels of deployment b into registers, thread m holding
// antenna m's column h[0 .. 15]: rows i < K (rows past K stay zero); lanes
// m >= M compute antenna M - 1's terms from the clamped inputs (written to
// the pad column of LDS, which nothing reads).  Returns the lane's largest
// |Re h|, |Im h| (MIX).
template <int MODE, bool RICIAN, bool WANT_H>
__device__ __forceinline__ float bb_synth_rows(const BbDev& a, int64_t b, const BbShared& S, const BbIn& in,
                                               int K, int M, int tid, float2 (&h)[kBbK]) {
    const bool live = tid < M;
    float2* const Hb = WANT_H ? a.H + b * K * M + tid : nullptr;
    const float a_los = (float)a.w.a_los, a_nlos = (float)a.w.a_nlos;
    float mx = 0.0f;
#pragma unroll
    for (int i = 0; i < kBbK; ++i) {
        h[i] = make_float2(0.0f, 0.0f);
        if (i >= K) continue;   // uniform; the loop stays fully unrolled
        const TermF32 t = wave_term_f32(S.user[i][0] - in.ax, S.user[i][1] - in.ay, S.user[i][2] - in.az,
                                        a.w.inv_lam, (float)a.w.amp_c, (float)a.w.inv_dmin);
        float2 v;
        if constexpr (RICIAN) {
            const float2 g = in.g[i];
            v.x = t.amp * fmaf(a_los, t.c, a_nlos * g.x);
            v.y = t.amp * fmaf(-a_los, t.s, a_nlos * g.y);
        } else {
            v.x = t.amp * t.c;
            v.y = -t.amp * t.s;
        }
        if constexpr (WANT_H) {
            if (live) Hb[i * M] = v;
        }
        if constexpr (MODE != 0) mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
        h[i] = v;
    }
    return mx;
}

template <int MODE, bool HIN>
__device__ __forceinline__ float bb_synth(const BbDev& a, int64_t b, const BbShared& S, const BbIn& in,
                                          int K, int M, int tid, float2 (&h)[kBbK]) {
    if constexpr (HIN) {
        // the loaded column: rows past K zero, lanes m >= M hold antenna M - 1's
        float mx = 0.0f;
#pragma unroll
        for (int i = 0; i < kBbK; ++i) {
            h[i] = i < K ? in.g[i] : make_float2(0.0f, 0.0f);
            if constexpr (MODE != 0) mx = fmaxf(mx, fmaxf(fabsf(h[i].x), fabsf(h[i].y)));
        }
        return mx;
    }
    if (a.nlos)
        return a.H ? bb_synth_rows<MODE, true, true>(a, b, S, in, K, M, tid, h)
                   : bb_synth_rows<MODE, true, false>(a, b, S, in, K, M, tid, h);
    return a.H ? bb_synth_rows<MODE, false, true>(a, b, S, in, K, M, tid, h)
               : bb_synth_rows<MODE, false, false>(a, b, S, in, K, M, tid, h);
}

// The synthesised column to LDS (H, [K][M] padded to 16 x 256 with zeros) and
// the wave's largest component to hmax (MIX).
template <int MODE>
__device__ __forceinline__ void bb_store_h(BbShared& S, const float2 (&h)[kBbK], float mx, int M, int tid) {
    const int col = tid < M ? tid : kBbP - 1;
#pragma unroll
    for (int i = 0; i < kBbK; ++i) S.h[i][col] = h[i];
    if constexpr (MODE != 0) {
        mx = wave_max_f(mx);
        if ((tid & 63) == 0) S.hmax[tid >> 6] = mx;
    }
    (void)mx;
}

// One deployment b, with H(b) in LDS: its Gram, precoder and epilogues, while
// the next deployment's channel (b + gridDim.x, if `more1`) is synthesised
// into hn and the one after (if `more2`) is loaded into `in`.
//   A  users of b + grid to LDS; the Gram partials of b
//   S  wave 0: G, G^-1 and the scales of b;  waves 1 - 3: their columns of
//      H(b + grid), then the loads of b + 2 grid
//   X  wave 0: its columns of H(b + grid), its loads, the gains and SINR_k
//      of b;  waves 1 - 3: X, W and p_m of b
//   W  H(b + grid) to LDS; the scalar outputs of b
// Four barriers per deployment.  The FP64 solve of b runs beside the
// synthesis of b + grid instead of before it.
template <int MODE, bool HIN>
__device__ __forceinline__ void bb_step(const BbDev& a, int64_t b, BbShared& S, BbIn& in,
                                        float2 (&hn)[kBbK], bool more1, bool more2, int K, int M,
                                        int tid) {
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const bool zf = a.precoder == DMIMO_ZF;
    const int64_t bn = b + gridDim.x;
    // A.  `in` holds the inputs of b + grid (loaded one deployment ago)
    if (!HIN && more1 && tid < 3 * K) S.user[tid / 3][tid - 3 * (tid / 3)] = in.u;
    // MIX: largest |h| of the deployment scaled into [2^13, 2^14) for the
    // FP16 products (the Gram in FP16 mode, X = G^-1 H in both)
    int xexp = 0;
    if constexpr (MODE != 0) {
        const float m4 = fmaxf(fmaxf(S.hmax[0], S.hmax[1]), fmaxf(S.hmax[2], S.hmax[3]));
        xexp = m4 > 0.0f ? 14 - (ilogbf(m4) + 1) : 0;
    }
    const int hexp = MODE == 1 ? xexp : 0;

    // 2. the Gram, per wave
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

    // S.
    float mxn = 0.0f;
    // 3. wave 0: the partials added in wave order in FP64 (upper triangle,
    //    mirrored: G exactly Hermitian), G^-1 (ZF), the scale of every row of W
    if (wave == 0) {
        // the solve is the deployment's longest dependent chain: this wave
        // issues ahead of the other waves on its SIMD until the scales are out
        __builtin_amdgcn_s_setprio(3);
        const int r = lane >> 2, q = lane & 3;
        double2 v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * q + e;
            const int ii = r <= j ? r : j, jj = r <= j ? j : r;
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
            gim = r == j ? 0.0 : (r > j ? -gim : gim);
            v[e] = make_double2(gr, gim);
            S.g0[r][j] = v[e];
        }
        int fail = 0, aexp = 0;
        double t = 0.0;
        if (zf) {
            // padded to 16 x 16 with the identity outside K x K
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = 4 * q + e;
                if (r >= K || j >= K) v[e] = make_double2(r == j ? 1.0 : 0.0, 0.0);
            }
            fail = bb_gauss_jordan(v, S.u.prow, a.pivot_tol, lane);
            double mx = 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int j = 4 * q + e;
                const double2 x = r < K && j < K && !fail ? v[e] : make_double2(0.0, 0.0);
                S.gi[r][j] = x;
                if (j == r) t = x.x;
                mx = fmax(mx, fmax(fabs(x.x), fabs(x.y)));
            }
            if (MODE != 0) {
                // the exponent of the largest entry: the largest exponent
                const int e = wave_max_i(mx > 0.0 ? ilogb(mx) : -(1 << 20));
                aexp = e > -(1 << 20) ? 14 - (e + 1) : 0;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (4 * q + e == r) t = v[e].x;
        }
        const double tr = wave_sum(t);   // tr(G^-1) (ZF) or tr(G) (MR)
        if (lane < kBbK) {
            double c;
            if (a.p_total > 0.0)
                c = tr > 0.0 ? sqrt(a.p_total / tr) : 0.0;
            else
                c = zf ? S.cpaper[lane] : 1.0;
            S.c[lane] = fail || lane >= K ? 0.0 : c;
        }
        if (lane == 0) {
            S.fail = fail;
            S.aexp = aexp;
        }
        __builtin_amdgcn_s_setprio(0);
    }
    else if (more1) {
        mxn = bb_synth<MODE, HIN>(a, bn, S, in, K, M, tid, hn);
        if (more2) bb_fetch<HIN>(a, bn + gridDim.x, tid, in, K, M);
    }
    __syncthreads();
    const int fail = S.fail;

    // X.
    if (wave == 0) {
        if (more1) {
            mxn = bb_synth<MODE, HIN>(a, bn, S, in, K, M, tid, hn);
            if (more2) bb_fetch<HIN>(a, bn + gridDim.x, tid, in, K, M);
        }
        bb_gains(a, b, S, K, lane, fail, zf);
    } else {
        // the loads of b + 2 grid, issued during the solve, are waited for
        // before this wave's stores: the loads and the stores share one
        // counter, and a later wait for a load behind pending stores would be
        // a wait for the stores as well
        bb_settle(in);
    }
    // 4. waves 1 - 3: X = G^-1 H (or H), W = c conj(X), p_m (FP32 sum of
    //    the 16 |w_km|^2); wave w takes the 16-antenna tiles w - 1, w + 2,
    //    w + 5, ...  A failed deployment has c = 0, hence W = 0 (X is finite).
    double l21_part = 0.0;
    if (wave != 0) {
        const int g = lane >> 4, col = lane & 15;    // operand lane (g, i) / output lane (g, c)
        float2* const Wt = a.W ? a.W + (b * K + 4 * g) * M + col : nullptr;
        double* const Pt = a.p_ant ? a.p_ant + b * M + col : nullptr;
        auto tiles = [&](auto zf_c) {
            constexpr bool ZF = decltype(zf_c)::value;
            float ar[4], ai[4];
            u32x4 arh, arl, aih, ail;
            int xs = 0;                              // X is 2^xs times G^-1 H
            if constexpr (ZF) {
                if constexpr (MODE == 0) {
                    // 16x16x4: lane (k', i) holds G^-1[i][4 t + k']
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const double2 v = S.gi[col][4 * t + g];
                        ar[t] = (float)v.x;
                        ai[t] = (float)v.y;
                    }
                } else {
                    // 16x16x32 over [re; im] of 16 users: lane (g, i) holds
                    // [Gr | -Gi][i][8 g ..] (Xr) and [Gi | Gr][i][8 g ..] (Xi),
                    // scaled by 2^aexp and split in FP16 hi/lo
                    const int aexp = S.aexp;
                    const int l0 = 8 * (g & 1);
                    const bool lower = g < 2;
#pragma unroll
                    for (int e = 0; e < 8; e += 2) {
                        const double2 v0 = S.gi[col][l0 + e], v1 = S.gi[col][l0 + e + 1];
                        const float r0 = (float)ldexp(lower ? v0.x : -v0.y, aexp);
                        const float r1 = (float)ldexp(lower ? v1.x : -v1.y, aexp);
                        const float i0 = (float)ldexp(lower ? v0.y : v0.x, aexp);
                        const float i1 = (float)ldexp(lower ? v1.y : v1.x, aexp);
                        float q0, q1;
                        arh[e >> 1] = pack_hi<false>(r0, r1, q0, q1);
                        arl[e >> 1] = pack_lo<false>(q0, q1);
                        aih[e >> 1] = pack_hi<false>(i0, i1, q0, q1);
                        ail[e >> 1] = pack_lo<false>(q0, q1);
                    }
                    xs = aexp + xexp;
                }
            }
            float cs[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) cs[r] = ldexpf((float)S.c[4 * g + r], -xs);
            for (int tt = wave - 1; tt < 16; tt += 3) {
                const int m0 = 16 * tt;
                if (m0 >= M) break;
                f32x4 xr = {0.f, 0.f, 0.f, 0.f}, xi = {0.f, 0.f, 0.f, 0.f};
                if constexpr (!ZF) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float2 hv = S.h[4 * g + r][m0 + col];
                        xr[r] = hv.x;
                        xi[r] = hv.y;
                    }
                } else if constexpr (MODE == 0) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float2 hv = S.h[4 * t + g][m0 + col];
                        xr = mfma4(ar[t], hv.x, xr);
                        xr = mfma4(-ai[t], hv.y, xr);
                        xi = mfma4(ar[t], hv.y, xi);
                        xi = mfma4(ai[t], hv.x, xi);
                    }
                } else {
                    // lane (g, j): [Hr; Hi][8 g .. 8 g + 7][m0 + j], hi/lo split
                    const float* hp = &S.h[8 * (g & 1)][m0 + col].x + (g < 2 ? 0 : 1);
                    u32x4 bh, bl;
#pragma unroll
                    for (int e = 0; e < 8; e += 2) {
                        float q0, q1;
                        bh[e >> 1] = pack_hi<false>(ldexpf(hp[e * 2 * kBbP], xexp),
                                                    ldexpf(hp[(e + 1) * 2 * kBbP], xexp), q0, q1);
                        bl[e >> 1] = pack_lo<false>(q0, q1);
                    }
                    xr = mfma16<false>(arh, bh, xr);
                    xr = mfma16<false>(arl, bh, xr);
                    xr = mfma16<false>(arh, bl, xr);
                    xi = mfma16<false>(aih, bh, xi);
                    xi = mfma16<false>(ail, bh, xi);
                    xi = mfma16<false>(aih, bl, xi);
                }
                // lane (g, c) holds X[4 g + r][m0 + c]
                const bool live = m0 + col < M;
                float pm = 0.0f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float2 wv = make_float2(cs[r] * xr[r], -cs[r] * xi[r]);
                    if (Wt && live && 4 * g + r < K) Wt[r * M + m0] = wv;
                    pm = fmaf(wv.x, wv.x, fmaf(wv.y, wv.y, pm));
                }
                pm = sum_rows4(pm);
                if (g == 0 && live) {
                    if (Pt) Pt[m0] = (double)pm;
                    l21_part += (double)__builtin_amdgcn_sqrtf(pm);   // hardware sqrt, within an ulp
                }
            }
        };
        if (zf)
            tiles(std::true_type{});
        else
            tiles(std::false_type{});
    }
    l21_part = row_sum16(l21_part);   // lanes 16 .. 63 hold zero
    if (lane == 0) S.red[wave] = l21_part;

    __syncthreads();
    // W.
    if (more1) bb_store_h<MODE>(S, hn, mxn, M, tid);
    if (tid == 0) {
        double rs = 0.0;
#pragma unroll
        for (int k = 0; k < kBbK; ++k) rs += k < K ? S.rate[k] : 0.0;
        if (a.rsum) a.rsum[b] = fail ? 0.0 : rs;
        if (a.l21) a.l21[b] = fail ? 0.0 : ((S.red[0] + S.red[1]) + S.red[2]) + S.red[3];
        if (a.info) a.info[b] = fail;
    }
    __syncthreads();
}

// Persistent: workgroup w takes deployments w, w + gridDim.x, ...
template <int MODE, bool HIN>
__global__ __launch_bounds__(kBbThreads) __attribute__((amdgpu_waves_per_eu(3)))
void beamform_batched_kernel(BbDev a) {
    __shared__ BbShared S;
    const int tid = threadIdx.x;
    BbIn in;
    float2 hn[kBbK];
    if (tid < kBbK) S.cpaper[tid] = a.cpaper[tid];
    // H's columns M .. 255 stay zero for the whole launch (lanes m >= M
    // write only the pad column)
#pragma unroll
    for (int i = 0; i < kBbK; ++i) S.h[i][tid] = make_float2(0.0f, 0.0f);
    // the first deployment's channel (the grid has at most B workgroups)
    const int64_t b0 = blockIdx.x;
    bb_fetch<HIN>(a, b0, tid, in, a.K, a.M);
    bb_settle(in);
    if (!HIN && tid < 3 * a.K) S.user[tid / 3][tid - 3 * (tid / 3)] = in.u;
    __syncthreads();
    const float mx0 = bb_synth<MODE, HIN>(a, b0, S, in, a.K, a.M, tid, hn);
    if (b0 + gridDim.x < a.B) {
        bb_fetch<HIN>(a, b0 + gridDim.x, tid, in, a.K, a.M);
        bb_settle(in);
    }
    bb_store_h<MODE>(S, hn, mx0, a.M, tid);
    __syncthreads();
    for (int64_t b = b0; b < a.B; b += gridDim.x) {
        // K, M and the thread index made opaque in every iteration: what is
        // derived from them is formed where it is used instead of held in
        // registers across the loop
        int K = a.K, M = a.M, t = tid;
        asm volatile("" : "+s"(K), "+s"(M), "+v"(t));
        bb_step<MODE, HIN>(a, b, S, in, hn, b + gridDim.x < a.B, b + 2 * (int64_t)gridDim.x < a.B, K, M, t);
    }
}

// dmimo_gram at K <= 16, M <= 256 in FP32 or MIX: G = H H^H of many
// deployments with the products of the fused kernel's step 2.  Persistent
// 256-thread workgroups, four per CU, take deployments blockIdx.x,
// blockIdx.x + grid, ...: thread m holds antenna m's column of the next
// deployment in registers (16 coalesced loads, issued while the current one
// is reduced), puts it in LDS, and every wave forms the partial of its 64
// antennas on the matrix cores; the four partials are added in wave order in
// FP64 and rounded once, the upper triangle mirrored (G exactly Hermitian).
// H is read once, G written once: 8 K M + 8 K^2 bytes per deployment.
struct GmShared {
    union {
        float2 h[kBbK][kBbP];                    // the channel, zero past K and M
        float part[4][2][kBbK][kBbK + 1];        // the waves' partials (over h)
    } u;
    float hmax[4];
};

__device__ __forceinline__ void gm_load(const float2* H, int64_t b, int K, int M, int tid,
                                        float2 (&h)[kBbK]) {
    // clamped indices: every lane loads a valid address, unused values are never read
    const float2* hb = H + b * K * M + (tid < M ? tid : M - 1);
#pragma unroll
    for (int i = 0; i < kBbK; ++i) h[i] = hb[(i < K ? i : K - 1) * M];
}

template <int MODE>
__global__ __launch_bounds__(kBbThreads) __attribute__((amdgpu_waves_per_eu(4)))
void gram_batched_kernel(const float2* __restrict__ H, float2* __restrict__ G, int64_t B, int K,
                         int M) {
    __shared__ GmShared S;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float2 h[kBbK];
    gm_load(H, blockIdx.x, K, M, tid, h);
    for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
        // the column to LDS (zero past K and M) and the wave's largest component
        const bool live = tid < M;
        float mx = 0.0f;
#pragma unroll
        for (int i = 0; i < kBbK; ++i) {
            const float2 v = live && i < K ? h[i] : make_float2(0.0f, 0.0f);
            S.u.h[i][tid] = v;
            if constexpr (MODE == 1) mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
        }
        if constexpr (MODE == 1) {
            mx = wave_max_f(mx);
            if (lane == 0) S.hmax[wave] = mx;
        }
        __syncthreads();
        if (b + gridDim.x < B) gm_load(H, b + gridDim.x, K, M, tid, h);
        // FP16: the largest |h| of the deployment scaled into [2^13, 2^14)
        int hexp = 0;
        if constexpr (MODE == 1) {
            const float m4 = fmaxf(fmaxf(S.hmax[0], S.hmax[1]), fmaxf(S.hmax[2], S.hmax[3]));
            hexp = m4 > 0.0f ? 14 - (ilogbf(m4) + 1) : 0;
        }
        f32x4 gr = {0.f, 0.f, 0.f, 0.f}, gim = {0.f, 0.f, 0.f, 0.f};
        if (64 * wave < M) gram_partial<MODE>(S.u.h, wave, lane, hexp, gr, gim);
        __syncthreads();
        {
            const int g = lane >> 4, j = lane & 15;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                S.u.part[wave][0][4 * g + r][j] = gr[r];
                S.u.part[wave][1][4 * g + r][j] = gim[r];
            }
        }
        __syncthreads();
        // thread (r, c), r <= c < K: entry (r, c) and its mirror
        const int r = tid >> 4, c = tid & 15;
        if (r <= c && c < K) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                re += (double)S.u.part[w][0][r][c];
                im += (double)S.u.part[w][1][r][c];
            }
            const float fr = (float)ldexp(re, -2 * hexp);
            const float fi = r == c ? 0.0f : (float)ldexp(im, -2 * hexp);
            float2* Gb = G + b * K * K;
            Gb[r * K + c] = make_float2(fr, fi);
            if (r != c) Gb[c * K + r] = make_float2(fr, -fi);
        }
        __syncthreads();
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

namespace {

BbDev bb_dev(const BeamformArgs& ba) {
    BbDev d;
    d.w = WaveConst{};
    d.B = ba.B;
    d.K = ba.K;
    d.M = (int)ba.M;
    d.precoder = ba.precoder;
    d.prec = ba.prec;
    d.ap = nullptr;
    d.users = nullptr;
    d.nlos = nullptr;
    d.Hin = nullptr;
    for (int k = 0; k < kBbK; ++k) d.cpaper[k] = std::sqrt(ba.sigma2) * std::sqrt(ba.gamma[k]);
    d.sigma2 = ba.sigma2;
    d.p_total = ba.p_total;
    d.pivot_tol = ba.prec == DMIMO_MIX_BF16X3 ? 1e-4 : 1e-6;
    d.H = nullptr;
    d.W = reinterpret_cast<float2*>(ba.W);
    d.p_ant = ba.p_ant;
    d.l21 = ba.l21;
    d.sinr = ba.sinr;
    d.rsum = ba.rsum;
    d.info = ba.info;
    return d;
}

template <bool HIN>
dmimo_status bb_launch(const BbDev& d, int prec, hipStream_t s) {
    // persistent workgroups: three per CU fit the 51 KB of LDS
    const int64_t wgs = 3 * (int64_t)device_cus();
    const dim3 grid((unsigned)std::min<int64_t>(d.B, wgs)), block(kBbThreads);
    if (prec == DMIMO_MIX_F16X3)
        beamform_batched_kernel<1, HIN><<<grid, block, 0, s>>>(d);
    else if (prec == DMIMO_MIX_BF16X3)
        beamform_batched_kernel<2, HIN><<<grid, block, 0, s>>>(d);
    else
        beamform_batched_kernel<0, HIN><<<grid, block, 0, s>>>(d);
    return check_launch("beamform_batched_kernel");
}

dmimo_status bb_check(const BeamformArgs& ba) {
    if (ba.K < 1 || ba.K > kBbK || ba.M < 1 || ba.M > kBbM)
        return fail(DMIMO_E_SHAPE, "beamform_batched: K <= 16 and M <= 256");
    if (ba.B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "beamform_batched: B too large");
    return DMIMO_OK;
}

}  // namespace

dmimo_status launch_beamform_batched(const BeamformArgs& ba, const WaveConst& w,
                                     const double* ap_xyz, const double* user_xyz,
                                     const void* nlos, void* H, hipStream_t s) {
    if (const dmimo_status st = bb_check(ba)) return st;
    if (ba.B == 0) return DMIMO_OK;
    BbDev d = bb_dev(ba);
    d.w = w;
    d.ap = ap_xyz;
    d.users = user_xyz;
    d.nlos = reinterpret_cast<const float2*>(nlos);
    d.H = reinterpret_cast<float2*>(H);
    return bb_launch<false>(d, ba.prec, s);
}

// dmimo_gram's FP32 and MIX Gram at K <= 16, M <= 256 (G: [B][K][K] complex64).
dmimo_status launch_gram_batched(int64_t B, int K, int64_t M, const void* H, int prec, void* G,
                                 hipStream_t s) {
    if (K < 1 || K > kBbK || M < 1 || M > kBbM)
        return fail(DMIMO_E_SHAPE, "gram_batched: K <= 16 and M <= 256");
    if (B > 0x7fffffff) return fail(DMIMO_E_SHAPE, "gram_batched: B too large");
    if (B == 0) return DMIMO_OK;
    // persistent workgroups: four per CU fit the 33 KB of LDS
    const int64_t wgs = 4 * (int64_t)device_cus();
    const dim3 grid((unsigned)std::min<int64_t>(B, wgs)), block(kBbThreads);
    const float2* h = static_cast<const float2*>(H);
    float2* g = static_cast<float2*>(G);
    if (prec == DMIMO_MIX_F16X3)
        gram_batched_kernel<1><<<grid, block, 0, s>>>(h, g, B, K, (int)M);
    else if (prec == DMIMO_MIX_BF16X3)
        gram_batched_kernel<2><<<grid, block, 0, s>>>(h, g, B, K, (int)M);
    else
        gram_batched_kernel<0><<<grid, block, 0, s>>>(h, g, B, K, (int)M);
    return check_launch("gram_batched_kernel");
}

// The kernel with the channel given (ba.H, [B][K][M] complex64): the MR and
// ZF calls of dmimo_beamform at 8 < K <= 16, M <= 256 in FP32 or MIX.
dmimo_status launch_beamform_batched_h(const BeamformArgs& ba, hipStream_t s) {
    if (const dmimo_status st = bb_check(ba)) return st;
    if (ba.B == 0) return DMIMO_OK;
    BbDev d = bb_dev(ba);
    d.Hin = reinterpret_cast<const float2*>(ba.H);
    return bb_launch<true>(d, ba.prec, s);
}

}  // namespace dmimo
