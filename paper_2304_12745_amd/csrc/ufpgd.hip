// Unsupervised training of the unfolded PGD network (Sec. V, unsupervised
// cost; Sec. VI-A, Adam with projections), K <= 8 users, M <= 256 antennas.
//
// ufpgd_grad_kernel: one workgroup per channel of the batch, ceil(M / 64)
// waves.  Forward through the I layers exactly as the inference kernel, but
// taping each layer's pre-prox V (output layout, 16 floats per lane) and its
// embedded (A - D) operand (4 floats per lane, wave 0).  Then the cost
//   C = lambda_c ||W||_{2,1} + ||X||_F^2,   X = W H^T - D   (= R^T),
// its cotangent Gbar = 2 X H^* + lambda_c w_m / ||w_m||, and the reverse pass
// per layer i = I-1 .. 0 (cotangent Gbar = dC/dRe + j dC/dIm):
//   prox:  n = ||v_m||, t = lambda eta, rho = Re(v^H gbar):
//          gv = (1 - t/n) gbar + (t rho / n^3) v  for n > t, else 0
//          (identity at t = 0);  dC/dt -= rho / n
//   step:  A' = Gv H^T (MFMA, as step 1);  Gbar = Gv - eta A' H^* (as step 2)
//          dC/deta_step = -Re sum conj(Gv) ((A - D) H^*) = -Re sum_kj X_kj conj(A'_kj),
//          read off the two embedded operands as -1/2 sum(E .* E').
//   dC/dlambda = eta dC/dt,  dC/deta = dC/deta_step + lambda dC/dt.
// The reverse pass costs the same three MFMA products as two forward layers.
//
// ufpgd_adam_kernel: batch mean of the per-channel gradients (fixed order,
// one wave per parameter),
// one Adam update (Kingma and Ba, Algorithm 1) of [lambda; eta] in FP64, then
// the projections lambda >= 0 and eta in [1/(2 L~), 1/L~], L~ = (sqrt K + sqrt M)^2.
#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "pgd_mfma.h"

namespace dmimo {

namespace {

struct UfpgdDev {
    int K, M, layers, n_channels;
    const float2* H;
    const int32_t* idx;
    const double* lambdas;
    const double* etas;
    float d[8];
    float lam_c;        // cotangent
    double lam_cd;      // cost value
    float* tapeV;       // [B][I][nw][64][16], NULL: cost only
    float* tapeE;       // [B][I][64][4]
    double* cost;       // [B] or NULL
    double* dlam;       // [B][I]
    double* deta;       // [B][I]
};

__device__ __forceinline__ double wave_sum_d(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

template <int AW, int NW>
__global__ __launch_bounds__(64 * NW) void ufpgd_grad_kernel(UfpgdDev a) {
    constexpr int nw = NW;
    constexpr int NQ = AW / 16;                // 16-antenna blocks per wave
    constexpr int TV = AW / 4;                 // tape floats per lane and layer
    extern __shared__ float smem[];
    const int stride = pl_stride(AW * NW);
    float* sX = smem;                                   // [16][stride]
    float* sD = smem + 16 * stride;                     // [2][nw][16][17]
    double* sT = reinterpret_cast<double*>(sD + 2 * nw * kPartFloats);   // [2][nw]

    const PgdLane<AW> L;
    const int64_t b = blockIdx.x;
    const int K = a.K, M = a.M, I = a.layers;
    const int64_t ch = a.idx ? (int64_t)a.idx[b] : b;
    if (ch < 0 || ch >= a.n_channels) {                // uniform over the block
        if (L.tid == 0 && a.cost) a.cost[b] = __builtin_nan("");
        if (a.tapeV)
            for (int i = L.tid; i < I; i += blockDim.x) a.dlam[b * I + i] = a.deta[b * I + i] = 0.0;
        return;
    }
    const float2* Hb = a.H + ch * K * M;
    const bool grad = a.tapeV != nullptr;

    load_planar<AW / 8>(sX, stride, AW * nw, Hb, K, M, false);
    __syncthreads();
    float HA[AW / 4], HB[NQ][4];
    read_op_a(sX, stride, L, HA);
    read_op_b2(sX, stride, L, HB);
    __syncthreads();
    load_planar<AW / 8>(sX, stride, AW * nw, Hb, K, M, true);  // W(0) = H^*
    __syncthreads();
    float WD[NQ][4], WA[AW / 4];
    read_out_d(sX, stride, L, WD);
    read_op_a(sX, stride, L, WA);
    const float dg = a.d[L.lo & 7];
    int ph = 0;

    // forward, taping V and (A - D)
    for (int i = 0; i < I; ++i) {
        const float eta = (float)a.etas[i];
        const float thr = (float)(a.lambdas[i] * a.etas[i]);
        put_partial(sD + (ph * nw + L.wave) * kPartFloats, L, d1_partial<AW>(WA, HA));
        __syncthreads();
        float E[4];
        embed_operand<NW>(sD + ph * nw * kPartFloats, L, dg, E);
        ph ^= 1;
        if (grad && L.wave == 0)
            *reinterpret_cast<float4*>(a.tapeE + ((b * I + i) * 64 + L.lane) * 4) =
                make_float4(E[0], E[1], E[2], E[3]);
        float* tv = grad ? a.tapeV + (((b * I + i) * nw + L.wave) * 64 + L.lane) * TV : nullptr;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const f32x4 g = apply_block(E, HB, q);
            float v[4];
            float n2 = 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[r] = fmaf(-eta, g[r], WD[q][r]);
                n2 = fmaf(v[r], v[r], n2);
            }
            if (grad) *reinterpret_cast<float4*>(tv + 4 * q) = make_float4(v[0], v[1], v[2], v[3]);
            const float sc = prox_scale(col_norm(column_sum(n2)), thr);
#pragma unroll
            for (int r = 0; r < 4; ++r) WD[q][r] = sc * v[r];
        }
        write_out_d(sX, stride, L, WD);
        wave_lds_sync();
        read_op_a(sX, stride, L, WA);
    }

    // cost and its cotangent
    float nrm[NQ];
    double l21 = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        float n2 = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) n2 = fmaf(WD[q][r], WD[q][r], n2);
        nrm[q] = col_norm(column_sum(n2));
        if (L.hi == 0) l21 += nrm[q];
    }
    l21 = wave_sum_d(l21);
    if (L.lane == 0) sT[ph * nw + L.wave] = l21;
    put_partial(sD + (ph * nw + L.wave) * kPartFloats, L, d1_partial<AW>(WA, HA));
    __syncthreads();
    float E[4];
    embed_operand<NW>(sD + ph * nw * kPartFloats, L, dg, E);
    double fro = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) fro += (double)E[s] * E[s];
    fro = wave_sum_d(fro);
    if (L.tid == 0 && a.cost) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += sT[ph * nw + w];
        a.cost[b] = a.lam_cd * t + 0.5 * fro;
    }
    ph ^= 1;
    if (!grad) return;

    float Gb[NQ][4];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const f32x4 g = apply_block(E, HB, q);
        const float inv = nrm[q] > 0.0f ? a.lam_c * __builtin_amdgcn_rcpf(nrm[q]) : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) Gb[q][r] = fmaf(2.0f, g[r], inv * WD[q][r]);
    }

    // reverse pass
    for (int i = I - 1; i >= 0; --i) {
        const double lam_d = a.lambdas[i], eta_d = a.etas[i];
        const float eta = (float)eta_d;
        const float t = (float)(lam_d * eta_d);
        const float* tv = a.tapeV + (((b * I + i) * nw + L.wave) * 64 + L.lane) * TV;
        float Gv[NQ][4];
        double dtp = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float4 vv = *reinterpret_cast<const float4*>(tv + 4 * q);
            const float v[4] = {vv.x, vv.y, vv.z, vv.w};
            float n2 = 0.0f, rho = 0.0f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                n2 = fmaf(v[r], v[r], n2);
                rho = fmaf(Gb[q][r], v[r], rho);
            }
            n2 = column_sum(n2);
            rho = column_sum(rho);
            const float n = col_norm(n2);
            if (n > t) {
                const float inv = __builtin_amdgcn_rcpf(n);
                const float s = 1.0f - t * inv;
                const float coef = t * rho * inv * inv * inv;
#pragma unroll
                for (int r = 0; r < 4; ++r) Gv[q][r] = fmaf(s, Gb[q][r], coef * v[r]);
                if (L.hi == 0) dtp -= (double)rho * inv;
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) Gv[q][r] = t == 0.0f ? Gb[q][r] : 0.0f;
            }
        }
        dtp = wave_sum_d(dtp);
        write_out_d(sX, stride, L, Gv);
        wave_lds_sync();
        float GA[AW / 4];
        read_op_a(sX, stride, L, GA);
        put_partial(sD + (ph * nw + L.wave) * kPartFloats, L, d1_partial<AW>(GA, HA));
        if (L.lane == 0) sT[ph * nw + L.wave] = dtp;
        __syncthreads();
        float E2[4];                                     // A' = Gv H^T, embedded, no shift
        embed_operand<NW>(sD + ph * nw * kPartFloats, L, 0.0f, E2);
        if (L.wave == 0) {
            const float4 ee = *reinterpret_cast<const float4*>(a.tapeE + ((b * I + i) * 64 + L.lane) * 4);
            double de = (double)ee.x * E2[0] + (double)ee.y * E2[1] + (double)ee.z * E2[2] +
                        (double)ee.w * E2[3];
            de = wave_sum_d(de);
            if (L.lane == 0) {
                double dt = 0.0;
                for (int w = 0; w < nw; ++w) dt += sT[ph * nw + w];
                a.dlam[b * I + i] = eta_d * dt;
                a.deta[b * I + i] = -0.5 * de + lam_d * dt;
            }
        }
        ph ^= 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const f32x4 g = apply_block(E2, HB, q);
#pragma unroll
            for (int r = 0; r < 4; ++r) Gb[q][r] = fmaf(-eta, g[r], Gv[q][r]);
        }
    }
}

struct AdamDev {
    int I, B;
    double lr, beta1, beta2, eps;
    double eta_lo, eta_hi;
    double* lambdas;
    double* etas;
    double* m;          // [2I]
    double* v;          // [2I]
    const double* dlam; // [B][I]
    const double* deta;
    const double* cost; // [B]
};

// One wave per parameter (waves stride over the 2I parameters): lanes sum
// the batch entries b = lane, lane + 64, ... in order, then a fixed xor tree;
// the result does not depend on timing.
__device__ __forceinline__ double batch_mean(const double* src, int stride, int B, int lane) {
    double s = 0.0;
    for (int b = lane; b < B; b += 64) s += src[(int64_t)b * stride];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s / B;
}

__global__ __launch_bounds__(1024) void ufpgd_adam_kernel(AdamDev a, int64_t t, double* batch_cost) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int n = 2 * a.I;
    const double bc1 = 1.0 - pow(a.beta1, (double)t);
    const double bc2 = 1.0 - pow(a.beta2, (double)t);
    for (int j = wave; j < n; j += nwaves) {
        const bool is_lam = j < a.I;
        const int col = is_lam ? j : j - a.I;
        const double g = batch_mean((is_lam ? a.dlam : a.deta) + col, a.I, a.B, lane);
        if (lane == 0) {
            const double m = a.beta1 * a.m[j] + (1.0 - a.beta1) * g;
            const double v = a.beta2 * a.v[j] + (1.0 - a.beta2) * g * g;
            a.m[j] = m;
            a.v[j] = v;
            double* p = is_lam ? a.lambdas + col : a.etas + col;
            double x = *p - a.lr * (m / bc1) / (sqrt(v / bc2) + a.eps);
            x = is_lam ? fmax(x, 0.0) : fmin(fmax(x, a.eta_lo), a.eta_hi);
            *p = x;
        }
    }
    if (wave == nwaves - 1 && batch_cost) {
        const double c = batch_mean(a.cost, 1, a.B, lane);
        if (lane == 0) *batch_cost = c;
    }
}

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct UfpgdWs {
    size_t tapeV, tapeE, dlam, deta, cost, total;
};

UfpgdWs ufpgd_ws_layout(int64_t B, int M, int layers) {
    // the tape of V has M rounded up to the antennas of the waves (any AW)
    // times 16 floats per 4 antennas (64 lanes x AW/4 floats per AW antennas)
    const int aw = pgd_antennas_per_wave(B, M);
    const int nw = (M + aw - 1) / aw;
    UfpgdWs w;
    size_t off = 0;
    w.tapeV = off;
    off = align_up(off + sizeof(float) * (size_t)B * layers * nw * 64 * (aw / 4));
    w.tapeE = off;
    off = align_up(off + sizeof(float) * (size_t)B * layers * 64 * 4);
    w.dlam = off;
    off = align_up(off + sizeof(double) * (size_t)B * layers);
    w.deta = off;
    off = align_up(off + sizeof(double) * (size_t)B * layers);
    w.cost = off;
    off = align_up(off + sizeof(double) * (size_t)B);
    w.total = off;
    return w;
}

size_t ufpgd_lds_bytes(int aw, int nw) { return pgd_mfma_lds_bytes(aw, nw) + sizeof(double) * 2 * nw; }

template <int AW>
void launch_grad_aw(const UfpgdDev& d, dim3 grid, int nw, hipStream_t s) {
    const size_t lds = ufpgd_lds_bytes(AW, nw);
    switch (nw) {
        case 1: ufpgd_grad_kernel<AW, 1><<<grid, dim3(64), lds, s>>>(d); break;
        case 2: ufpgd_grad_kernel<AW, 2><<<grid, dim3(128), lds, s>>>(d); break;
        case 3: ufpgd_grad_kernel<AW, 3><<<grid, dim3(192), lds, s>>>(d); break;
        default: ufpgd_grad_kernel<AW, 4><<<grid, dim3(256), lds, s>>>(d); break;
    }
}

// The antennas per wave follow pgd_antennas_per_wave(B, M), the same choice
// the workspace layout makes.
void launch_grad(const UfpgdDev& d, int64_t B, hipStream_t s) {
    const dim3 grid((unsigned)B);
    const int aw = pgd_antennas_per_wave(B, d.M);
    const int nw = (d.M + aw - 1) / aw;
    if (aw == 16) launch_grad_aw<16>(d, grid, nw, s);
    else if (aw == 32) launch_grad_aw<32>(d, grid, nw, s);
    else launch_grad_aw<64>(d, grid, nw, s);
}

UfpgdDev make_dev(const UfpgdArgs& g) {
    UfpgdDev d;
    d.K = g.K;
    d.M = g.M;
    d.layers = g.layers;
    d.n_channels = g.n_channels;
    d.H = reinterpret_cast<const float2*>(g.H);
    d.idx = g.idx;
    d.lambdas = g.lambdas;
    d.etas = g.etas;
    const double sigma = std::sqrt(g.sigma2);
    for (int k = 0; k < 8; ++k)
        d.d[k] = k < g.K ? (float)(sigma * std::sqrt(g.gamma ? g.gamma[k] : 1.0)) : 0.0f;
    d.lam_c = (float)g.lam_c;
    d.lam_cd = g.lam_c;
    d.tapeV = d.tapeE = nullptr;
    d.cost = d.dlam = d.deta = nullptr;
    return d;
}

}  // namespace

size_t ufpgd_workspace_bytes(int64_t B, int M, int layers) {
    return ufpgd_ws_layout(B, M, layers).total;
}

dmimo_status launch_ufpgd_grad(const UfpgdArgs& g, double* cost, double* dlam, double* deta,
                               void* ws, hipStream_t s) {
    UfpgdDev d = make_dev(g);
    d.cost = cost;
    if (dlam) {
        const UfpgdWs w = ufpgd_ws_layout(g.B, g.M, g.layers);
        char* base = static_cast<char*>(ws);
        d.tapeV = reinterpret_cast<float*>(base + w.tapeV);
        d.tapeE = reinterpret_cast<float*>(base + w.tapeE);
        d.dlam = dlam;
        d.deta = deta;
    }
    launch_grad(d, g.B, s);
    return check_launch("ufpgd_grad_kernel");
}

dmimo_status launch_ufpgd_train(const UfpgdArgs& g, const UfpgdTrainArgs& t, void* ws,
                                hipStream_t s) {
    const UfpgdWs w = ufpgd_ws_layout(g.B, g.M, g.layers);
    char* base = static_cast<char*>(ws);
    UfpgdDev d = make_dev(g);
    d.tapeV = reinterpret_cast<float*>(base + w.tapeV);
    d.tapeE = reinterpret_cast<float*>(base + w.tapeE);
    d.dlam = reinterpret_cast<double*>(base + w.dlam);
    d.deta = reinterpret_cast<double*>(base + w.deta);
    d.cost = reinterpret_cast<double*>(base + w.cost);

    AdamDev a;
    a.I = g.layers;
    a.B = (int)g.B;
    a.lr = t.lr;
    a.beta1 = t.beta1;
    a.beta2 = t.beta2;
    a.eps = t.eps;
    const double Lt = (std::sqrt((double)g.K) + std::sqrt((double)g.M)) * (std::sqrt((double)g.K) + std::sqrt((double)g.M));
    a.eta_lo = 1.0 / (2.0 * Lt);
    a.eta_hi = 1.0 / Lt;
    a.lambdas = t.lambdas;
    a.etas = t.etas;
    a.m = t.adam_m;
    a.v = t.adam_v;
    a.dlam = d.dlam;
    a.deta = d.deta;
    a.cost = d.cost;
    const int adam_threads = 64 * std::min(16, 2 * g.layers);
    for (int64_t step = 0; step < t.steps; ++step) {
        d.idx = t.idx + step * g.B;
        launch_grad(d, g.B, s);
        ufpgd_adam_kernel<<<dim3(1), dim3(adam_threads), 0, s>>>(a, t.t0 + step + 1,
                                                        t.batch_cost ? t.batch_cost + step : nullptr);
    }
    return check_launch("ufpgd_train");
}

}  // namespace dmimo
