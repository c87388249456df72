// Launchers of the device kernels (host functions, one per entry point).
#pragma once

#include "dmimo_internal.h"

namespace dmimo {

dmimo_status launch_channel(const WaveConst& w, const PointsDev& P, bool rician, int64_t B,
                            int64_t M, const double* ap, const void* nlos, bool f64, void* H,
                            hipStream_t s);

dmimo_status launch_gram(int64_t B, int K, int64_t M, const void* H, int prec, void* G,
                         hipStream_t s);

struct BeamformArgs {
    int precoder;
    int64_t B;
    int K;
    int64_t M;
    const void* H;
    double gamma[DMIMO_K_MAX];
    double sigma2;
    double p_total;
    int prec;
    void* W;
    double* p_ant;
    double* l21;
    double* sinr;
    double* rsum;
    int32_t* info;
    void* ws;
};

dmimo_status launch_beamform(const BeamformArgs& a, hipStream_t s);
// Workspace of a launch_beamform call.  ZF: the Gram, plus the wide path's
// G^-1 and per-tile shares when that path applies (few deployments, many
// antennas).  MR and equal-gain MR: the wide path's per-tile shares, else 0.
size_t beamform_workspace_bytes(int precoder, int64_t B, int K, int64_t M, int prec);
// precoders[0 .. P) of the same channels (1 <= P <= 8): outputs of precoder p at
// offset p of a leading [P] dimension, workspace slices in order, each rounded
// up to 256 B.  One launch when every precoder takes the one-pass kernel
// (precoder p on grid row p), else one launch_beamform per precoder.
dmimo_status launch_beamform_multi(const BeamformArgs& a, int P, const int* precoders, hipStream_t s);
size_t beamform_multi_workspace_bytes(int P, const int* precoders, int64_t B, int K, int64_t M,
                                      int prec);
// launch_beamform_multi of the users' LoS channels, H ([B][K][M], a.H) written
// by the call: for the one-pass shapes synthesised inside the precoder kernel
// (the channel kernel's terms, the same bits), else by the channel kernel first.
dmimo_status launch_beamform_users(const BeamformArgs& a, int P, const int* precoders,
                                   const WaveConst& w, const double* ap_xyz, const double* user_xyz,
                                   hipStream_t s);
// The users' channels (LoS, or Rician with nlos [B][K][M]), MR or ZF and the
// epilogues of many small deployments in one launch (K <= 16, M <= 256;
// FP32 or MIX precision): H ([B][K][M], optional) and a.W optional, no
// workspace.
dmimo_status launch_beamform_batched(const BeamformArgs& a, const WaveConst& w,
                                     const double* ap_xyz, const double* user_xyz,
                                     const void* nlos, void* H, hipStream_t s);

// `maps` precoders over the same antennas and points, one launch: W
// [maps][K][M], every output [maps][N] ([maps][N][K] per stream); map p is
// grid row p (blockIdx.y) of every map kernel.
struct PowermapArgs {
    WaveConst w;
    PointsDev P;
    int M;
    int K;
    int maps = 1;
    const double* ap;
    const void* W;
    double sigma2;
    int prec;
    void* power;
    void* sinr;
    int32_t* best_k;
    void* per_stream;
};

dmimo_status launch_powermap(const PowermapArgs& a, hipStream_t s);

dmimo_status launch_pgd(int64_t B, int K, int M, const void* H, const double* gamma, double sigma2,
                        int layers, const double* lambdas, const double* etas, const void* W0,
                        void* W, double* l21, double* rsum, int prec, hipStream_t s);

// {1/s, 1/lambda_max(Hn Hn^H)} per channel into pa [B][2] (K <= 32)
dmimo_status launch_pa_prepare(int64_t B, int K, int M, const void* H, double* pa, hipStream_t s);

// workspace of the slab path of the PA precoder (K > 16 or M > 256), after
// the [B][2] normalisation factors
size_t pa_large_workspace_bytes(int64_t B, int K, int M);

// the slab path (K <= 32, M <= 4096): ws holds the [B][2] factors, then at
// byte pa_bytes the partials and E
dmimo_status launch_pa_large(int64_t B, int K, int M, const void* H, const double* gamma,
                             double sigma2, int layers, const double* lambdas, const double* eta_rel,
                             void* W, double* p_ant, double* l21, double* sinr, double* rsum,
                             void* ws, size_t pa_bytes, hipStream_t s);

// ws: [B][2] FP64 normalisation factors, written here
dmimo_status launch_pa_precoder(int64_t B, int K, int M, const void* H, const double* gamma,
                                double sigma2, int layers, const double* lambdas,
                                const double* eta_rel, void* W, double* p_ant, double* l21,
                                double* sinr, double* rsum, void* ws, int prec, hipStream_t s);

struct UfpgdArgs {
    int64_t B;              // channels per launch (the batch)
    int K, M, layers, n_channels;
    const void* H;          // complex64 [n_channels][K][M]
    const int32_t* idx;     // [B] channel of each batch entry, or NULL (entry b = channel b)
    const double* gamma;    // host [K] or NULL
    double sigma2, lam_c;
    const double* lambdas;  // device [layers]
    const double* etas;
};

struct UfpgdTrainArgs {
    double* lambdas;        // device [layers], updated in place
    double* etas;
    double* adam_m;         // device [2 layers]
    double* adam_v;
    int64_t t0;             // Adam steps already taken
    double lr, beta1, beta2, eps;
    int64_t steps;
    const int32_t* idx;     // device [steps][B]
    double* batch_cost;     // device [steps] or NULL
};

size_t ufpgd_workspace_bytes(int64_t B, int M, int layers);
dmimo_status launch_ufpgd_grad(const UfpgdArgs& g, double* cost, double* dlam, double* deta,
                               void* ws, hipStream_t s);
dmimo_status launch_ufpgd_train(const UfpgdArgs& g, const UfpgdTrainArgs& t, void* ws,
                                hipStream_t s);

}  // namespace dmimo
