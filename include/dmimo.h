/*
 * dmimo.h - C ABI of the MI355X (gfx950) distributed-MIMO channel,
 * beamforming and power-map library (libdmimo.so).
 *
 * Notation follows the paper (Sec. II-A): M transmit antennas, K
 * single-antenna users, precoder W in C^{K x M}.  The transmitted vector is
 * x = W^T s and the channel is H in C^{K x M}, so user k receives
 * r_k = sum_m h_km x_m + noise.  Coherent sums multiply h by w with no
 * conjugate, and maximum-ratio precoding is W = H^*.
 *
 * Conventions shared by every call:
 *  - Array arguments are DEVICE pointers owned by the caller, unless the
 *    comment says "host".  The library never frees or keeps them.
 *  - Complex arrays are interleaved (re, im).  They are complex128 (two
 *    doubles) when the call's precision is DMIMO_F64, and complex64 (two
 *    floats) otherwise.  Multi-dimensional arrays are dense and row-major in
 *    the order written, e.g. H[b][k][m].
 *  - Every call is asynchronous and ordered on `stream` (a hipStream_t;
 *    NULL = the legacy default stream).  Nothing synchronises the host.
 *  - The return value reports only what the host can check before launching:
 *    arguments, shapes, precision and workspace size, plus HIP launch errors
 *    (DMIMO_E_HIP, detail in dmimo_last_error()).  Argument errors are
 *    detected before any HIP runtime call is made.
 *  - Numeric failures found on the device go to a per-deployment `info[b]`
 *    (0 = ok, j > 0 = ZF pivot j not positive).  A failed deployment
 *    does not affect the others.
 *  - B = 0 or N = 0 (an empty batch) is valid and launches nothing.
 *  - K and M must be >= 1.  K is at most DMIMO_K_MAX.
 *  - The calls are thread-safe on distinct streams.  No C++ exception
 *    crosses the ABI.
 */
#ifndef DMIMO_H
#define DMIMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DMIMO_K_MAX 32

typedef enum {
    DMIMO_OK = 0,
    DMIMO_E_ARG = 1,          /* NULL required pointer, bad scalar (freq <= 0, sigma2 < 0, ...) */
    DMIMO_E_SHAPE = 2,        /* K < 1, M < 1, K > M for ZF, K > DMIMO_K_MAX, negative B/N, ... */
    DMIMO_E_DTYPE = 3,        /* unknown precision / channel model / precoder / point kind       */
    DMIMO_E_WORKSPACE = 4,    /* workspace smaller than dmimo_workspace_size()                   */
    DMIMO_E_HIP = 5,          /* a HIP runtime call or kernel launch failed                      */
    DMIMO_E_UNSUPPORTED = 6,  /* valid but not provided (e.g. Rician power maps)                 */
    DMIMO_E_BUSY = 7,         /* server: no free slot now                                        */
    DMIMO_E_NOMEM = 8,        /* server: query can never fit the HBM budget                      */
    DMIMO_E_NOTFOUND = 9      /* server: unknown ticket or deployment                            */
} dmimo_status;

/* Arithmetic of a call.  Distances and phases are computed in FP64 in every mode. */
typedef enum {
    DMIMO_F64 = 0,        /* FP64 end to end; complex arrays are complex128           */
    DMIMO_F32 = 1,        /* FP32 amplitude / sin / cos and FP32 contractions          */
    DMIMO_MIX_F16X3 = 2,  /* contractions on FP16 MFMA, hi/lo split x3, FP32 accumulate */
    DMIMO_MIX_BF16X3 = 3  /* contractions on BF16 MFMA, hi/lo split x3, FP32 accumulate */
} dmimo_precision;

typedef enum { DMIMO_CH_LOS = 0, DMIMO_CH_RICIAN = 1 } dmimo_chmodel;

typedef enum {
    DMIMO_MR = 0,        /* W = c H^*                                  */
    DMIMO_ZF = 1,        /* W = scale * conj(G^-1 H), G = H H^H        */
    DMIMO_MR_PHASE = 2,  /* equal-gain MR, w_km = a exp(-j angle h_km) */
    DMIMO_PA = 3         /* PA-consumption-aware (dmimo_pa_precoder); serving only */
} dmimo_precoder;

typedef enum { DMIMO_PTS_GRID = 0, DMIMO_PTS_LIST = 1 } dmimo_points_kind;

/* Channel model.  The paper is silent on geometry; the line-of-sight term is
 * the free-space spherical wave h = lambda/(4 pi max(d, d_min)) exp(-j 2 pi d/lambda),
 * with lambda = 299792458 / freq_hz.  Rician:
 * h = lambda/(4 pi max(d,d_min)) [sqrt(k/(1+k)) exp(-j 2 pi d/lambda) + sqrt(1/(1+k)) g],
 * with g ~ CN(0,1) supplied by the caller. */
typedef struct {
    double freq_hz;      /* carrier frequency (> 0)                              */
    int32_t model;       /* dmimo_chmodel                                        */
    double kappa_lin;    /* Rician K-factor, linear (>= 0); ignored for LoS      */
    double d_min_m;      /* near-field clamp; <= 0 selects lambda / (4 pi)       */
} dmimo_channel_params;

/* Evaluation or user points.
 * GRID: cell centres p(i,j) = (x0 + (i+1/2) dx, y0 + (j+1/2) dy, z), flat index
 *       n = j * nx + i, N = nx * ny.  Shared by every deployment of a call.
 * LIST: `xyz` is a device FP64 array of n points [n][3] per deployment
 *       (dmimo_channel: [B][n][3]; dmimo_powermap: [n][3]). */
typedef struct {
    int32_t kind;            /* dmimo_points_kind              */
    int32_t nx, ny;          /* GRID                           */
    double x0, y0, dx, dy, z;/* GRID                           */
    const double* xyz;       /* LIST, device                   */
    int32_t n;               /* LIST: points per deployment    */
} dmimo_points;

/* Channel synthesis.  H[b][n][m] = h(point n of deployment b, antenna m of
 * deployment b).
 *   params  host; model LoS or Rician.
 *   B, M    deployments and antennas per deployment (B >= 0, M >= 1).
 *   ap_xyz  device FP64 [B][M][3] antenna positions (metres).
 *   pts     host descriptor; N points per deployment.
 *   nlos    Rician only: device complex64 [B][N][M] CN(0,1) draws; NULL for LoS.
 *   out     DMIMO_F64 -> H is complex128, DMIMO_F32 -> complex64 (MIX modes
 *           are not defined for a materialised channel: DMIMO_E_UNSUPPORTED).
 *   H       device [B][N][M] output. */
dmimo_status dmimo_channel(const dmimo_channel_params* params, int32_t B, int32_t M,
                           const double* ap_xyz, const dmimo_points* pts,
                           const void* nlos, int32_t out, void* H, void* stream);

/* K x K Gram G[b] = H[b] H[b]^H (the K x K form of the paper's H^T H^*,
 * Sec. IV).
 *   H    device [B][K][M], complex128 for DMIMO_F64, else complex64.
 *   prec DMIMO_F64: FP64 FMA.  DMIMO_F32: FP32 FMA (FP32 matrix-core products
 *        at 12 < K <= 16, 128 < M <= 256).  MIX modes: hi/lo split FP16 or
 *        BF16 MFMA products with FP32 accumulation.  At K <= 16, M <= 256
 *        (FP32 as above; MIX when K M > 512) the deployment's four 64-antenna
 *        partial sums are added in FP64 and rounded once.
 *   G    device [B][K][K], complex128 for DMIMO_F64, else complex64; full
 *        Hermitian matrix written. */
dmimo_status dmimo_gram(int32_t B, int32_t K, int32_t M, const void* H, int32_t prec,
                        void* G, void* stream);

/* Precoder and its power / SINR epilogues (Sec. II-B, III, VI-B).
 *   precoder  dmimo_precoder.
 *   H         device [B][K][M] (complex128 for DMIMO_F64, else complex64).
 *   gamma_lin host [K] per-user SINR targets (linear); NULL = all ones.  Used by
 *             ZF with p_total <= 0 only.
 *   sigma2    noise power (>= 0).
 *   p_total   > 0: scale W so that ||W||_F^2 = p_total (eq. txpower).  For ZF
 *             every user then has the same SINR.
 *             <= 0: MR uses W = H^*; ZF uses the constraint of eq. (optim1),
 *             H W^T = sqrt(sigma2) D_gamma^{1/2}; equal-gain MR uses |w| = 1.
 *   prec      precision of the Gram (ZF) for K > 8 or M > 256 (M > 128 for
 *             DMIMO_F64); G^-1 (Gauss-Jordan) and G^-1 H are FP64 in every mode.
 *             Smaller deployments run in one kernel that forms G in FP64 from
 *             the stored H and inverts it by FP64 Gauss-Jordan elimination, in
 *             every mode (the MIX modes then equal DMIMO_F32 bit for bit).
 *             ZF calls of at most 64 deployments with at least 8 tiles of 64
 *             antennas (M > 448) also form G in FP64, from per-tile sums
 *             computed in parallel workgroups and added in tile order (MR
 *             calls of that shape sum ||H||_F^2 the same way).
 *             MR and ZF with 8 < K <= 16, M <= 256 in DMIMO_F32 or a MIX mode
 *             run on the kernel of dmimo_beamform_batched with H given (the
 *             same bits as that call on the H it writes): the Gram on the
 *             matrix cores in the precision asked for, G^-1 in FP64, G^-1 H by
 *             FP32 (DMIMO_F32) or split-FP16 (MIX) matrix-core products, and
 *             SINR_k from the gains' identities (ZF: c_k^2 / sigma2; MR: from
 *             G in FP64).
 * Outputs (device; any may be NULL except W):
 *   W      [B][K][M] precoder, same complex type as H.
 *   p_ant  FP64 [B][M]  per-antenna power p_m = sum_k |w_km|^2.
 *   l21    FP64 [B]     ||W||_{2,1} = sum_m sqrt(p_m); consumed PA power is alpha * l21.
 *   sinr   FP64 [B][K]  SINR_k = |A_kk|^2 / (sum_{j!=k} |A_kj|^2 + sigma2), A = H W^T.
 *   rsum   FP64 [B]     sum rate, sum_k log2(1 + SINR_k).
 *   info   int32 [B]    0 ok; j > 0 (ZF): pivot j, the diagonal entry of the
 *                       Schur complement after j - 1 elimination steps (L_jj^2
 *                       of the Cholesky factor), is not above tol * G_jj, tol =
 *                       1e-12 for FP64 input, else 1e-6 (1e-4 with the BF16x3
 *                       Gram); W,
 *                       p_ant, l21, sinr and rsum are zero for that deployment.
 *   ws, ws_bytes  device workspace of at least
 *                 dmimo_workspace_size(DMIMO_CALL_BEAMFORM_ZF, B, K, M, 0, prec) bytes
 *                 for ZF, or of dmimo_workspace_size(DMIMO_CALL_BEAMFORM_MR, ...)
 *                 for MR and equal-gain MR.  The MR size is 0 (NULL accepted)
 *                 except for calls of at most 64 deployments with M > 448, which
 *                 spread each deployment over parallel workgroups of 64 antennas
 *                 and keep per-tile shares there; the ZF size is 0 on the
 *                 batched kernel's shapes above.  A smaller workspace returns
 *                 DMIMO_E_WORKSPACE. */
dmimo_status dmimo_beamform(int32_t precoder, int32_t B, int32_t K, int32_t M,
                            const void* H, const double* gamma_lin, double sigma2,
                            double p_total, int32_t prec, void* W, double* p_ant,
                            double* l21, double* sinr, double* rsum, int32_t* info,
                            void* ws, size_t ws_bytes, void* stream);

/* The batched workload of many small deployments (independent rooms), fused
 * into one launch: for each deployment b, the users' channels
 * H[b] = dmimo_channel(params, ap_xyz[b], users user_xyz[b], nlos[b]) (LoS, or
 * Rician with CN(0,1) draws; the same H bits as dmimo_channel), the precoder
 * of dmimo_beamform (MR or ZF, with its scaling rules) and the epilogues,
 * with the channel kept on chip.  K x K Gram on the matrix cores (DMIMO_F32:
 * FP32 products; MIX modes: FP16 / BF16 hi/lo split products, FP32
 * accumulation), inverse in FP64 (Gauss-Jordan, the pivot test of
 * dmimo_beamform), G^-1 H by FP32 matrix-core products.  SINR_k uses the gains
 * A = H W^T, which for ZF equal D_c (no interference: SINR_k = c_k^2 / sigma2)
 * and for MR c G (Sec. II-A; exact identities of W = conj(G^-1 H) D_c and
 * G = H H^H), the latter formed in FP64.
 *   precoder   DMIMO_MR or DMIMO_ZF.
 *   params     LoS or Rician; nlos: device complex64 [B][K][M] for Rician,
 *              NULL for LoS.
 *   B, K, M    1 <= K <= 16, K <= M for ZF, M <= 256 (larger deployments:
 *              dmimo_channel then dmimo_beamform; DMIMO_E_UNSUPPORTED here).
 *   ap_xyz     device FP64 [B][M][3]; user_xyz device FP64 [B][K][3].
 *   prec       DMIMO_F32, DMIMO_MIX_F16X3 or DMIMO_MIX_BF16X3.
 *   H, W       device complex64 [B][K][M] outputs, each may be NULL (not written).
 *   p_ant, l21, sinr, rsum, info  as for dmimo_beamform, each may be NULL.
 * No workspace.  gamma_lin, sigma2, p_total as for dmimo_beamform. */
dmimo_status dmimo_beamform_batched(int32_t precoder, const dmimo_channel_params* params,
                                    int32_t B, int32_t K, int32_t M, const double* ap_xyz,
                                    const double* user_xyz, const void* nlos,
                                    const double* gamma_lin, double sigma2, double p_total,
                                    int32_t prec, void* H, void* W, double* p_ant, double* l21,
                                    double* sinr, double* rsum, int32_t* info, void* stream);

/* dmimo_beamform for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, bit for bit, with the scratch taken from a
 * static device array of DMIMO_NOALLOC_SCRATCH_BYTES that each GPU holds from
 * the first call on it until the process ends.  Nothing is allocated, and no
 * ws argument is taken.
 *   Every argument and output as for dmimo_beamform.
 *   A call whose workspace (dmimo_workspace_size of dmimo_beamform) exceeds
 *   DMIMO_NOALLOC_SCRATCH_BYTES returns DMIMO_E_WORKSPACE before any launch
 *   (e.g. FP32 ZF with K = 16, M = 300 fits up to B = 4096; K = 16, M <= 256
 *   needs none).
 *   All calls on one device share the array: calls that overlap on one device
 *   (on different streams or host threads) race and must be serialised by the
 *   caller.  No call depends on what an earlier call left in the array. */
#define DMIMO_NOALLOC_SCRATCH_BYTES (8 << 20)
dmimo_status dmimo_beamform_noalloc(int32_t precoder, int32_t B, int32_t K, int32_t M,
                                    const void* H, const double* gamma_lin, double sigma2,
                                    double p_total, int32_t prec, void* W, double* p_ant,
                                    double* l21, double* sinr, double* rsum, int32_t* info,
                                    void* stream);

/* Several precoders of the same channels in one call, as Sec. VI compares MR
 * and ZF (and the PA-aware precoder) on one deployment: precoder p is
 * dmimo_beamform(precoders[p], ...) with every output at offset p of a
 * leading [P] dimension, so that the results equal P separate calls bit for
 * bit.  When every precoder takes the one-pass kernel (K <= 8, M <= 256; 128
 * for DMIMO_F64) the P precoders run side by side in one launch; other shapes
 * make one launch sequence per precoder, in order.
 *   P          0 <= P <= 8 (0: nothing to do); precoders host [P] of
 *              DMIMO_MR, DMIMO_ZF, DMIMO_MR_PHASE.
 *   W          device [P][B][K][M]; p_ant [P][B][M]; l21, rsum, info [P][B];
 *              sinr [P][B][K] (any may be NULL except W).
 *   ws         device workspace of dmimo_beamform_multi_workspace_size(...)
 *              bytes: precoder p's dmimo_workspace_size, each rounded up to
 *              256 B, in order.
 *   Every other argument as for dmimo_beamform; an invalid precoder or shape
 *   in any entry fails the whole call before any launch. */
dmimo_status dmimo_beamform_multi(int32_t P, const int32_t* precoders, int32_t B, int32_t K,
                                  int32_t M, const void* H, const double* gamma_lin,
                                  double sigma2, double p_total, int32_t prec, void* W,
                                  double* p_ant, double* l21, double* sinr, double* rsum,
                                  int32_t* info, void* ws, size_t ws_bytes, void* stream);
/* The users' LoS channels and several precoders of them in one call, the
 * channel synthesis of dmimo_channel and the precoders that Sec. VI compares:
 * H = dmimo_channel(params, B, M, ap_xyz, list points user_xyz,
 * out = DMIMO_F64 if prec is DMIMO_F64 else DMIMO_F32), then
 * dmimo_beamform_multi(P, precoders, ..., H, ...), with the same results bit
 * for bit.  For the one-pass shapes (K <= 8, M <= 256; 128 for DMIMO_F64) one
 * launch does both: each workgroup synthesises its deployment's K x M terms
 * with the channel kernel's arithmetic instead of reading H, and the
 * workgroups of the first precoder write H.  Other shapes launch the channel
 * kernel, then the precoders.
 *   params     LoS model only (DMIMO_E_UNSUPPORTED otherwise).
 *   ap_xyz     device FP64 [B][M][3]; user_xyz device FP64 [B][K][3].
 *   H          device [B][K][M] output, complex FP64 for prec DMIMO_F64, else
 *              complex FP32.
 *   Every other argument, and the workspace, as for dmimo_beamform_multi. */
dmimo_status dmimo_beamform_users(int32_t P, const int32_t* precoders,
                                  const dmimo_channel_params* params, int32_t B, int32_t K,
                                  int32_t M, const double* ap_xyz, const double* user_xyz,
                                  const double* gamma_lin, double sigma2, double p_total,
                                  int32_t prec, void* H, void* W, double* p_ant, double* l21,
                                  double* sinr, double* rsum, int32_t* info, void* ws,
                                  size_t ws_bytes, void* stream);
/* Workspace bytes of dmimo_beamform_multi (0 for an invalid list).  Pure host
 * function. */
size_t dmimo_beamform_multi_workspace_size(int32_t P, const int32_t* precoders, int32_t B,
                                           int32_t K, int32_t M, int32_t prec);

/* Fused channel synthesis and coherent sums at N points.  h[n][m] is never
 * stored.
 *   z_k[n]    = sum_m h[n][m] w_km         (x = W^T s, Sec. II-A)
 *   power[n]  = sum_k |z_k[n]|^2           (for K = 1: |sum_m h w|^2)
 *   sinr[n]   = max_k |z_k|^2 / (sum_{j!=k} |z_j|^2 + sigma2), ties to the lowest k
 *   best_k[n] = the maximising k
 *   per_stream[n][k] = |z_k[n]|^2
 *   params  LoS only (Rician maps: DMIMO_E_UNSUPPORTED).
 *   ap_xyz  device FP64 [M][3].  W device [K][M] (complex128 for DMIMO_F64, else
 *           complex64).
 *   pts     host descriptor (GRID, or LIST of device FP64 [n][3]).
 *   prec    DMIMO_F64: outputs FP64.  DMIMO_F32 and MIX: outputs FP32.
 *   power   required.  sinr, best_k, per_stream may be NULL. */
dmimo_status dmimo_powermap(const dmimo_channel_params* params, int32_t M,
                            const double* ap_xyz, int32_t K, const void* W,
                            const dmimo_points* pts, double sigma2, int32_t prec,
                            void* power, void* sinr, int32_t* best_k, void* per_stream,
                            void* stream);

/* The maps of `maps` precoders of one deployment over the same points in one
 * launch, as Sec. VI compares the coverage of several precoders (MR, ZF, the
 * PA-aware one) on one room: map p is dmimo_powermap of W[p].  Saves the
 * per-launch ramp and drain of every map after the first.  With K <= 8 and
 * 8 < maps K <= 32 in DMIMO_F32 or a MIX mode (K >= 3 for DMIMO_F32), the maps
 * are one contraction of all maps K streams (each channel term synthesised
 * once), whose results equal the single calls to the rounding of the products
 * rather than bit for bit; otherwise they are bitwise the single calls.
 *   maps    0 <= maps <= 65535 (0: nothing to do).
 *   W       device [maps][K][M] (complex128 for DMIMO_F64, else complex64).
 *   power, sinr, best_k  device [maps][N]; per_stream [maps][N][K].
 *   Every other argument, and every output value, as for dmimo_powermap. */
dmimo_status dmimo_powermap_batch(const dmimo_channel_params* params, int32_t M,
                                  const double* ap_xyz, int32_t maps, int32_t K, const void* W,
                                  const dmimo_points* pts, double sigma2, int32_t prec,
                                  void* power, void* sinr, int32_t* best_k, void* per_stream,
                                  void* stream);

/* Proximal gradient descent on the PA-consumption Lagrangian
 * lambda ||W||_{2,1} + ||H W^T - sigma D_gamma^{1/2}||_F^2 (Sec. III eq. l; Sec. IV
 * eq. proxgd), and its deep-unfolded form with per-layer parameters (Sec. V,
 * eq. unfoldednet).  Layer i, with sigma = sqrt(sigma2):
 *   V   = W - eta_i (W H^T H^* - sigma D_gamma^{1/2} H^*)
 *   w_m = (1 - lambda_i eta_i / max(||v_m||, lambda_i eta_i)) v_m   for every antenna m,
 * starting from W(0) = H^* (W0 == NULL) or from W0.
 *   H         device complex64 [B][K][M]; 1 <= K <= 16, 1 <= M <= 256.
 *   gamma_lin host [K] SINR targets (linear), NULL = ones.
 *   layers    I >= 0; lambdas, etas: device FP64 [I] (a constant schedule is
 *             plain PGD; projections onto lambda >= 0 and the eta interval
 *             are the caller's).
 *   W0        device complex64 [B][K][M] or NULL.
 *   prec      DMIMO_F32 (FP32 arithmetic), or DMIMO_MIX_BF16X3 for K <= 8: both
 *             products of the layer on BF16 matrix cores, every operand split
 *             as hi + lo and three products accumulated in FP32 (relative
 *             error near 2^-17 per product); others: DMIMO_E_UNSUPPORTED.
 *   W         device complex64 [B][K][M] output.
 *   l21       device FP64 [B] or NULL: ||W||_{2,1} of the output (PA consumed
 *             power / alpha, eq. effmodel).
 *   rsum      device FP64 [B] or NULL: sum rate of the output, noise sigma2. */
dmimo_status dmimo_pgd(int32_t B, int32_t K, int32_t M, const void* H, const double* gamma_lin,
                       double sigma2, int32_t layers, const double* lambdas, const double* etas,
                       const void* W0, int32_t prec, void* W, double* l21, double* rsum,
                       void* stream);

/* PA-consumption-aware precoder of distributed deployments: eq. (optim1)
 * (Sec. III) solved by PGD / unfolded PGD (Sec. IV-V) on channels of any
 * scale and correlation, in the deployment's own units.  Per deployment:
 *   s = RMS |h_km|, Hn = H / s, L = largest eigenvalue of Hn Hn^H (FP64
 *   power iteration), the layers of dmimo_pgd on Hn with unit noise
 *   (d_k = sqrt(gamma_k)), step eta_i = eta_rel[i] / L, threshold
 *   lambdas[i] eta_i, from W(0) = Hn^*; then W = (sqrt(sigma2) / s) Wn.
 * The back-mapping is exact for the constraint: H W^T = sqrt(sigma2) Hn Wn^T.
 * lambdas keep the meaning they have for unit-variance channels (1/15 in
 * Sec. VI-C); eta_rel = 1 is the largest step of Sec. IV.
 *   H          device complex64 [B][K][M]; 1 <= K <= 32, 1 <= M <= 4096.
 *              K <= 16 and M <= 256: one workgroup per deployment for all
 *              layers.  Larger deployments (e.g. 32 users on 1024 APs): slabs
 *              of 64 antennas, one workgroup each, two launches per layer,
 *              at most 65535 deployments per call.
 *   gamma_lin  host [K] SINR targets (linear) or NULL (ones); sigma2 > 0.
 *   lambdas, eta_rel  device FP64 [layers].
 *   W          device complex64 [B][K][M] output.
 *   p_ant      device FP64 [B][M] or NULL: p_m = sum_k |w_km|^2 (zero for
 *              antennas the precoder switches off).
 *   l21        device FP64 [B] or NULL: ||W||_{2,1} (consumed PA power / alpha).
 *   sinr       device FP64 [B][K] or NULL; rsum device FP64 [B] or NULL.
 *   ws         device workspace of dmimo_workspace_size(DMIMO_CALL_PA_PRECODER,
 *              B, K, M, 0, DMIMO_F32) bytes.
 * An all-zero channel gives W = 0.  prec: DMIMO_F32, or DMIMO_MIX_BF16X3 for
 * K <= 8 and M <= 256 (as in dmimo_pgd). */
dmimo_status dmimo_pa_precoder(int32_t B, int32_t K, int32_t M, const void* H,
                               const double* gamma_lin, double sigma2, int32_t layers,
                               const double* lambdas, const double* eta_rel, int32_t prec,
                               void* W, double* p_ant, double* l21, double* sinr, double* rsum,
                               void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Unsupervised training of the unfolded network (Sec. V; Sec. VI-A).
 *
 * The network is the layer of dmimo_pgd applied I times from W(0) = H^*,
 * with per-layer lambda_i, eta_i.  Its cost on one channel (Sec. V,
 * unsupervised cost) is
 *   C = lam_c ||W(I)||_{2,1} + ||H W(I)^T - sigma D_gamma^{1/2}||_F^2,
 * with lam_c the cost's fixed lambda (1/15 in Sec. VI-C).  Gradients are
 * exact reverse-mode derivatives of the FP32 forward pass; at a prox
 * threshold of 0 the prox is the identity.  K <= 8 (8 < K <= 16:
 * DMIMO_E_UNSUPPORTED), M <= 256, FP32 only.
 * --------------------------------------------------------------------------- */

/* Scratch for dmimo_ufpgd_grad / dmimo_ufpgd_train with B channels (or a
 * batch of B) and I layers: the per-layer tape (pre-prox V and the K x K
 * step operand) plus per-channel gradients.  0 for unsupported shapes. */
size_t dmimo_ufpgd_workspace_size(int32_t B, int32_t K, int32_t M, int32_t layers);

/* Per-channel cost of the network output and its gradient with respect to
 * every lambda_i and eta_i.
 *   B          channels to evaluate; entry b uses channel idx[b] of H, or
 *              channel b when idx == NULL (then n_channels >= B).  An idx entry
 *              outside [0, n_channels) yields cost NaN and zero gradients.
 *   H          device complex64 [n_channels][K][M].
 *   idx        device int32 [B] or NULL.
 *   gamma_lin  host [K] SINR targets (linear) or NULL (ones); sigma2 >= 0.
 *   lambdas, etas  device FP64 [layers], used as given (no projection).
 *   cost       device FP64 [B] or NULL.
 *   dlam, deta device FP64 [B][layers], both or neither.  With neither, only
 *              the forward pass and cost run and ws may be NULL.
 *   ws         device scratch of dmimo_ufpgd_workspace_size(B, K, M, layers). */
dmimo_status dmimo_ufpgd_grad(int32_t B, int32_t n_channels, int32_t K, int32_t M, const void* H,
                              const int32_t* idx, const double* gamma_lin, double sigma2,
                              double lam_c, int32_t layers, const double* lambdas,
                              const double* etas, int32_t prec, double* cost, double* dlam,
                              double* deta, void* ws, size_t ws_bytes, void* stream);

/* Adam hyper-parameters (Kingma and Ba; the paper trains with lr = 1e-3). */
typedef struct {
    double lr;
    double beta1;
    double beta2;
    double eps;
} dmimo_adam_params;

/* `steps` training steps, stream-ordered, no host synchronisation.  Step s:
 *   1. the gradient of the mean cost over the batch idx[s][0..batch-1];
 *   2. one Adam update of [lambda; eta] (bias correction with step number
 *      t0 + s + 1; moments adam_m, adam_v of length 2 layers, lambdas first);
 *   3. the projections lambda_i >= 0, eta_i in [1/(2 L~), 1/L~] with
 *      L~ = (sqrt K + sqrt M)^2 (Sec. V).
 *   lambdas, etas, adam_m, adam_v  device FP64, updated in place.
 *   idx        device int32 [steps][batch], channel indices into H (the
 *              caller draws the epoch permutations).
 *   batch_cost device FP64 [steps] or NULL: mean cost of each step's batch,
 *              before its update.
 *   ws         dmimo_ufpgd_workspace_size(batch, K, M, layers) bytes. */
dmimo_status dmimo_ufpgd_train(int32_t n_channels, int32_t K, int32_t M, const void* H,
                               const double* gamma_lin, double sigma2, double lam_c,
                               int32_t layers, double* lambdas, double* etas, double* adam_m,
                               double* adam_v, int64_t t0, const dmimo_adam_params* opt,
                               int32_t batch, int32_t steps, const int32_t* idx,
                               double* batch_cost, int32_t prec, void* ws, size_t ws_bytes,
                               void* stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of power-map queries on one GPU.
 *
 * A server owns one HIP stream, one worker thread and one device arena of
 * hbm_budget_bytes, allocated at creation; nothing is allocated afterwards.
 * Deployments (antenna positions) are uploaded once and stay resident.
 * Each query:
 *   - names a deployment and brings K user positions (host), a precoder
 *     (MR / ZF / equal-gain MR at p_total, with the same scaling rules as
 *     dmimo_beamform, gamma = 1), the evaluation points and caller-owned
 *     device outputs power[N] and sinr[N] (FP32; sinr may be NULL);
 *   - is admitted when a slot is free and its footprint fits the budget.
 *     The footprint is the server scratch for H, W and the Gram plus the
 *     4 or 8 bytes per point of its maps.
 * The worker then computes the user channel and the precoder, and evaluates
 * the maps in persistent launches.  Each launch loops over tiles of every
 * active query, smallest remaining work first, so queries that arrive while
 * others run share the device from the next launch on.  A query's maps are
 * bitwise identical whether it runs alone or among others.
 * Times are seconds of CLOCK_MONOTONIC.  The output buffers must stay valid
 * until the query is done.
 * -------------------------------------------------------------------------*/
typedef struct dmimo_server dmimo_server;

/* Query states.  FAILED: a ZF query whose pivot test failed (two users at the
 * same place, or nearly collinear channels; dmimo_server_query_info gives the
 * pivot), a launch that failed, or a query that cannot be admitted even with
 * no other query running.  CANCELLED: dmimo_server_cancel before admission.
 * TIMED_OUT: waited for admission longer than the server's queue time-out. */
enum { DMIMO_Q_QUEUED = 0, DMIMO_Q_RUNNING = 1, DMIMO_Q_DONE = 2, DMIMO_Q_FAILED = 3,
       DMIMO_Q_CANCELLED = 4, DMIMO_Q_TIMED_OUT = 5 };

/* Create a server on `device` with an arena of hbm_budget_bytes (>= 1 MiB)
 * and at most max_inflight (1..4096) admitted queries. */
dmimo_status dmimo_server_create(int32_t device, size_t hbm_budget_bytes, int32_t max_inflight,
                                 dmimo_server** srv);
/* Upload a deployment: host FP64 [M][3] antenna positions, LoS params.
 * DMIMO_E_NOMEM if the geometry does not fit the budget. */
dmimo_status dmimo_server_add_deployment(dmimo_server* srv, const dmimo_channel_params* params,
                                         int32_t M, const double* ap_xyz_host, int32_t* dep_id);
/* Queue a power-map query; returns at once with a ticket.  Queries are
 * admitted in arrival order; query scratch comes from the bottom of the
 * arena and resident data (geometry, the DMIMO_PA schedule) from its top, so
 * resident uploads never fragment the space queries draw from.
 *   user_xyz_host  host FP64 [K][3] (copied); 1 <= K <= 32, K <= M for ZF.
 *   pts            GRID, or LIST of device points that outlive the query.
 *   prec           DMIMO_F32, DMIMO_MIX_F16X3 or DMIMO_MIX_BF16X3.
 * DMIMO_E_NOMEM if the query could never fit the budget, DMIMO_E_BUSY if the
 * pending queue (64 x max_inflight) is full, DMIMO_E_NOTFOUND for an unknown
 * deployment. */
dmimo_status dmimo_server_submit(dmimo_server* srv, int32_t dep_id, int32_t K,
                                 const double* user_xyz_host, int32_t precoder,
                                 const dmimo_points* pts, double sigma2, double p_total,
                                 int32_t prec, float* power_out_dev, float* sinr_out_dev,
                                 uint64_t* ticket);
/* State (DMIMO_Q_*) and times of a ticket (t_done is 0 until done). */
dmimo_status dmimo_server_poll(dmimo_server* srv, uint64_t ticket, int32_t* state,
                               double* t_submit, double* t_done);
/* Block until the ticket is done or failed, or timeout_s elapses. */
dmimo_status dmimo_server_wait(dmimo_server* srv, uint64_t ticket, double timeout_s,
                               int32_t* state);
/* Layer schedule of DMIMO_PA queries (eq. optim1 by normalised PGD, as in
 * dmimo_pa_precoder): lambdas and eta_rel, host FP64 [layers], and one SINR
 * target gamma_lin > 0 for every user.  Copied into the server's memory;
 * set once per server, before the first DMIMO_PA query (a second call:
 * DMIMO_E_BUSY).  DMIMO_PA queries need K <= 16, M <= 256, sigma2 > 0, and
 * their p_total is unused. */
dmimo_status dmimo_server_set_pa_schedule(dmimo_server* srv, int32_t layers,
                                          const double* lambdas, const double* eta_rel,
                                          double gamma_lin);
/* Withdraw a query that has not been admitted yet: it ends in
 * DMIMO_Q_CANCELLED and its outputs are never written.  DMIMO_E_BUSY if it was
 * admitted already (admitted work runs to completion) or is finished. */
dmimo_status dmimo_server_cancel(dmimo_server* srv, uint64_t ticket);
/* Queued queries that wait longer than `seconds` for admission end in
 * DMIMO_Q_TIMED_OUT (their outputs are never written); 0 (the default) waits
 * forever.  Applies to queries already queued. */
dmimo_status dmimo_server_set_queue_timeout(dmimo_server* srv, double seconds);
/* The precoder's info word of a finished query: 0, or for a ZF query that
 * ended DMIMO_Q_FAILED the failed pivot j > 0 (as info[b] of dmimo_beamform).
 * 0 while the query is not finished. */
dmimo_status dmimo_server_query_info(dmimo_server* srv, uint64_t ticket, int32_t* info);
/* Forget a finished ticket (DMIMO_E_BUSY if it is not finished). */
dmimo_status dmimo_server_release(dmimo_server* srv, uint64_t ticket);
/* Counters: queries completed, channel terms completed, launches issued,
 * queries queued and running now.  Any pointer may be NULL. */
dmimo_status dmimo_server_stats(dmimo_server* srv, int64_t* completed, int64_t* terms,
                                int64_t* ticks, int32_t* queued, int32_t* running);
/* Finish every submitted query, then free everything. */
dmimo_status dmimo_server_destroy(dmimo_server* srv);

enum { DMIMO_CALL_CHANNEL = 0, DMIMO_CALL_GRAM = 1, DMIMO_CALL_BEAMFORM_MR = 2,
       DMIMO_CALL_BEAMFORM_ZF = 3, DMIMO_CALL_POWERMAP = 4, DMIMO_CALL_PA_PRECODER = 5 };

/* Workspace bytes a call needs (0 if none).  Pure host function. */
size_t dmimo_workspace_size(int32_t call, int32_t B, int32_t K, int32_t M, int32_t N,
                            int32_t prec);

const char* dmimo_status_string(int32_t status);
/* Detail of the last non-OK status on the calling thread (empty if none). */
const char* dmimo_last_error(void);
/* Library version string. */
const char* dmimo_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DMIMO_H */
