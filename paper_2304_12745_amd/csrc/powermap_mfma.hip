// Power maps with the K-stream contraction on the matrix cores: one launch
// per map.  The per-workgroup bodies (and the description of the method) are
// in powermap_body.h.
#include "powermap_body.h"
#include "powermap_mfma.h"

namespace dmimo {

namespace {

template <int NT, int PT, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void powermap_mfma_kernel(PmMapDev a) {
    __shared__ __attribute__((aligned(16))) char smem[f32_lds_bytes<NT, PT, WAVES>()];
    map_f32_wg<NT, PT, WAVES>(map_of(a, blockIdx.y), (int64_t)blockIdx.x * (WAVES * 16 * PT), smem);
}

template <int NT, int PT, bool BF16, int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(4))) void powermap_x3_kernel(PmMapDev a) {
    __shared__ __attribute__((aligned(16))) char smem[x3_lds_bytes<NT, PT, WAVES>()];
    __shared__ float s_red[WAVES];
    map_x3_wg<NT, PT, BF16, WAVES>(map_of(a, blockIdx.y), (int64_t)blockIdx.x * (WAVES * 16 * PT), smem,
                                   s_red);
}

// The split-precision map for K > 8 (map_x3w_wg): PT tiles of 16 points per
// wave, WAVES waves per workgroup, at least OCC waves per SIMD.
#ifndef DMIMO_X3W_PT
#define DMIMO_X3W_PT 2
#endif
#ifndef DMIMO_X3W_WAVES
#define DMIMO_X3W_WAVES 8
#endif
#ifndef DMIMO_X3W_OCC
#define DMIMO_X3W_OCC 2
#endif
constexpr int kX3wPt = DMIMO_X3W_PT;
constexpr int kX3wWaves = DMIMO_X3W_WAVES;

template <int NT, int PT, bool BF16, int WAVES>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(DMIMO_X3W_OCC)))
void powermap_x3w_kernel(PmMapDev a) {
    __shared__ __attribute__((aligned(16))) char smem[x3w_lds_bytes<NT, PT, WAVES>()];
    map_x3w_wg<NT, PT, BF16, WAVES>(map_of(a, blockIdx.y), (int64_t)blockIdx.x * (WAVES * 16 * PT),
                                    smem);
}

#ifndef DMIMO_PM_WAVES
#define DMIMO_PM_WAVES 8   // wavefronts per workgroup of the map kernels (measured best of 4, 8, 16)
#endif
constexpr int kWaves = DMIMO_PM_WAVES;

template <int PT, typename F>
dmimo_status launch_blocks(const PmMapDev& d, int maps, F&& launch) {
    const int64_t blocks = ceil_div(d.P.n, kWaves * 16 * PT);
    if (blocks > 0x7fffffff) return fail(DMIMO_E_SHAPE, "powermap: too many points");
    launch(dim3((unsigned)blocks, (unsigned)maps));
    return check_launch("powermap_mfma");
}

template <int NT>
dmimo_status launch_f32(const PmMapDev& d, int maps, hipStream_t s) {
    // four 16-point tiles per wave at K <= 8 (measured 6% faster than two)
    constexpr int PT = NT == 1 ? 4 : 2;
    return launch_blocks<PT>(
        d, maps, [&](dim3 g) { powermap_mfma_kernel<NT, PT, kWaves><<<g, 64 * kWaves, 0, s>>>(d); });
}

template <int NT, bool BF16>
dmimo_status launch_x3w(const PmMapDev& d, int maps, hipStream_t s) {
    const int64_t blocks = ceil_div(d.P.n, kX3wWaves * 16 * kX3wPt);
    if (blocks > 0x7fffffff) return fail(DMIMO_E_SHAPE, "powermap: too many points");
    powermap_x3w_kernel<NT, kX3wPt, BF16, kX3wWaves>
        <<<dim3((unsigned)blocks, (unsigned)maps), 64 * kX3wWaves, 0, s>>>(d);
    return check_launch("powermap_x3w");
}

template <int NT, bool BF16>
dmimo_status launch_x3(const PmMapDev& d, int maps, hipStream_t s) {
    // one 16-point tile per wave for K > 8 keeps the kernel within 128 VGPRs
    // (4 waves per SIMD) without spills
    constexpr int PT = NT == 1 ? 2 : 1;
    return launch_blocks<PT>(
        d, maps, [&](dim3 g) { powermap_x3_kernel<NT, PT, BF16, kWaves><<<g, 64 * kWaves, 0, s>>>(d); });
}

}  // namespace

// Several maps of K <= 8 streams each (8 < maps K <= 32) run as one contraction
// of maps K streams (W [maps][K][M] is [maps K][M]), whose epilogue splits the
// streams into the maps: every channel term is synthesised once for all maps.
static bool joint_maps(const PowermapArgs& a) { return a.maps > 1 && a.K <= 8 && a.maps * a.K > 8 && a.maps * a.K <= 32; }

static PmMapDev joint_dev(const PowermapArgs& a) {
    PmMapDev d = make_map_dev(a);
    d.K = a.maps * a.K;
    d.G = a.K;
    return d;
}

dmimo_status launch_powermap_f32_mfma(const PowermapArgs& a, hipStream_t s) {
    if (joint_maps(a)) {
        const PmMapDev d = joint_dev(a);
        return d.K <= 16 ? launch_f32<2>(d, 1, s) : launch_f32<4>(d, 1, s);
    }
    const PmMapDev d = make_map_dev(a);
    if (a.K <= 8) return launch_f32<1>(d, a.maps, s);
    if (a.K <= 16) return launch_f32<2>(d, a.maps, s);
    return launch_f32<4>(d, a.maps, s);
}

dmimo_status launch_powermap_mfma(const PowermapArgs& a, hipStream_t s) {
    if (joint_maps(a)) {
        const PmMapDev d = joint_dev(a);
        if (a.prec == DMIMO_MIX_BF16X3)
            return d.K <= 16 ? launch_x3w<2, true>(d, 1, s) : launch_x3w<4, true>(d, 1, s);
        return d.K <= 16 ? launch_x3w<2, false>(d, 1, s) : launch_x3w<4, false>(d, 1, s);
    }
    const PmMapDev d = make_map_dev(a);
    if (a.prec == DMIMO_MIX_BF16X3) {
        if (a.K <= 8) return launch_x3<1, true>(d, a.maps, s);
        if (a.K <= 16) return launch_x3w<2, true>(d, a.maps, s);
        return launch_x3w<4, true>(d, a.maps, s);
    }
    if (a.K <= 8) return launch_x3<1, false>(d, a.maps, s);
    if (a.K <= 16) return launch_x3w<2, false>(d, a.maps, s);
    return launch_x3w<4, false>(d, a.maps, s);
}

}  // namespace dmimo
