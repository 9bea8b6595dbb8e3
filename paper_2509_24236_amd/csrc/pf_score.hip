// Particle scoring for gfx950: the fitness equation of Sec. III-B evaluated for many poses.
//
// E_k = (1/|X_k|) sum_{x in X_k} |T(R_k x + t_k)|, T the trilinear interpolation of the 8 voxel
// centres around the point, x in X_k iff the stencil is inside the grid and all 8 stored values
// have |T| < 1 ("valid grids": observed and within the truncation band), E_k = 1 if X_k = {}.
//
// Work decomposition: a workgroup owns TK consecutive poses and sweeps every point; each lane
// keeps one point's camera coordinates in registers and evaluates it against the TK poses, so
// the point load is amortised over TK gathers and the poses are uniform across the wave
// (scalar registers). All lanes of a wave touch 64 consecutive points of the raster-ordered
// cloud, so their 8-corner stencils fall in nearby voxels. A workgroup covers all points of its
// poses, so the (sum, count) of each pose is reduced once, inside the workgroup, in a fixed
// order: results are bitwise reproducible and no cross-workgroup pass is needed.
//
// The point set is HBM/L2-bound gather work (8 x 4 B per sample for FP32 storage), not a
// contraction, so it runs on the vector ALUs, not on the matrix cores.
#include <math.h>

#include <atomic>

#include "pf_score_steps.hpp"

namespace pf {
namespace {

// With an optimizer state, the launch returns at once when the stop rule has ended the
// optimization, or when `regime` >= 0 and the particles' spread is in another regime. NARROW: the
// volume passes narrow_grid.
template <int FMT, int LAYOUT, int TK, int BLOCK, bool MASK, bool NARROW>
__global__ __launch_bounds__(BLOCK) void k_score(VolView vv, const float* __restrict__ px, const float* __restrict__ py,
                                                 const float* __restrict__ pz, int n_host, const int* __restrict__ n_dev,
                                                 const float* __restrict__ poses, int K, float* __restrict__ fitness,
                                                 int* __restrict__ n_valid, const pf_track_state* st, int regime) {
    if (st && (st->done || (regime >= 0 && spread_regime(st, vv.inv_vs) != regime))) return;
    score_step<FMT, LAYOUT, TK, BLOCK, MASK, NARROW>(vv, px, py, pz, n_dev ? *n_dev : n_host, poses, K,
                                                    blockIdx.x * TK, fitness, n_valid);
}

template <int FMT, int LAYOUT, int TK, int BLOCK, bool MASK = false, bool NARROW = false>
int32_t launch_t(const VolView& vv, const Points& p, const float* poses, int K, float* fitness, int* n_valid,
                 const pf_track_state* st, int regime, hipStream_t s) {
    const int blocks = (K + TK - 1) / TK;
    hipLaunchKernelGGL((k_score<FMT, LAYOUT, TK, BLOCK, MASK, NARROW>), dim3(blocks), dim3(BLOCK), 0, s, vv, p.x, p.y,
                       p.z, p.n, p.n_dev, poses, K, fitness, n_valid, st, regime);
    return check_launch("particles_score");
}


// Launch shape of the many-pose scoring launches (pf_score_config): poses per workgroup and
// workgroup size, or 0 and 0 for the shape by spread regime (the default). Process-wide settings
// read by every caller; atomics, so a change while another thread launches is no data race (that
// launch takes the old or the new shape, which gives the same bits: the sums are exact).
std::atomic<int> g_tk{0}, g_block{0};

// Spread regimes whose automatic launches read the cell-validity mask (pf_score_mask), bit r for
// regime r; kMaskAlways also masks the launches without a spread (particles_score).
constexpr int kMaskAlways = 8;
std::atomic<int> g_mask_regimes{kMaskRegimes};

// Automatic shape for K poses: 4x256 (measured at K = 3073: the masked, compacting launch of the
// spread regime ran the headline sequence at 4.01 ms per frame at 4x256, 4.09 at 2x256, 4.16 at
// 1x256, 4.33 at 4x128; the tight launch is fastest at 4x256; the unmasked spread launch of the
// sparse layout ran its sequence at 4.92 ms at 4x256, 5.06 at 4x128, 5.35 at 2x64), or, when that
// launch would hold fewer than one wave per SIMD (1024 on MI355X), the first of 2x256, 1x256,
// 1x1024 that does: a few hundred poses must spread their points over more waves to fill the chip.
// Shape codes: 0 = 4x256, 1 = 2x256, 2 = 1x256, 3 = 1x1024.
constexpr int kMinWaves = 1024;

int auto_shape(int K) {
    static const int tk[4] = {4, 2, 1, 1}, wpg[4] = {4, 4, 4, 16};
    for (int c = 0; c < 3; ++c)
        if ((K + tk[c] - 1) / tk[c] * wpg[c] >= kMinWaves) return c;
    return 3;
}

// One launch of automatic shape code `shape` (the 4x256 shape of many poses also in its narrow
// form).
template <int FMT, int LAYOUT, bool MASK>
int32_t launch_shape(int shape, const VolView& vv, const Points& p, const float* poses, int K, float* fitness,
                     int* n_valid, const pf_track_state* st, int gate, hipStream_t s) {
    if constexpr (MASK && LAYOUT == PF_LAYOUT_LINEAR) {
        return set_error(PF_EUNSUPPORTED, "particles_score: the x-fastest layout has no mask");
    } else {
        switch (shape) {
            case 0:
                return narrow_grid(vv)
                           ? launch_t<FMT, LAYOUT, 4, 256, MASK, true>(vv, p, poses, K, fitness, n_valid, st, gate, s)
                           : launch_t<FMT, LAYOUT, 4, 256, MASK>(vv, p, poses, K, fitness, n_valid, st, gate, s);
            case 1: return launch_t<FMT, LAYOUT, 2, 256, MASK>(vv, p, poses, K, fitness, n_valid, st, gate, s);
            case 2: return launch_t<FMT, LAYOUT, 1, 256, MASK>(vv, p, poses, K, fitness, n_valid, st, gate, s);
            default: return launch_t<FMT, LAYOUT, 1, 1024, MASK>(vv, p, poses, K, fitness, n_valid, st, gate, s);
        }
    }
}

// The configured shape (pf_score_config); in automatic mode with an optimizer state, either the
// one shape of the expected regime (`expect` >= 0, the caller's forecast; the launch then runs
// whatever the spread, so a wrong forecast costs speed only), or one launch per spread regime, each
// reading the search size on the device (all but one return at once).
template <int FMT, int LAYOUT>
int32_t launch_fl(const VolView& vv, const Points& p, const float* poses, int K, float* fitness, int* n_valid,
                  const pf_track_state* st, hipStream_t s, int expect) {
    constexpr bool kMasked = LAYOUT != PF_LAYOUT_LINEAR;   // the layouts with a cell-validity mask
    const bool mask_all = kMasked && (g_mask_regimes & kMaskAlways);
    // few poses: spread the points over a wide workgroup
    if (K <= 64)
        return mask_all ? launch_t<FMT, LAYOUT, 1, 1024, kMasked>(vv, p, poses, K, fitness, n_valid, st, -1, s)
                        : launch_t<FMT, LAYOUT, 1, 1024>(vv, p, poses, K, fitness, n_valid, st, -1, s);
#define PF_SHAPE(TK, B)                                                                                       \
    if (g_tk == TK && g_block == B)                                                                           \
        return mask_all ? launch_t<FMT, LAYOUT, TK, B, kMasked>(vv, p, poses, K, fitness, n_valid, st, -1, s) \
                        : launch_t<FMT, LAYOUT, TK, B>(vv, p, poses, K, fitness, n_valid, st, -1, s);
    PF_SHAPE(1, 256) PF_SHAPE(2, 256) PF_SHAPE(8, 256)
    PF_SHAPE(1, 512) PF_SHAPE(2, 512) PF_SHAPE(4, 512) PF_SHAPE(8, 512)
    PF_SHAPE(2, 128) PF_SHAPE(4, 128) PF_SHAPE(8, 128)
    PF_SHAPE(2, 64) PF_SHAPE(4, 64) PF_SHAPE(8, 64)
#undef PF_SHAPE
    if (g_tk == 0 && st) {
        int32_t rc = PF_OK;
        for (int regime = 0; regime < kRegimes && !rc; ++regime) {
            if (expect >= 0 && regime != expect) continue;
            const int gate = expect >= 0 ? -1 : regime;
            const bool mask = kMasked && ((g_mask_regimes >> regime) & 1);
            const int shape = auto_shape(K);
            rc = mask ? launch_shape<FMT, LAYOUT, true>(shape, vv, p, poses, K, fitness, n_valid, st, gate, s)
                      : launch_shape<FMT, LAYOUT, false>(shape, vv, p, poses, K, fitness, n_valid, st, gate, s);
        }
        return rc;
    }
    return mask_all ? launch_t<FMT, LAYOUT, 4, 256, kMasked>(vv, p, poses, K, fitness, n_valid, st, -1, s)
                    : launch_t<FMT, LAYOUT, 4, 256>(vv, p, poses, K, fitness, n_valid, st, -1, s);
}

}  // namespace

int32_t score_config(int tk, int block) {
    if (tk == 0 && block == 0) {
        g_tk = g_block = 0;
        return PF_OK;
    }
    const bool ok_tk = tk == 1 || tk == 2 || tk == 4 || tk == 8;
    const bool ok_b = block == 64 || block == 128 || block == 256 || block == 512;
    if (!ok_tk || !ok_b || (tk == 1 && block < 256))
        return set_error(PF_EINVAL, "pf_score_config: unsupported shape (%d poses, %d threads)", tk, block);
    g_tk = tk;
    g_block = block;
    return PF_OK;
}

int32_t score_mask(int mode) {
    switch (mode) {
        case PF_MASK_BY_SPREAD: g_mask_regimes = kMaskRegimes; return PF_OK;
        case PF_MASK_ALWAYS: g_mask_regimes = ((1 << kRegimes) - 1) | kMaskAlways; return PF_OK;
        case PF_MASK_NEVER: g_mask_regimes = 0; return PF_OK;
        default: return set_error(PF_EINVAL, "pf_score_mask: unknown mode %d", mode);
    }
}

int32_t launch_score(const VolView& vv, const Points& p, const float* poses, int K, float* fitness, int* n_valid,
                     hipStream_t s, const pf_track_state* st, int expect) {
    return with_volume(vv.format, vv.layout, [&](auto fmt, auto layout) {
        return launch_fl<decltype(fmt)::value, decltype(layout)::value>(vv, p, poses, K, fitness, n_valid, st, s,
                                                                          expect);
    });
}

int spread_regime_of(double s_rad, double s_m, float inv_vs) { return spread_regime_sm(s_rad, s_m, inv_vs); }

bool score_auto_4x256(int K) { return g_tk.load() == 0 && K > 64 && auto_shape(K) == 0; }

bool score_regime_masked(int layout, int regime) {
    return layout != PF_LAYOUT_LINEAR && ((g_mask_regimes.load() >> regime) & 1) != 0;
}

}  // namespace pf
