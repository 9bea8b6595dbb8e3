// The particle launch of the optimization loop that draws its own particles (Sec. III-B: sampling
// around the current pose, then the fitness of every particle), in one launch per iteration instead
// of a draw launch followed by a scoring launch.
#include <atomic>
#include <type_traits>

#include "pf_steps.hpp"

namespace pf {
namespace {

// The particle launch that draws its own particles: it completes iteration i - 1 and plans
// iteration i as the separate draw launch does (FIRST: iteration 1 around the initial state), then
// each 4-pose workgroup draws its particles 4 blockIdx.x + 1 .. 4 blockIdx.x + 4 (the same FP64
// composition, into `poses`, the state's deltas and LDS) and scores them on the view; workgroup 0
// also records slot 0 and E_0. One launch and one dependent-launch gap fewer per iteration.
// NARROW: the volume passes narrow_grid (score_step).
template <int FMT, int LAYOUT, bool MASK, bool NARROW>
__global__ __launch_bounds__(256) void k_draw_score(VolView vv, Points S, pf_track_state* st, int K, int n_partials,
                                                   int first, IterRec* recs, int e0_partials, float* poses,
                                                   float* fit, int* nv) {
    __shared__ float pose_sh[4 * 12];
    DrawPlan P;
    const bool lead_block = blockIdx.x == 0;
    const bool lead = lead_block && threadIdx.x == kWave;   // a thread of another wave than the draws
    const bool go =
        first ? draw_prologue<FMT, true>(st, K, n_partials, recs, lead_block, lead, e0_partials, fit, nv, P)
              : draw_prologue<FMT, false>(st, K, n_partials, recs, lead_block, lead, e0_partials, fit, nv, P);
    if (!go || P.stop) return;
    const int k0 = 4 * (int)blockIdx.x;
    if (threadIdx.x < 4 && k0 + 1 + (int)threadIdx.x <= P.K_it)
        draw_particle(st, P, k0 + 1 + (int)threadIdx.x, poses, pose_sh + 12 * threadIdx.x);
    if (lead) draw_particle(st, P, 0, poses, nullptr);
    __syncthreads();
    const int Kl = min(4, P.K_it - k0);
    if (Kl <= 0) return;
    score_step<FMT, LAYOUT, 4, 256, MASK, NARROW>(vv, S.x, S.y, S.z, S.n_dev ? *S.n_dev : S.n, pose_sh, Kl, 0, fit + 1 + k0,
                                          nv + 1 + k0);
}

}  // namespace

void warm_draw_score(int format, int layout) {
    // The runtime loads a kernel's code on its first launch (about a millisecond). Frames without a
    // regime forecast (the first of a sequence) do not launch this kernel, so the first call on a
    // device loads it up front, by querying the attributes of the volume's instantiations: the
    // next frame's launches then find it loaded.
    static std::atomic<unsigned> warmed[64][3][3];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || format < 0 || format > 2 || layout < 0 ||
        layout > 2)
        return;
    if (warmed[dev][format][layout].exchange(1u)) return;
    with_volume(format, layout, [&](auto fmt, auto lay) {
        constexpr int F = decltype(fmt)::value, LY = decltype(lay)::value;
        hipFuncAttributes attr;
        auto warm = [&](auto narrow) {
            constexpr bool C = decltype(narrow)::value;
            (void)hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_draw_score<F, LY, false, C>));
            if constexpr (LY != PF_LAYOUT_LINEAR)
                (void)hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(&k_draw_score<F, LY, true, C>));
        };
        warm(std::true_type{});
        warm(std::false_type{});
        return PF_OK;
    });
}

int32_t launch_draw_score(const VolView& vv, const Points& S, pf_track_state* st, int K, int K_i, int n_partials,
                          bool first, IterRec* recs, int e0_partials, float* poses, float* fit, int* nv, int regime,
                          hipStream_t s) {
    const dim3 grid((unsigned)((K_i + 3) / 4));
    const bool mask = score_regime_masked(vv.layout, regime);
    const bool narrow = narrow_grid(vv);
    return with_volume(vv.format, vv.layout, [&](auto fmt, auto layout) {
        constexpr int F = decltype(fmt)::value, LY = decltype(layout)::value;
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, grid, dim3(256), 0, s, vv, S, st, K, n_partials, first ? 1 : 0, recs,
                               e0_partials, poses, fit, nv);
            return check_launch("track_frame particle launch");
        };
        if constexpr (LY != PF_LAYOUT_LINEAR) {
            if (mask) return narrow ? go(k_draw_score<F, LY, true, true>) : go(k_draw_score<F, LY, true, false>);
        }
        return narrow ? go(k_draw_score<F, LY, false, true>) : go(k_draw_score<F, LY, false, false>);
    });
}

}  // namespace pf
