// Step bodies of the particle-scoring launches (Sec. III-B, fitness equation), apart from the
// per-sample evaluation in pf_sample.hpp: the spread regimes that choose the launch, the
// compacting path through the cell-validity mask, the per-lane path, and the workgroup step that
// scores a group of poses over all points.
#pragma once

#include "pf_sample.hpp"

namespace pf {

// ------------------------------------------------------------------ spread regimes
// Spread regime of the particles being scored, from the search size that drew them: the largest
// displacement of a point 2 m from the rotation centre, in voxels. While the particles are spread
// over more than a quarter voxel (regime 0), their samples land in cells scattered over and around
// the band, many of them invalid (over 90% at 10 deg around a prior a few degrees off, about half
// at a few voxels): the scoring reads the cell-validity mask first and gathers and interpolates the
// valid samples only, compacted into full waves. Once they have gathered (regime 1), neighbouring
// particles sample the same cells, most samples are valid, and the per-lane path with its reuse of
// the previous particle's corners is bound by the vector ALUs; the mask's extra round trip would
// cost more than it saves. The choice changes speed only, since the sums are exact.
constexpr double kSpreadLever = 2.0;    // metres
constexpr double kSpreadTight = 0.25;   // voxels
constexpr int kRegimes = 2;

// Regimes in which the replica is read through the cell-validity mask (bit r for regime r).
constexpr int kMaskRegimes = 1;

__host__ __device__ inline int spread_regime_sm(double s_rad, double s_m, float inv_vs) {
    const double d = (s_rad * kSpreadLever + s_m) * (double)inv_vs;
    return d > kSpreadTight ? 0 : 1;
}

__device__ inline int spread_regime(const pf_track_state* st, float inv_vs) {
    return spread_regime_sm(st->s_rad, st->s_m, inv_vs);
}

// ------------------------------------------------------------------ particle scoring
// Masked scoring with compaction, for wide spreads, where most samples fail the mask test: with one
// sample per (lane, pose) a wave would still compute the cell address and interpolation of every
// pose of every lane as long as one of its lanes needs them. Here each wave keeps one queue per
// pose in LDS. A pass over 64 points appends the valid samples of each pose (cell index and
// fractions) in lane order (ballot and mbcnt), and whenever a queue holds a full wave of samples,
// the wave gathers and interpolates them with every lane busy. Sums are exact integers, so the
// order in which the samples are added does not change a pose's fitness: the result is bitwise that
// of the per-lane path.
constexpr int kQueue = 128;   // entries per pose queue: up to 63 waiting + 64 appended in one pass

// Whether the queues of a workgroup fit the LDS budget of the compacting path (32 KB).
template <int TK, int BLOCK>
constexpr bool compact_fits() {
    return (BLOCK / kWave) * TK * kQueue * 16 <= 32768;
}

template <int FMT, int LAYOUT, int TK, int BLOCK, bool NARROW, bool PRIO>
__attribute__((always_inline))
__device__ inline void score_points_compact(const VolView& vv, const float* __restrict__ px,
                                            const float* __restrict__ py, const float* __restrict__ pz, int n,
                                            const float* __restrict__ poses, int K, int k0, FixSum (&sum)[TK],
                                            int (&cnt)[TK]) {
    static_assert(LAYOUT == PF_LAYOUT_CELLS || LAYOUT == PF_LAYOUT_BRICKS, "the mask exists for these layouts");
    __shared__ uint4 queue[BLOCK / kWave][TK][kQueue];
    const Gather<FMT, LAYOUT> G = make_gather<FMT, LAYOUT>(vv);
    GridPose g[TK];
#pragma unroll
    for (int j = 0; j < TK; ++j)
        g[j] = fold_pose(poses + (size_t)min(k0 + j, K - 1) * 12, vv.inv_vs, vv.gx0, vv.gy0, vv.gz0);
    const unsigned lx = (unsigned)(vv.nx - 1), ly = (unsigned)(vv.ny - 1), lz = (unsigned)(vv.nz - 1);
    const int lane = threadIdx.x & (kWave - 1);
    uint4(*Q)[kQueue] = queue[threadIdx.x / kWave];
    int head[TK], fill[TK];   // wave-uniform ring state of each pose's queue
#pragma unroll
    for (int j = 0; j < TK; ++j) {
        sum[j] = 0;
        cnt[j] = 0;
        head[j] = 0;
        fill[j] = 0;
    }
    // gathers and interpolates the first m entries of pose j's queue, one per lane
    auto drain = [&](int j, int m) {
        const uint4 e = Q[j][(head[j] + lane) & (kQueue - 1)];
        if (lane < m) {
            float c[8];
            if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
            G.load(G.at(e.x), c);
            if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
            const float v = trilerp(__uint_as_float(e.y), __uint_as_float(e.z), __uint_as_float(e.w), c);
            sum[j] += (FixSum)fixed_point<FMT>(v);
            cnt[j] += 1;
        }
        head[j] = (head[j] + m) & (kQueue - 1);
        fill[j] -= m;
    };
    const float s = vv.inv_vs;
    const int passes = (n + BLOCK - 1) / BLOCK;   // the same for every lane: the ballots need them all
    float nx = 0.0f, ny = 0.0f, nz = 0.0f;
    if ((int)threadIdx.x < n) {
        nx = px[threadIdx.x];
        ny = py[threadIdx.x];
        nz = pz[threadIdx.x];
    }
    for (int pass = 0; pass < passes; ++pass) {
        const int q = pass * BLOCK + (int)threadIdx.x;
        const bool active = q < n;
        const unsigned long long mact = __builtin_amdgcn_ballot_w64(active);
        const float x = nx * s, y = ny * s, z = nz * s;
        if (q + BLOCK < n) {
            nx = px[q + BLOCK];
            ny = py[q + BLOCK];
            nz = pz[q + BLOCK];
        }
        // cells, fractions and mask words of all poses (the mask loads in flight together)
        int cl[TK][3];
        float f[TK][3];
        bool inb[TK];
        unsigned long long minb[TK];   // the wave's lanes whose sample of pose j is in the grid
        unsigned long long mw[TK];
        unsigned cell[TK], bit[TK];   // the cell's index in the replica or the pool, its mask bit
#pragma unroll
        for (int j = 0; j < TK; ++j) {
            const float gx = fmaf(g[j].r[0], x, fmaf(g[j].r[1], y, fmaf(g[j].r[2], z, g[j].t[0])));
            const float gy = fmaf(g[j].r[3], x, fmaf(g[j].r[4], y, fmaf(g[j].r[5], z, g[j].t[1])));
            const float gz = fmaf(g[j].r[6], x, fmaf(g[j].r[7], y, fmaf(g[j].r[8], z, g[j].t[2])));
            const unsigned ux = (unsigned)floor_to_int(gx), uy = (unsigned)floor_to_int(gy),
                           uz = (unsigned)floor_to_int(gz);
            const bool ig = in_grid<NARROW>(ux, uy, uz, lx, ly, lz);
            minb[j] = __builtin_amdgcn_ballot_w64(ig) & mact;
            inb[j] = ig && active;
            if constexpr (LAYOUT == PF_LAYOUT_CELLS) {
                // the replica: the cell as computed (outside the grid it is not used, and its mask
                // word is read at offset 0 instead)
                cl[j][0] = (int)ux;
                cl[j][1] = (int)uy;
                cl[j][2] = (int)uz;
            } else {
                cl[j][0] = (int)min(ux, lx - 1u);
                cl[j][1] = (int)min(uy, ly - 1u);
                cl[j][2] = (int)min(uz, lz - 1u);
            }
            f[j][0] = __builtin_amdgcn_fractf(gx);
            f[j][1] = __builtin_amdgcn_fractf(gy);
            f[j][2] = __builtin_amdgcn_fractf(gz);
        }
        // (the mask loads, and each drain's gathers below, are issued at a raised wave priority, as
        // in eval_poses: -23 us per frame on the headline sequence)
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
        if constexpr (LAYOUT == PF_LAYOUT_CELLS) {
#pragma unroll
            for (int j = 0; j < TK; ++j) {
                const unsigned ux = (unsigned)cl[j][0], uy = (unsigned)cl[j][1], uz = (unsigned)cl[j][2];
                mw[j] = G.mask_at(select_u32(minb[j], G.mask_index(ux, uy, uz), 0u));
                cell[j] = G.index(ux, uy, uz);
                bit[j] = G.mask_shift(ux, uy, uz);
            }
        } else {
            // sparse: the brick's slot first (one round for all poses), then its mask word; a
            // brick without a slot has no valid cell (its word is read from slot 0, in bounds,
            // and ignored)
            int slot[TK];
#pragma unroll
            for (int j = 0; j < TK; ++j) slot[j] = G.slot(G.key(cl[j][0], cl[j][1], cl[j][2]));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < TK; ++j) {
                inb[j] &= slot[j] >= 0;
                minb[j] &= __builtin_amdgcn_ballot_w64(slot[j] >= 0);
                const unsigned sl = (unsigned)max(slot[j], 0);
                const unsigned loc = G.local(cl[j][0], cl[j][1], cl[j][2]);
                mw[j] = G.M[sl * kBrickMaskWords + (loc >> 6)];
                cell[j] = (sl << 9) | loc;
                bit[j] = loc & 63u;
            }
        }
        // (the loads are issued for every lane, in bounds thanks to the clamp, and kept together:
        // a short-circuit test would move a load into a branch and wait for it there)
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_sched_barrier(0);
        // append the valid samples of each pose to its queue, in lane order
#pragma unroll
        for (int j = 0; j < TK; ++j) {
            bool set;
            if constexpr (LAYOUT == PF_LAYOUT_CELLS)
                set = word_bit(mw[j], bit[j]) != 0;
            else
                set = ((mw[j] >> bit[j]) & 1ull) != 0;
            // (the lanes to append as one scalar mask, which also guards the append)
            const unsigned long long m = __builtin_amdgcn_ballot_w64(set) & minb[j];
            if (__builtin_amdgcn_inverse_ballot_w64(m)) {
                const unsigned below =
                    __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                Q[j][(head[j] + fill[j] + (int)below) & (kQueue - 1)] = make_uint4(
                    cell[j], __float_as_uint(f[j][0]), __float_as_uint(f[j][1]), __float_as_uint(f[j][2]));
            }
            fill[j] += __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
        // (draining the full queues one after the other measured faster than issuing all their
        // gathers before the first wait)
#pragma unroll
        for (int j = 0; j < TK; ++j)
            if (fill[j] >= kWave) drain(j, kWave);
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int j = 0; j < TK; ++j)
        if (fill[j] > 0) drain(j, fill[j]);
}

// Per-lane path: every lane keeps one point in registers and evaluates it against the TK poses
// (uniform, in scalar registers; eval_poses), without the mask or through it when the compacting
// queues do not fit.
template <int FMT, int LAYOUT, int TK, int BLOCK, bool MASK, bool NARROW, bool PRIO>
__attribute__((always_inline))
__device__ inline void score_points_lanes(const VolView& vv, const float* __restrict__ px,
                                          const float* __restrict__ py, const float* __restrict__ pz, int n,
                                          const float* __restrict__ poses, int K, int k0, FixSum (&sum)[TK],
                                          int (&cnt)[TK]) {
    const Gather<FMT, LAYOUT> G = make_gather<FMT, LAYOUT>(vv);
    GridPose g[TK];
#pragma unroll
    for (int j = 0; j < TK; ++j)
        g[j] = fold_pose(poses + (size_t)min(k0 + j, K - 1) * 12, vv.inv_vs, vv.gx0, vv.gy0, vv.gz0);
    const unsigned lx = (unsigned)(vv.nx - 1), ly = (unsigned)(vv.ny - 1), lz = (unsigned)(vv.nz - 1);
#pragma unroll
    for (int j = 0; j < TK; ++j) {
        sum[j] = 0;
        cnt[j] = 0;
    }
    const float s = vv.inv_vs;
    // the next point is loaded while the current one's gathers are in flight, so every pass of
    // the loop waits for one memory round trip instead of two. Every lane runs every pass (a lane
    // past the end holds no point), so a wave counts its valid samples with one scalar population
    // count; lane 0 (the wave's first point) then holds the wave's counts.
    const int passes = (n + BLOCK - 1) / BLOCK;
    float nx = 0.0f, ny = 0.0f, nz = 0.0f;
    if ((int)threadIdx.x < n) {
        nx = px[threadIdx.x];
        ny = py[threadIdx.x];
        nz = pz[threadIdx.x];
    }
    for (int pass = 0; pass < passes; ++pass) {
        const int q = pass * BLOCK + (int)threadIdx.x;
        const float x = nx * s, y = ny * s, z = nz * s;
        // (the next point's registers are free only now; its index is clamped into the cloud, so
        // every lane loads without a branch, from a 32-bit offset)
        __builtin_amdgcn_sched_barrier(0);
        const unsigned off = (unsigned)min(q + BLOCK, n - 1) * 4u;   // (a cloud holds < 2^30 points)
        nx = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(px) + off);
        ny = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(py) + off);
        nz = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(pz) + off);
        eval_poses<FMT, LAYOUT, TK, MASK, NARROW, true, PRIO>(G, lx, ly, lz, g, x, y, z, sum, cnt, q < n);
    }
    if ((threadIdx.x & (kWave - 1)) != 0) {
#pragma unroll
        for (int j = 0; j < TK; ++j) cnt[j] = 0;
    }
}

// Workgroup of BLOCK threads scoring poses k0 .. k0+TK-1 over all n points, through the
// cell-validity mask when MASK (compacting the valid samples when the queues fit in 32 KB of LDS).
// The sums are exact, so the result of a pose does not depend on TK, BLOCK, MASK or the workgroup.
// NARROW: the volume passes narrow_grid (eval_poses: the same answer with fewer instructions).
// PRIO: the scoring paths' raised-priority windows (off in the batched kernels).
template <int FMT, int LAYOUT, int TK, int BLOCK, bool MASK = false, bool NARROW = false, bool PRIO = true>
__attribute__((always_inline))
__device__ inline void score_step(const VolView& vv, const float* __restrict__ px, const float* __restrict__ py,
                                  const float* __restrict__ pz, int n, const float* __restrict__ poses, int K, int k0,
                                  float* __restrict__ fitness, int* __restrict__ n_valid) {
    FixSum sum[TK];
    int cnt[TK];
    if constexpr (MASK && LAYOUT != PF_LAYOUT_LINEAR && compact_fits<TK, BLOCK>())
        score_points_compact<FMT, LAYOUT, TK, BLOCK, NARROW, PRIO>(vv, px, py, pz, n, poses, K, k0, sum, cnt);
    else   // (the sparse layout reads its mask only when compacting: the mask changes speed only)
        score_points_lanes<FMT, LAYOUT, TK, BLOCK, MASK && LAYOUT == PF_LAYOUT_CELLS, NARROW, PRIO>(vv, px, py, pz, n,
                                                                                           poses, K, k0, sum, cnt);
    block_reduce<TK, BLOCK>(sum, cnt);
    if (threadIdx.x < TK) {
        const int k = k0 + threadIdx.x;
        if (k < K) {
            fitness[k] = fitness_from<FMT>(sum[0], cnt[0]);
            n_valid[k] = cnt[0];
        }
    }
    __syncthreads();
}

// score_step through the cell-validity mask when the replica has one and the particles' spread
// regime `regime` is one of kMaskRegimes (uniform across the workgroup).
template <int FMT, int LAYOUT, int TK, int BLOCK, bool PRIO = true>
__attribute__((always_inline))
__device__ inline void score_step_regime(const VolView& vv, const float* __restrict__ px,
                                         const float* __restrict__ py, const float* __restrict__ pz, int n,
                                         const float* __restrict__ poses, int K, int k0, float* __restrict__ fitness,
                                         int* __restrict__ n_valid, int regime) {
    if constexpr (LAYOUT != PF_LAYOUT_LINEAR) {
        if ((kMaskRegimes >> regime) & 1) {
            score_step<FMT, LAYOUT, TK, BLOCK, true, false, PRIO>(vv, px, py, pz, n, poses, K, k0, fitness, n_valid);
            return;
        }
    }
    score_step<FMT, LAYOUT, TK, BLOCK, false, false, PRIO>(vv, px, py, pz, n, poses, K, k0, fitness, n_valid);
}

}  // namespace pf
