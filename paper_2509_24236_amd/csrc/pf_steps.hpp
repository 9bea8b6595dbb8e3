// Step bodies of the per-frame optimization as device functions taking an explicit workgroup
// index: the single-problem kernels and the batched persistent kernels call the same code, so a
// batched problem computes bit for bit what the plain path computes.
#pragma once

#include <math.h>

#include "pf_sample.hpp"
#include "pf_score_steps.hpp"

namespace pf {

constexpr int kBpThreads = 256;
constexpr int kBpPerThread = 4;
constexpr int kBpChunk = kBpThreads * kBpPerThread;  // pixels per workgroup, in raster order

struct BpArgs {
    const float* depth;
    int width, height, stride;
    float fx, fy, cx, cy;
    int* pix;                    // optional: pixel index of every compacted point
    unsigned long long* masks;   // optional: view-tile masks cleared by the count step
    int n_masks, nblocks;        // masks to clear; workgroups of the count step
};

__device__ inline bool bp_valid(const BpArgs& a, int pix, float& z) {
    const int n = a.width * a.height;
    if (pix >= n) return false;
    const int v = pix / a.width, u = pix - v * a.width;
    if ((u % a.stride) != 0 || (v % a.stride) != 0) return false;
    z = a.depth[pix];
    return isfinite(z) && z > 0.0f;
}

__device__ inline void bp_count_step(const BpArgs& a, int* counts, int blk) {
    for (int i = blk * kBpThreads + threadIdx.x; i < a.n_masks; i += a.nblocks * kBpThreads) a.masks[i] = 0ull;
    const int base = blk * kBpChunk + threadIdx.x * kBpPerThread;
    int c = 0;
#pragma unroll
    for (int q = 0; q < kBpPerThread; ++q) {
        float z;
        c += bp_valid(a, base + q, z) ? 1 : 0;
    }
    __shared__ int red[kBpThreads / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kBpThreads / kWave; ++w) s += red[w];
        counts[blk] = s;
    }
    __syncthreads();
}

// Each workgroup sums the counts of the workgroups before it (a few hundred integers), scans
// its own pixels and writes them in raster order; workgroup 0 also writes the total.
__device__ inline void bp_scatter_step(const BpArgs& a, const int* counts, int nblocks, float* px, float* py,
                                       float* pz, int* n_out, int blk) {
    __shared__ int red[kBpThreads / kWave];
    __shared__ int wsum[kBpThreads / kWave];
    __shared__ int base_sh, total_sh;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int before = 0, all = 0;
    for (int b = threadIdx.x; b < nblocks; b += kBpThreads) {
        const int c = counts[b];
        all += c;
        if (b < blk) before += c;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        before += __shfl_xor(before, off);
        all += __shfl_xor(all, off);
    }
    if (lane == 0) {
        red[wid] = before;
        wsum[wid] = all;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0, t = 0;
        for (int w = 0; w < kBpThreads / kWave; ++w) {
            s += red[w];
            t += wsum[w];
        }
        base_sh = s;
        total_sh = t;
        if (blk == 0) *n_out = t;
    }
    __syncthreads();
    // in-workgroup exclusive scan of the per-thread counts (thread order = raster order)
    const int pbase = blk * kBpChunk + threadIdx.x * kBpPerThread;
    float zs[kBpPerThread];
    bool ok[kBpPerThread];
    int c = 0;
#pragma unroll
    for (int q = 0; q < kBpPerThread; ++q) {
        ok[q] = bp_valid(a, pbase + q, zs[q]);
        c += ok[q] ? 1 : 0;
    }
    int incl = c;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    __shared__ int wtot[kBpThreads / kWave];
    if (lane == kWave - 1) wtot[wid] = incl;
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wid; ++w) woff += wtot[w];
    int pos = base_sh + woff + incl - c;
#pragma unroll
    for (int q = 0; q < kBpPerThread; ++q) {
        if (ok[q]) {
            const int pix = pbase + q;
            const int v = pix / a.width, u = pix - v * a.width;
            const float z = zs[q];
            px[pos] = ((float)u - a.cx) * z / a.fx;
            py[pos] = ((float)v - a.cy) * z / a.fy;
            pz[pos] = z;
            if (a.pix) a.pix[pos] = pix;
            ++pos;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ sub-sampled views
// S_r holds M[j r] for j < ceil(n / r) (the set the method defines), copied contiguously in an order
// chosen for the gathers: tiles of 32 image rows by 2 r columns, row by row inside a tile. A
// wavefront's 64 lanes then take a 32 x 2 patch of neighbouring points instead of 64 points
// spread along a row, r pixels apart, and its stencils share cache lines. Sums over a view are
// exact integers or are taken in this fixed order, so the order changes speed only. Two points
// of S_r in one row are at least r pixels apart, so a row puts at most one point in each half of
// a tile: (row mod 32, half) is a distinct bit of the tile's 64-bit mask, and a point's place in
// the view is its tile's start plus the number of lower bits set.
constexpr int kTileRows = 32;

struct ViewTiles {
    unsigned long long* mask;   // per tile
    int* start;                 // per tile: position of its first point in the view
    int tiles_x, n_tiles;
};

__host__ __device__ inline int view_tiles_x(int width, int r) { return (width + 2 * r - 1) / (2 * r); }
__host__ __device__ inline int view_n_tiles(int width, int height, int r) {
    return view_tiles_x(width, r) * ((height + kTileRows - 1) / kTileRows);
}

__device__ inline int view_tile(int pix, int width, int r, int tiles_x, int& bit) {
    const int v = pix / width, u = pix - v * width;
    const int cx = u / (2 * r);
    bit = (v % kTileRows) * 2 + (u - cx * 2 * r >= r ? 1 : 0);
    return (v / kTileRows) * tiles_x + cx;
}

// Sets the bit of every point of S_r (the masks were cleared by the count step).
__device__ inline void view_mark_step(const int* pix, const int* n_all, int r, int width, const ViewTiles& t, int blk) {
    const int m = (*n_all + r - 1) / r;
    const int j = blk * 256 + threadIdx.x;
    if (j >= m) return;
    int bit;
    const int tile = view_tile(pix[j * r], width, r, t.tiles_x, bit);
    atomicOr(&t.mask[tile], 1ull << bit);
}

// Exclusive scan of the tiles' point counts; one workgroup of 256 threads.
__device__ inline void view_scan_step(const ViewTiles& t) {
    __shared__ int part[256];
    const int per = (t.n_tiles + 255) / 256;
    const int q0 = threadIdx.x * per, q1 = min(t.n_tiles, q0 + per);
    int c = 0;
    for (int q = q0; q < q1; ++q) c += __popcll(t.mask[q]);
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < 256; ++w) {
            const int x = part[w];
            part[w] = acc;
            acc += x;
        }
    }
    __syncthreads();
    int acc = part[threadIdx.x];
    for (int q = q0; q < q1; ++q) {
        t.start[q] = acc;
        acc += __popcll(t.mask[q]);
    }
}

// Writes every point of S_r at its place; the count goes to *n_view.
__device__ inline void view_scatter_step(const float* px, const float* py, const float* pz, const int* pix,
                                         const int* n_all, int r, int width, const ViewTiles& t, float* vx, float* vy,
                                         float* vz, int* n_view, int blk) {
    const int m = (*n_all + r - 1) / r;
    const int j = blk * 256 + threadIdx.x;
    if (j == 0) *n_view = m;
    if (j >= m) return;
    const int q = j * r;
    int bit;
    const int tile = view_tile(pix[q], width, r, t.tiles_x, bit);
    const int pos = t.start[tile] + __popcll(t.mask[tile] & ((1ull << bit) - 1ull));
    vx[pos] = px[q];
    vy[pos] = py[q];
    vz[pos] = pz[q];
}

// ------------------------------------------------------------------ optimizer state
struct IterRec {
    float E0, Estar;
    int n_adv, n_sub, n_valid, n_particles;
    double s_rad, s_m;
};

struct Partial {
    FixSum sum;
    int cnt;
    int pad;
};

__host__ __device__ inline size_t partials_offset(int K) {
    return PF_STATE_DELTAS_OFFSET + (((size_t)(K + 1) * 6 * sizeof(double) + 255) & ~(size_t)255);
}

__device__ inline double* state_deltas(pf_track_state* st) {
    return reinterpret_cast<double*>(reinterpret_cast<char*>(st) + PF_STATE_DELTAS_OFFSET);
}

__device__ inline Partial* state_partials(pf_track_state* st, int K) {
    return reinterpret_cast<Partial*>(reinterpret_cast<char*>(st) + partials_offset(K));
}

// The second set of partials: the pose just computed scored on the next iteration's view, which is
// that iteration's E_0 (slot 0), so the particle launch scores the K particles alone.
__device__ inline Partial* state_partials_next(pf_track_state* st, int K) { return state_partials(st, K) + kMaxPartials; }

// The view of the next iteration (x == nullptr: none).
struct NextView {
    const float* x;
    const float* y;
    const float* z;
    const int* n_dev;
};


constexpr int kAdvThreads = 256;

// Field ownership keeps every kernel free of read-after-write hazards across its workgroups:
// k_adv reads (R, t, s, iter, deltas, fitness) and workgroup 0 writes (R_prev, t_prev, R_new,
// t_new, s_*_done, iter_done, E0, mean, n_adv, n_sub); k_next reads the latter and writes the
// former.
//
// k_adv, ADV = true: after the pending particles of iteration i were scored on S_i, every
// workgroup forms the advantage set A = {k >= 1 : E_k < E_0} and the mean delta over A in the
// same fixed order (so all compute the same P^(i) in FP64), then scores P^(i) on its chunk of
// S_i; the chunk's (sum, count) goes to the partials. ADV = false scores the pending pose P
// (used for the returned pose's final fitness).
//
// With a next view `nv` (x != nullptr), the workgroup also scores the new pose (ADV) or the pending
// pose (not ADV) on its chunk of that view, into the second set of partials: next_step turns them
// into the next iteration's E_0. Without ADV the first set is then left alone. PRIO: the scoring
// loop's raised-priority window (left off by the batched kernels).
template <int FMT, int LAYOUT, bool ADV, bool PRIO = true>
__device__ inline void adv_step(const VolView& vv, const float* __restrict__ px, const float* __restrict__ py,
                                const float* __restrict__ pz, int n_host, const int* __restrict__ n_dev,
                                const float* __restrict__ fitness, pf_track_state* st, int K, int blk, int nblk,
                                NextView nv = NextView{nullptr, nullptr, nullptr, nullptr}) {
    if (st->K != K) {
        if (blk == 0 && threadIdx.x == 0) st->flags |= 1;
        return;
    }
    if (ADV && st->done) return;   // the stop rule ended the optimization
    __shared__ float pose_sh[12];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int n = n_dev ? *n_dev : n_host;
    // This workgroup's chunk of the view (and of the next view): the first kPts points of each per
    // thread are loaded now, while the pose they are scored at is being formed; the update step's
    // chunks hold at most kPts * kAdvThreads points (a chunk beyond that is scored point by point).
    constexpr int kPts = 2;
    const bool score1 = ADV || !nv.x, score2 = nv.x != nullptr;
    const float sc = vv.inv_vs;
    int q0[2] = {0, 0}, q1[2] = {0, 0};
    float xs[2 * kPts], ys[2 * kPts], zs[2 * kPts];
    bool act[2 * kPts];
    {
        // (a lane without a point reads point 0 of a view that exists, always in bounds)
        const float* X[2] = {px, score2 ? nv.x : px};
        const float* Y[2] = {py, score2 ? nv.y : py};
        const float* Z[2] = {pz, score2 ? nv.z : pz};
        const int m[2] = {n, score2 ? *nv.n_dev : 0};
        const bool on[2] = {score1, score2};
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int chunk = (m[v] + nblk - 1) / nblk;
            q0[v] = blk * chunk;
            q1[v] = on[v] ? min(m[v], q0[v] + chunk) : 0;
#pragma unroll
            for (int r = 0; r < kPts; ++r) {
                const int q = q0[v] + (int)threadIdx.x + r * kAdvThreads;
                const int s = v * kPts + r;
                act[s] = q < q1[v];
                const int qq = act[s] ? q : 0;
                xs[s] = X[v][qq] * sc;
                ys[s] = Y[v][qq] * sc;
                zs[s] = Z[v][qq] * sc;
            }
        }
    }
    if constexpr (ADV) {
        const double* dl = state_deltas(st);
        const float E0 = fitness[0];
        const int Kc = st->K_cur;   // particles of the iteration just scored
        double acc[6] = {0, 0, 0, 0, 0, 0};
        int na = 0;
        // Twelve particles per pass (all of them for K = 3072) with all their loads issued together:
        // membership is a 0/1 factor (adding an exact zero leaves a sum unchanged), so there is no
        // branch to serialise the loads; indices past K_cur read in-bounds slots (the buffers hold
        // K + 1) with factor 0.
        constexpr int kU = 12;
        for (int kb = 1 + threadIdx.x; kb <= Kc; kb += kU * kAdvThreads) {
            double m[kU];
            int kk[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int k = kb + u * kAdvThreads;
                kk[u] = min(k, K);
                const float fk = fitness[kk[u]];
                m[u] = ((k <= Kc) & (fk < E0)) ? 1.0 : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
#pragma unroll
                for (int d = 0; d < 6; ++d) acc[d] += dl[6 * kk[u] + d] * m[u];
                na += m[u] != 0.0 ? 1 : 0;
            }
        }
        __shared__ double dred[6][kAdvThreads / kWave];
        __shared__ int cred[kAdvThreads / kWave];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
#pragma unroll
            for (int d = 0; d < 6; ++d) acc[d] += __shfl_xor(acc[d], off);
            na += __shfl_xor(na, off);
        }
        if (lane == 0) {
#pragma unroll
            for (int d = 0; d < 6; ++d) dred[d][wid] = acc[d];
            cred[wid] = na;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double sm[6] = {0, 0, 0, 0, 0, 0};
            int c = 0;
            for (int w = 0; w < kAdvThreads / kWave; ++w) {
                for (int d = 0; d < 6; ++d) sm[d] += dred[d][w];
                c += cred[w];
            }
            double R[9], t[3], mean[6] = {0, 0, 0, 0, 0, 0};
            for (int q = 0; q < 9; ++q) R[q] = st->R[q];
            for (int q = 0; q < 3; ++q) t[q] = st->t[q];
            if (c > 0) {
                for (int d = 0; d < 6; ++d) mean[d] = sm[d] / (double)c;
                double Ro[9], to[3];
                apply_delta(st->compose_mode, mean, mean + 3, R, t, Ro, to);
                for (int q = 0; q < 9; ++q) R[q] = Ro[q];
                for (int q = 0; q < 3; ++q) t[q] = to[q];
            }
            store_pose12(pose_sh, R, t);
            if (blk == 0) {
                for (int q = 0; q < 9; ++q) st->R_prev[q] = st->R[q];
                for (int q = 0; q < 3; ++q) st->t_prev[q] = st->t[q];
                for (int q = 0; q < 9; ++q) st->R_new[q] = R[q];
                for (int q = 0; q < 3; ++q) st->t_new[q] = t[q];
                for (int d = 0; d < 6; ++d) st->mean[d] = mean[d];
                st->n_adv = c;
                st->E0 = (double)E0;
                st->s_rad_done = st->s_rad;
                st->s_m_done = st->s_m;
                st->iter_done = st->iter;
                st->n_sub = n;
            }
        }
    } else {
        if (threadIdx.x == 0) {
            double R[9], t[3];
            for (int q = 0; q < 9; ++q) R[q] = st->R[q];
            for (int q = 0; q < 3; ++q) t[q] = st->t[q];
            store_pose12(pose_sh, R, t);
        }
    }
    __syncthreads();
    // the chunks scored with the scoring kernel's arithmetic: the preloaded samples of both views
    // with their gathers in flight together, then any points beyond them one by one
    const Gather<FMT, LAYOUT> G = make_gather<FMT, LAYOUT>(vv);
    GridPose g[1] = {fold_pose(pose_sh, vv.inv_vs, vv.gx0, vv.gy0, vv.gz0)};
    const unsigned lx = (unsigned)(vv.nx - 1), ly = (unsigned)(vv.ny - 1), lz = (unsigned)(vv.nz - 1);
    FixSum ss[2 * kPts];
    int cs[2 * kPts];
#pragma unroll
    for (int s = 0; s < 2 * kPts; ++s) {
        ss[s] = 0;
        cs[s] = 0;
    }
    eval_pose_points<FMT, LAYOUT, 2 * kPts>(G, lx, ly, lz, g[0], xs, ys, zs, act, ss, cs);
    FixSum sum[2];
    int cnt[2];
    const float* X[2] = {px, nv.x};
    const float* Y[2] = {py, nv.y};
    const float* Z[2] = {pz, nv.z};
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        FixSum s1[1] = {0};
        int c1[1] = {0};
        for (int q = q0[v] + (int)threadIdx.x + kPts * kAdvThreads; q < q1[v]; q += kAdvThreads)
            eval_poses<FMT, LAYOUT, 1, false, false, false, PRIO>(G, lx, ly, lz, g, X[v][q] * sc, Y[v][q] * sc,
                                                                 Z[v][q] * sc, s1, c1);
        sum[v] = s1[0];
        cnt[v] = c1[0];
#pragma unroll
        for (int r = 0; r < kPts; ++r) {
            sum[v] += ss[v * kPts + r];
            cnt[v] += cs[v * kPts + r];
        }
    }
    block_reduce<2, kAdvThreads>(sum, cnt);
    if (threadIdx.x == 0 && score1) {
        Partial* pt = state_partials(st, K);
        pt[blk].sum = sum[0];
        pt[blk].cnt = cnt[0];
    }
    if (threadIdx.x == 1 && score2) {
        Partial* pt = state_partials_next(st, K);
        pt[blk].sum = sum[0];
        pt[blk].cnt = cnt[0];
    }
    __syncthreads();
}

// (sum, count) of n_partials exact partials, in every thread of a 256-thread workgroup.
template <int FMT>
__device__ inline void partials_sum(const Partial* pt, int n_partials, FixSum& out_sum, int& out_cnt) {
    __shared__ FixSum rs[256 / kWave];
    __shared__ int rc[256 / kWave];
    FixSum sum = 0;
    int cnt = 0;
    for (int b = threadIdx.x; b < n_partials; b += 256) {
        sum += pt[b].sum;
        cnt += pt[b].cnt;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        sum += __shfl_xor(sum, off);
        cnt += __shfl_xor(cnt, off);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        rs[threadIdx.x / kWave] = sum;
        rc[threadIdx.x / kWave] = cnt;
    }
    __syncthreads();
    out_sum = 0;
    out_cnt = 0;
    for (int w = 0; w < 256 / kWave; ++w) {
        out_sum += rs[w];
        out_cnt += rc[w];
    }
    __syncthreads();
}

// The draw of one iteration, the same in every thread of the grid: P (the pose the particles are
// drawn around), the search size s, the iteration index, its particle count and the stop rule.
struct DrawPlan {
    double R[9], t[3], s_rad, s_m;
    uint32_t it;
    int K_it;
    bool stop;
};

// Completes iteration i (unless FIRST) and plans the draw of iteration i + 1: E* from the
// partials in order, s^(i+1) = s^(i) (beta + (1 - beta) E*), P = P^(i), and the stop rule on
// s^(i+1). FIRST plans iteration 1 around the initial state. Returns false (uniformly) when the
// state belongs to another K or the optimization has stopped.
//
// e0_partials > 0: the second set of partials (that many) holds P^(i) (FIRST: the initial pose)
// scored on the drawn iteration's view, and the workgroup with lead_block writes that E_0 and its
// count to fit0[0] and nv0[0], the slot 0 the particle launch does not score (or, after the last
// iteration, the returned pose's fitness on the densest view). The one thread with `lead` (in
// lead_block) records iteration i and moves the state on to iteration i + 1. Fields read here are
// never written here, apart from `done`, which is set only when the stop rule ends the
// optimization, in which case no thread draws.
template <int FMT, bool FIRST>
__device__ inline bool draw_prologue(pf_track_state* st, int K, int n_partials, IterRec* recs, bool lead_block,
                                     bool lead, int e0_partials, float* fit0, int* nv0, DrawPlan& P) {
    if (st->K != K || st->done) return false;
    if (e0_partials > 0 && lead_block) {
        FixSum sum;
        int cnt;
        partials_sum<FMT>(state_partials_next(st, K), e0_partials, sum, cnt);
        if (threadIdx.x == 0) {
            fit0[0] = fitness_from<FMT>(sum, cnt);
            nv0[0] = cnt;
        }
    }
    __shared__ double sh_s[2];
    __shared__ int sh_cnt;
    __shared__ float sh_E;
    if (!FIRST) {
        // E* from the exact partials (integer sums, so the reduction order is free)
        FixSum sum;
        int cnt;
        partials_sum<FMT>(state_partials(st, K), n_partials, sum, cnt);
        if (threadIdx.x == 0) {
#pragma clang fp contract(off)
            // (rounded step by step, as every kernel that updates s does)
            const float Es = fitness_from<FMT>(sum, cnt);
            const double f = st->beta + (1.0 - st->beta) * (double)Es;
            sh_s[0] = st->s_rad_done * f;
            sh_s[1] = st->s_m_done * f;
            sh_cnt = cnt;
            sh_E = Es;
        }
        __syncthreads();
    }
    if (FIRST) {
        for (int q = 0; q < 9; ++q) P.R[q] = st->R[q];
        for (int q = 0; q < 3; ++q) P.t[q] = st->t[q];
        P.s_rad = st->s_rad;
        P.s_m = st->s_m;
        P.it = (uint32_t)st->iter;
    } else {
        for (int q = 0; q < 9; ++q) P.R[q] = st->R_new[q];
        for (int q = 0; q < 3; ++q) P.t[q] = st->t_new[q];
        P.s_rad = sh_s[0];
        P.s_m = sh_s[1];
        P.it = (uint32_t)st->iter_done + 1u;
    }
    // particles of iteration `it` (Sec. IV-A alternation pairs them with the sampling rate), and
    // the stop rule on the updated search size s^(it)
    P.K_it = st->alt_K ? st->Ks[(P.it - 1u) % (uint32_t)st->n_rates] : st->K;
    P.stop = !FIRST && st->stop_rad > 0.0 && st->stop_m > 0.0 && P.s_rad < st->stop_rad && P.s_m < st->stop_m;
    __syncthreads();   // every thread has read the state before it is rewritten below
    if (!FIRST && lead) {
        const int i = st->iter_done;
        if (recs && i >= 1 && i <= PF_MAX_ITERS) {
            IterRec& r = recs[i - 1];
            r.E0 = (float)st->E0;
            r.Estar = sh_E;
            r.n_adv = st->n_adv;
            r.n_sub = st->n_sub;
            r.n_valid = sh_cnt;
            r.s_rad = st->s_rad_done;
            r.s_m = st->s_m_done;
            r.n_particles = st->K_cur;
        }
        st->Estar = (double)sh_E;
        st->n_valid_star = sh_cnt;
        for (int q = 0; q < 9; ++q) st->R[q] = P.R[q];
        for (int q = 0; q < 3; ++q) st->t[q] = P.t[q];
        st->s_rad = P.s_rad;
        st->s_m = P.s_m;
        st->iter = (int)P.it;
        st->K_cur = P.K_it;
        if (P.stop) st->done = 1;
    }
    return true;
}

// Particle k of the planned iteration: the delta (omega a[0:3], v a[3:6]) with a from the counter
// stream, composed with P in FP64 and rounded to FP32 into poses[k] (and into pose_copy when given);
// slot 0 is P itself with a zero delta.
__device__ inline void draw_particle(pf_track_state* st, const DrawPlan& P, int k, float* poses, float* pose_copy) {
    double* dl = state_deltas(st);
    if (k == 0) {
        store_pose12(poses, P.R, P.t);
        for (int d = 0; d < 6; ++d) dl[d] = 0.0;
        return;
    }
    const uint64_t seed = st->seed;
    const uint32_t fr = (uint32_t)st->frame_index;
    double r[3], tau[3];
    for (int d = 0; d < 3; ++d) r[d] = P.s_rad * draw_pm1(seed, fr, P.it, (uint32_t)k, (uint32_t)d);
    for (int d = 0; d < 3; ++d) tau[d] = P.s_m * draw_pm1(seed, fr, P.it, (uint32_t)k, (uint32_t)(3 + d));
    double Ro[9], to[3];
    apply_delta(st->compose_mode, r, tau, P.R, P.t, Ro, to);
    store_pose12(poses + (size_t)k * 12, Ro, to);
    if (pose_copy) store_pose12(pose_copy, Ro, to);
    for (int d = 0; d < 3; ++d) {
        dl[6 * k + d] = r[d];
        dl[6 * k + 3 + d] = tau[d];
    }
}

// The separate draw launch: completes iteration i (unless FIRST) and draws the K_(i+1) particles of
// the next one, particle k in thread k of the grid (draw = 0: completes only).
template <int FMT, bool FIRST>
__device__ inline void next_step(pf_track_state* st, int K, int n_partials, int draw, float* next_poses, IterRec* recs,
                                 int blk, int e0_partials = 0, float* fit0 = nullptr, int* nv0 = nullptr) {
    const int k = blk * 256 + threadIdx.x;
    DrawPlan P;
    if (!draw_prologue<FMT, FIRST>(st, K, n_partials, recs, blk == 0, k == 0, e0_partials, fit0, nv0, P)) return;
    if (draw && !P.stop && k <= P.K_it) draw_particle(st, P, k, next_poses, nullptr);
    __syncthreads();
}


int n_partials_for(int cap);

// The particle launch of iteration i that draws its own particles (K_i of them, 4 poses x 256
// threads, spread regime `regime` forecast, through the cell-validity mask when that regime reads
// it): first = iteration 1 (planned around the initial state; e0_partials = the initial pose's
// partials on the first view); otherwise it completes iteration i - 1 from the previous update
// step's n_partials partials (E*) and e0_partials second partials (E_0 of iteration i). Particles go
// to poses[1..K_i] (slot 0 = the pose they are drawn around), fitness to fit / nv [1..K_i] (slot 0 =
// E_0), iteration i - 1's record to recs.
int32_t launch_draw_score(const VolView& vv, const Points& S, pf_track_state* st, int K, int K_i, int n_partials,
                          bool first, IterRec* recs, int e0_partials, float* poses, float* fit, int* nv, int regime,
                          hipStream_t s);
// Loads that launch's code for a volume of this format and layout on the current device (once).
void warm_draw_score(int format, int layout);

}  // namespace pf
