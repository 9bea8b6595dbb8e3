// Randomized optimization of one frame on gfx950 (Sec. III-B; schedule of Sec. IV-A):
// back-projection and compaction of the depth image, the sub-sampled point views, the FP64
// optimizer state (advantage set, averaged delta, pose and search-size updates), the drawing and
// composition of the delta poses, and the device-resident loop that ties them to the scoring
// kernel. The loop keeps its state on the device: one host synchronisation per frame.
#include <math.h>
#include <string.h>

#include "pf_sample.hpp"

namespace pf {

// ------------------------------------------------------------------ optional kernel timing
struct Timing {
    bool on = false;
    double ms = 0.0;
    int64_t launches = 0, evals = 0;
    hipEvent_t ev[2 * (PF_MAX_ITERS + 1)] = {};
    bool created = false;
};
static Timing g_timing;

int32_t timing_enable(int on) {
    if (on && !g_timing.created) {
        for (auto& e : g_timing.ev)
            if (hipEventCreate(&e) != hipSuccess) return set_error(PF_EHIP, "pf_timing_enable: hipEventCreate failed");
        g_timing.created = true;
    }
    g_timing.on = on != 0;
    return PF_OK;
}

int32_t timing_read(double* ms, int64_t* launches, int64_t* evals, int reset) {
    if (ms) *ms = g_timing.ms;
    if (launches) *launches = g_timing.launches;
    if (evals) *evals = g_timing.evals;
    if (reset) {
        g_timing.ms = 0.0;
        g_timing.launches = g_timing.evals = 0;
    }
    return PF_OK;
}

namespace {

// ------------------------------------------------------------------ back-projection
constexpr int kBpThreads = 256;
constexpr int kBpPerThread = 4;
constexpr int kBpChunk = kBpThreads * kBpPerThread;  // pixels per workgroup, in raster order

struct BpArgs {
    const float* depth;
    int width, height, stride;
    float fx, fy, cx, cy;
};

__device__ inline bool bp_valid(const BpArgs& a, int pix, float& z) {
    const int n = a.width * a.height;
    if (pix >= n) return false;
    const int v = pix / a.width, u = pix - v * a.width;
    if ((u % a.stride) != 0 || (v % a.stride) != 0) return false;
    z = a.depth[pix];
    return isfinite(z) && z > 0.0f;
}

__global__ __launch_bounds__(kBpThreads) void k_bp_count(BpArgs a, int* counts) {
    const int base = blockIdx.x * kBpChunk + threadIdx.x * kBpPerThread;
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
        counts[blockIdx.x] = s;
    }
}

// Each workgroup sums the counts of the workgroups before it (a few hundred integers), scans
// its own pixels and writes them in raster order; workgroup 0 also writes the total.
__global__ __launch_bounds__(kBpThreads) void k_bp_scatter(BpArgs a, const int* counts, int nblocks, float* px,
                                                           float* py, float* pz, int* n_out) {
    __shared__ int red[kBpThreads / kWave];
    __shared__ int wsum[kBpThreads / kWave];
    __shared__ int base_sh, total_sh;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int before = 0, all = 0;
    for (int b = threadIdx.x; b < nblocks; b += kBpThreads) {
        const int c = counts[b];
        all += c;
        if (b < (int)blockIdx.x) before += c;
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
        if (blockIdx.x == 0) *n_out = t;
    }
    __syncthreads();
    // in-workgroup exclusive scan of the per-thread counts (thread order = raster order)
    const int pbase = blockIdx.x * kBpChunk + threadIdx.x * kBpPerThread;
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
            ++pos;
        }
    }
}

// S_r[j] = M[j r] for j < ceil(n / r), copied contiguously; the count goes to *n_view.
__global__ __launch_bounds__(256) void k_view(const float* px, const float* py, const float* pz, const int* n_all,
                                              int r, int cap, float* vx, float* vy, float* vz, int* n_view) {
    const int n = *n_all;
    const int m = (n + r - 1) / r;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j == 0) *n_view = m;
    if (j < m && j < cap) {
        vx[j] = px[j * r];
        vy[j] = py[j * r];
        vz[j] = pz[j * r];
    }
}

// ------------------------------------------------------------------ optimizer state
struct IterRec {
    float E0, Estar;
    int n_adv, n_sub, n_valid, pad;
    double s_rad, s_m;
};

struct Partial {
    float sum;
    int cnt;
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

__global__ void k_state_set(pf_track_state* st, pf_track_state init) { *st = init; }

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
template <int FMT, int LAYOUT, bool ADV>
__global__ __launch_bounds__(kAdvThreads) void k_adv(VolView vv, const float* __restrict__ px,
                                                     const float* __restrict__ py, const float* __restrict__ pz,
                                                     int n_host, const int* __restrict__ n_dev,
                                                     const float* __restrict__ fitness, pf_track_state* st, int K) {
    if (st->K != K) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->flags |= 1;
        return;
    }
    __shared__ float pose_sh[12];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int n = n_dev ? *n_dev : n_host;
    if constexpr (ADV) {
        const double* dl = state_deltas(st);
        const float E0 = fitness[0];
        double acc[6] = {0, 0, 0, 0, 0, 0};
        int na = 0;
        for (int k = 1 + threadIdx.x; k <= K; k += kAdvThreads) {
            if (fitness[k] < E0) {
#pragma unroll
                for (int d = 0; d < 6; ++d) acc[d] += dl[6 * k + d];
                na += 1;
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
            if (blockIdx.x == 0) {
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
    // this workgroup's chunk of the view, scored with the scoring kernel's arithmetic
    const Gather<FMT, LAYOUT> G = make_gather<FMT, LAYOUT>(vv);
    GridPose g[1] = {fold_pose(pose_sh, vv.inv_vs, vv.gx0, vv.gy0, vv.gz0)};
    const unsigned lx = (unsigned)(vv.nx - 1), ly = (unsigned)(vv.ny - 1), lz = (unsigned)(vv.nz - 1);
    const int chunk = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    const int q0 = (int)blockIdx.x * chunk, q1 = min(n, q0 + chunk);
    float sum[1] = {0.0f};
    int cnt[1] = {0};
    const float sc = vv.inv_vs;
    for (int q = q0 + (int)threadIdx.x; q < q1; q += kAdvThreads)
        eval_poses<FMT, LAYOUT, 1>(G, lx, ly, lz, g, px[q] * sc, py[q] * sc, pz[q] * sc, sum, cnt);
    block_reduce<1, kAdvThreads>(sum, cnt);
    if (threadIdx.x == 0) {
        Partial* pt = state_partials(st, K);
        pt[blockIdx.x].sum = sum[0];
        pt[blockIdx.x].cnt = cnt[0];
    }
}

// Completes iteration i (unless FIRST) and draws the K particles of the next one:
// E* from the partials in order, s^(i+1) = s^(i) (beta + (1 - beta) E*), then particle k is the
// delta (omega a[0:3], v a[3:6]) with a from the counter stream, composed with P^(i) in FP64 and
// rounded to FP32; slot 0 is P^(i). FIRST draws iteration 1 around the initial state.
template <int FMT, bool FIRST>
__global__ __launch_bounds__(256) void k_next(pf_track_state* st, int K, int n_partials, int draw,
                                              float* next_poses, IterRec* recs) {
    if (st->K != K) return;
    __shared__ double sh_s[2];
    __shared__ int sh_cnt;
    __shared__ float sh_E;
    if (!FIRST && threadIdx.x == 0) {
        const Partial* pt = state_partials(st, K);
        float sum = 0.0f;
        int cnt = 0;
        for (int b = 0; b < n_partials; ++b) {
            sum += pt[b].sum;
            cnt += pt[b].cnt;
        }
        const float Es = cnt > 0 ? (sum * Fmt<FMT>::scale) / (float)cnt : 1.0f;
        const double f = st->beta + (1.0 - st->beta) * (double)Es;
        sh_s[0] = st->s_rad_done * f;
        sh_s[1] = st->s_m_done * f;
        sh_cnt = cnt;
        sh_E = Es;
    }
    __syncthreads();
    const int k = blockIdx.x * 256 + threadIdx.x;
    double R[9], t[3], s_rad, s_m;
    uint32_t it;
    if (FIRST) {
        for (int q = 0; q < 9; ++q) R[q] = st->R[q];
        for (int q = 0; q < 3; ++q) t[q] = st->t[q];
        s_rad = st->s_rad;
        s_m = st->s_m;
        it = (uint32_t)st->iter;
    } else {
        for (int q = 0; q < 9; ++q) R[q] = st->R_new[q];
        for (int q = 0; q < 3; ++q) t[q] = st->t_new[q];
        s_rad = sh_s[0];
        s_m = sh_s[1];
        it = (uint32_t)st->iter_done + 1u;
        if (k == 0) {
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
            }
            st->Estar = (double)sh_E;
            st->n_valid_star = sh_cnt;
            for (int q = 0; q < 9; ++q) st->R[q] = R[q];
            for (int q = 0; q < 3; ++q) st->t[q] = t[q];
            st->s_rad = s_rad;
            st->s_m = s_m;
            st->iter = (int)it;
        }
    }
    if (!draw || k > K) return;
    double* dl = state_deltas(st);
    if (k == 0) {
        store_pose12(next_poses, R, t);
        for (int d = 0; d < 6; ++d) dl[d] = 0.0;
        return;
    }
    const uint64_t seed = st->seed;
    const uint32_t fr = (uint32_t)st->frame_index;
    double r[3], tau[3];
    for (int d = 0; d < 3; ++d) r[d] = s_rad * draw_pm1(seed, fr, it, (uint32_t)k, (uint32_t)d);
    for (int d = 0; d < 3; ++d) tau[d] = s_m * draw_pm1(seed, fr, it, (uint32_t)k, (uint32_t)(3 + d));
    double Ro[9], to[3];
    apply_delta(st->compose_mode, r, tau, R, t, Ro, to);
    store_pose12(next_poses + (size_t)k * 12, Ro, to);
    for (int d = 0; d < 3; ++d) {
        dl[6 * k + d] = r[d];
        dl[6 * k + 3 + d] = tau[d];
    }
}

int n_partials_for(int cap) {
    const int g = (cap + 511) / 512;
    return g < 1 ? 1 : (g > kMaxPartials ? kMaxPartials : g);
}

template <int FMT, int LAYOUT>
int32_t launch_adv_t(bool adv, const VolView& vv, const Points& p, int G, const float* fitness, pf_track_state* st,
                     int K, hipStream_t s) {
    if (adv)
        hipLaunchKernelGGL((k_adv<FMT, LAYOUT, true>), dim3(G), dim3(kAdvThreads), 0, s, vv, p.x, p.y, p.z, p.n,
                           p.n_dev, fitness, st, K);
    else
        hipLaunchKernelGGL((k_adv<FMT, LAYOUT, false>), dim3(G), dim3(kAdvThreads), 0, s, vv, p.x, p.y, p.z, p.n,
                           p.n_dev, fitness, st, K);
    return check_launch("particles_update");
}

// adv = true: advantage set, P^(i) and the partials of E*; false: partials of the pending pose.
int32_t launch_adv(bool adv, const VolView& vv, const Points& p, int G, const float* fitness, pf_track_state* st,
                   int K, hipStream_t s) {
    const bool cells = vv.layout == PF_LAYOUT_CELLS;
    switch (vv.format) {
        case PF_F32_W_F32:
            return cells ? launch_adv_t<PF_F32_W_F32, PF_LAYOUT_CELLS>(adv, vv, p, G, fitness, st, K, s)
                         : launch_adv_t<PF_F32_W_F32, PF_LAYOUT_LINEAR>(adv, vv, p, G, fitness, st, K, s);
        case PF_F16_W_U8:
            return cells ? launch_adv_t<PF_F16_W_U8, PF_LAYOUT_CELLS>(adv, vv, p, G, fitness, st, K, s)
                         : launch_adv_t<PF_F16_W_U8, PF_LAYOUT_LINEAR>(adv, vv, p, G, fitness, st, K, s);
        case PF_I16_W_U8:
            return cells ? launch_adv_t<PF_I16_W_U8, PF_LAYOUT_CELLS>(adv, vv, p, G, fitness, st, K, s)
                         : launch_adv_t<PF_I16_W_U8, PF_LAYOUT_LINEAR>(adv, vv, p, G, fitness, st, K, s);
        default: return set_error(PF_EUNSUPPORTED, "unsupported format %d", vv.format);
    }
}

int32_t launch_next(int format, bool first, pf_track_state* st, int K, int G, bool draw, float* next_poses,
                    IterRec* recs, hipStream_t s) {
    const int blocks = draw ? (K + 1 + 255) / 256 : 1;
    const int d = draw ? 1 : 0;
#define PF_NEXT(F)                                                                                              \
    if (first)                                                                                                  \
        hipLaunchKernelGGL((k_next<F, true>), dim3(blocks), dim3(256), 0, s, st, K, G, d, next_poses, recs); \
    else                                                                                                        \
        hipLaunchKernelGGL((k_next<F, false>), dim3(blocks), dim3(256), 0, s, st, K, G, d, next_poses, recs);
    switch (format) {
        case PF_F32_W_F32: PF_NEXT(PF_F32_W_F32) break;
        case PF_F16_W_U8: PF_NEXT(PF_F16_W_U8) break;
        case PF_I16_W_U8: PF_NEXT(PF_I16_W_U8) break;
        default: return set_error(PF_EUNSUPPORTED, "unsupported format %d", format);
    }
#undef PF_NEXT
    return check_launch("particle draw");
}

pf_track_state make_state(const pf_pose* init, const pf_track_params* p) {
    pf_track_state h;
    memset(&h, 0, sizeof h);
    for (int q = 0; q < 9; ++q) h.R[q] = init->R[q];
    for (int q = 0; q < 3; ++q) h.t[q] = init->t[q];
    h.s_rad = p->s1_deg * (M_PI / 180.0);
    h.s_m = p->s1_m;
    h.beta = p->beta;
    h.E0 = h.Estar = 1.0;
    h.seed = p->seed;
    h.frame_index = p->frame_index;
    h.iter = 1;
    h.K = p->K;
    h.compose_mode = p->compose_mode;
    return h;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
    size_t pts, counts, views[3], vcount, poses, fit, nv, state, recs, polish, fin, total;
};

WsLayout ws_layout(const pf_intrinsics* K, const pf_track_params* p) {
    WsLayout L;
    const size_t npix = (size_t)K->width * K->height;
    size_t off = 0;
    L.pts = off;
    off += align_up(3 * npix * sizeof(float));
    L.counts = off;
    off += align_up(((npix + kBpChunk - 1) / kBpChunk + 1) * sizeof(int));
    for (int r = 0; r < 3; ++r) {
        L.views[r] = off;
        if (r < p->n_rates && p->rates[r] > 1) {
            const size_t m = (npix + p->rates[r] - 1) / p->rates[r];
            off += align_up(3 * m * sizeof(float));
        }
    }
    L.vcount = off;
    off += align_up(8 * sizeof(int));
    L.poses = off;
    off += align_up((size_t)(p->K + 1) * 12 * sizeof(float));
    L.fit = off;
    off += align_up((size_t)(p->K + 1) * sizeof(float));
    L.nv = off;
    off += align_up((size_t)(p->K + 1) * sizeof(int));
    L.state = off;
    off += align_up(partials_offset(p->K) + kMaxPartials * sizeof(Partial));
    L.recs = off;
    off += align_up(PF_MAX_ITERS * sizeof(IterRec) + 2 * sizeof(int));
    L.polish = off;
    off += align_up(polish_scratch_bytes(kMaxPartials));
    L.fin = off;
    off += align_up(256 + kMaxPartials * 8);
    L.total = off;
    return L;
}

}  // namespace

size_t state_bytes(int K) { return partials_offset(K) + kMaxPartials * sizeof(Partial); }

int32_t launch_backproject(const float* depth, const pf_intrinsics* K, int stride, float* px, float* py, float* pz,
                           int* n_out, int* block_counts, hipStream_t s) {
    BpArgs a;
    a.depth = depth;
    a.width = K->width;
    a.height = K->height;
    a.stride = stride;
    a.fx = (float)K->fx;
    a.fy = (float)K->fy;
    a.cx = (float)K->cx;
    a.cy = (float)K->cy;
    const int npix = K->width * K->height;
    const int nb = (npix + kBpChunk - 1) / kBpChunk;
    hipLaunchKernelGGL(k_bp_count, dim3(nb), dim3(kBpThreads), 0, s, a, block_counts);
    int32_t rc = check_launch("backproject");
    if (rc) return rc;
    hipLaunchKernelGGL(k_bp_scatter, dim3(nb), dim3(kBpThreads), 0, s, a, block_counts, nb, px, py, pz, n_out);
    return check_launch("backproject");
}

size_t backproject_scratch_ints(const pf_intrinsics* K) {
    const size_t npix = (size_t)K->width * K->height;
    return (npix + kBpChunk - 1) / kBpChunk + 1;
}

int32_t state_init(void* state, const pf_pose* init, const pf_track_params* p, int format, float* next_poses,
                   hipStream_t s) {
    pf_track_state h = make_state(init, p);
    pf_track_state* st = static_cast<pf_track_state*>(state);
    hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, s, st, h);
    int32_t rc = check_launch("particles_state_init");
    if (rc) return rc;
    return launch_next(format, true, st, p->K, 0, true, next_poses, nullptr, s);
}

int32_t update(const VolView& vv, const Points& pts, const float* fitness, void* state, int K, float* next_poses,
               hipStream_t s) {
    pf_track_state* st = static_cast<pf_track_state*>(state);
    const int G = n_partials_for(pts.n);
    int32_t rc = launch_adv(true, vv, pts, G, fitness, st, K, s);
    if (rc) return rc;
    return launch_next(vv.format, false, st, K, G, true, next_poses, nullptr, s);
}

size_t workspace_bytes(const pf_intrinsics* K, const pf_track_params* p) { return ws_layout(K, p).total; }

int32_t track(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* init,
              const pf_track_params* p, pf_pose* out, pf_track_stats* stats, void* workspace, size_t ws_bytes,
              hipStream_t s) {
    const WsLayout L = ws_layout(K, p);
    if (ws_bytes < L.total)
        return set_error(PF_ENOMEM, "track_frame: workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    char* ws = static_cast<char*>(workspace);
    const size_t npix = (size_t)K->width * K->height;
    float* px = reinterpret_cast<float*>(ws + L.pts);
    float* py = px + npix;
    float* pz = py + npix;
    int* counts = reinterpret_cast<int*>(ws + L.counts);
    int* vcount = reinterpret_cast<int*>(ws + L.vcount);  // [0] = n, [1 + r] = |S_r|
    float* poses = reinterpret_cast<float*>(ws + L.poses);
    float* fit = reinterpret_cast<float*>(ws + L.fit);
    int* nv = reinterpret_cast<int*>(ws + L.nv);
    pf_track_state* st = reinterpret_cast<pf_track_state*>(ws + L.state);
    IterRec* recs = reinterpret_cast<IterRec*>(ws + L.recs);
    const VolView vv = make_view(v);

    int32_t rc = launch_backproject(depth, K, p->pixel_stride, px, py, pz, vcount, counts, s);
    if (rc) return rc;
    Points views[3];
    for (int r = 0; r < p->n_rates; ++r) {
        const int rate = p->rates[r];
        if (rate == 1) {
            views[r] = Points{px, py, pz, 0, vcount};
            continue;
        }
        const int cap = (int)((npix + rate - 1) / rate);
        float* vx = reinterpret_cast<float*>(ws + L.views[r]);
        float* vy = vx + cap;
        float* vz = vy + cap;
        hipLaunchKernelGGL(k_view, dim3((cap + 255) / 256), dim3(256), 0, s, px, py, pz, vcount, rate, cap, vx, vy,
                           vz, vcount + 1 + r);
        if ((rc = check_launch("track_frame views"))) return rc;
        views[r] = Points{vx, vy, vz, 0, vcount + 1 + r};
    }
    if ((rc = state_init(st, init, p, vv.format, poses, s))) return rc;
    const bool timed = g_timing.on;
    int Gv[3];
    for (int r = 0; r < p->n_rates; ++r) Gv[r] = n_partials_for((int)((npix + p->rates[r] - 1) / p->rates[r]));
    for (int i = 1; i <= p->n_iters; ++i) {
        const int r = (i - 1) % p->n_rates;
        const Points& S = views[r];
        if (timed) (void)hipEventRecord(g_timing.ev[2 * (i - 1)], s);
        if ((rc = launch_score(vv, S, poses, p->K + 1, fit, nv, s))) return rc;
        if (timed) (void)hipEventRecord(g_timing.ev[2 * (i - 1) + 1], s);
        if ((rc = launch_adv(true, vv, S, Gv[r], fit, st, p->K, s))) return rc;
        // the last iteration only completes (E*, s); its particles stay in `poses` / `fit`
        if ((rc = launch_next(vv.format, false, st, p->K, Gv[r], i < p->n_iters, poses, recs, s))) return rc;
    }
    // optional gradient polish of the best candidate, on the densest view
    int densest = 0;
    for (int r = 1; r < p->n_rates; ++r)
        if (p->rates[r] < p->rates[densest]) densest = r;
    if (p->polish_steps > 0 &&
        (rc = launch_polish(vv, views[densest], Gv[densest], st, p->K, fit, p->compose_mode, v->voxel_size,
                            p->polish_steps, ws + L.polish, s)))
        return rc;
    // fitness of the returned pose on the densest view
    float* ef_dev = reinterpret_cast<float*>(recs + PF_MAX_ITERS);
    int* nvf_dev = reinterpret_cast<int*>(ef_dev + 1);
    if ((rc = launch_state_fitness(vv, views[densest], Gv[densest], st, ws + L.fin, ef_dev, nvf_dev, s))) return rc;

    pf_track_state hs;
    IterRec hr[PF_MAX_ITERS];
    float ef;
    int nvf, nall, accepted = 0;
    if (hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(hr, recs, sizeof(IterRec) * p->n_iters, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&ef, ef_dev, sizeof ef, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&nvf, nvf_dev, sizeof nvf, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&nall, vcount, sizeof nall, hipMemcpyDeviceToHost, s) != hipSuccess ||
        (p->polish_steps > 0 && hipMemcpyAsync(&accepted, ws + L.polish + polish_accepted_offset(), sizeof accepted,
                                               hipMemcpyDeviceToHost, s) != hipSuccess))
        return set_error(PF_EHIP, "track_frame: read-back failed: %s", hipGetErrorString(hipGetLastError()));
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(PF_EHIP, "track_frame: %s", hipGetErrorString(e));
    if (hs.flags) return set_error(PF_EINVAL, "track_frame: inconsistent optimizer state (flags %d)", hs.flags);
    if (timed) {
        for (int i = 0; i < p->n_iters; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, g_timing.ev[2 * i], g_timing.ev[2 * i + 1]) == hipSuccess) g_timing.ms += ms;
            g_timing.launches += 1;
            g_timing.evals += (int64_t)(p->K + 1) * hr[i].n_sub;
        }
    }
    for (int q = 0; q < 9; ++q) out->R[q] = hs.R[q];
    for (int q = 0; q < 3; ++q) out->t[q] = hs.t[q];
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->n_points = nall;
        stats->n_iters = p->n_iters;
        for (int i = 0; i < p->n_iters; ++i) {
            stats->E0[i] = hr[i].E0;
            stats->Estar[i] = hr[i].Estar;
            stats->n_adv[i] = hr[i].n_adv;
            stats->n_sub[i] = hr[i].n_sub;
            stats->n_valid[i] = hr[i].n_valid;
            stats->s_rad[i] = hr[i].s_rad;
            stats->s_m[i] = hr[i].s_m;
        }
        stats->E_final = ef;
        stats->polish_accepted = accepted;
        stats->n_valid_final = nvf;
        stats->lost = nvf < p->min_valid ? 1 : 0;
    }
    return PF_OK;
}

}  // namespace pf
