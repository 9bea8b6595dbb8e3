// Randomized optimization of one frame on gfx950 (Sec. III-B; schedule of Sec. IV-A):
// back-projection and compaction of the depth image, the sub-sampled point views, the FP64
// optimizer state (advantage set, averaged delta, pose and search-size updates), the drawing and
// composition of the delta poses, and the device-resident loop that ties them to the scoring
// kernel. The loop keeps its state on the device: one host synchronisation per frame.
#include <math.h>
#include <string.h>

#include "pf_steps.hpp"

namespace pf {

// ------------------------------------------------------------------ optional kernel timing
// Per host thread: each thread that calls track_frame brackets its own launches with its own
// events and accumulates its own counters, so concurrent callers do not share event slots.
struct Timing {
    bool on = false;
    double ms = 0.0;
    int64_t launches = 0, evals = 0;
    hipEvent_t ev[2 * (PF_MAX_ITERS + 1)] = {};
    bool created = false;
};
thread_local Timing g_timing;

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

// ------------------------------------------------------------------ single-problem kernels
__global__ __launch_bounds__(kBpThreads) void k_bp_count(BpArgs a, int* counts) { bp_count_step(a, counts, blockIdx.x); }

__global__ __launch_bounds__(kBpThreads) void k_bp_scatter(BpArgs a, const int* counts, int nblocks, float* px,
                                                           float* py, float* pz, int* n_out) {
    bp_scatter_step(a, counts, nblocks, px, py, pz, n_out, blockIdx.x);
}

// The sub-sampled views of a frame, built together: blockIdx.y is the view.
struct ViewSet {
    int rate[3];
    ViewTiles t[3];
    float* vx[3];
    float* vy[3];
    float* vz[3];
    int* n_view[3];
};

__global__ __launch_bounds__(256) void k_view_mark(const int* pix, const int* n_all, int width, ViewSet v) {
    view_mark_step(pix, n_all, v.rate[blockIdx.y], width, v.t[blockIdx.y], blockIdx.x);
}

__global__ __launch_bounds__(256) void k_view_scan(ViewSet v) { view_scan_step(v.t[blockIdx.x]); }

__global__ __launch_bounds__(256) void k_view_scatter(const float* px, const float* py, const float* pz, const int* pix,
                                                      const int* n_all, int width, ViewSet v) {
    const int y = blockIdx.y;
    view_scatter_step(px, py, pz, pix, n_all, v.rate[y], width, v.t[y], v.vx[y], v.vy[y], v.vz[y], v.n_view[y],
                      blockIdx.x);
}

__global__ void k_state_set(pf_track_state* st, pf_track_state init) { *st = init; }

// What track_frame reads back at the end of a frame, gathered into one block so that one copy
// brings it to the host.
struct Readback {
    pf_track_state st;
    IterRec recs[PF_MAX_ITERS];
    float ef;
    int nvf, nall, accepted;
};

__global__ __launch_bounds__(256) void k_readback(const pf_track_state* st, const IterRec* recs, const float* ef,
                                                  const int* nvf, const int* nall, const int* accepted,
                                                  Readback* rb) {
    const unsigned* a = reinterpret_cast<const unsigned*>(st);
    unsigned* b = reinterpret_cast<unsigned*>(&rb->st);
    for (int q = threadIdx.x; q < (int)(sizeof(pf_track_state) / 4); q += 256) b[q] = a[q];
    const unsigned* c = reinterpret_cast<const unsigned*>(recs);
    unsigned* d = reinterpret_cast<unsigned*>(rb->recs);
    for (int q = threadIdx.x; q < (int)(sizeof(rb->recs) / 4); q += 256) d[q] = c[q];
    if (threadIdx.x == 0) {
        rb->ef = *ef;
        rb->nvf = *nvf;
        rb->nall = *nall;
        rb->accepted = accepted ? *accepted : 0;
    }
}

template <int FMT, int LAYOUT, bool ADV>
__global__ __launch_bounds__(kAdvThreads) void k_adv(VolView vv, const float* __restrict__ px,
                                                     const float* __restrict__ py, const float* __restrict__ pz,
                                                     int n_host, const int* __restrict__ n_dev,
                                                     const float* __restrict__ fitness, pf_track_state* st, int K,
                                                     NextView nv) {
    adv_step<FMT, LAYOUT, ADV>(vv, px, py, pz, n_host, n_dev, fitness, st, K, blockIdx.x, gridDim.x, nv);
}

template <int FMT, bool FIRST>
__global__ __launch_bounds__(256) void k_next(pf_track_state* st, int K, int n_partials, int draw,
                                              float* next_poses, IterRec* recs, int e0_partials, float* fit0,
                                              int* nv0) {
    next_step<FMT, FIRST>(st, K, n_partials, draw, next_poses, recs, blockIdx.x, e0_partials, fit0, nv0);
}

}  // namespace

int n_partials_for(int cap) {
    const int g = (cap + 511) / 512;
    return g < 1 ? 1 : (g > kMaxPartials ? kMaxPartials : g);
}

namespace {

template <int FMT, int LAYOUT>
int32_t launch_adv_t(bool adv, const VolView& vv, const Points& p, int G, const float* fitness, pf_track_state* st,
                     int K, const NextView& nv, hipStream_t s) {
    if (adv)
        hipLaunchKernelGGL((k_adv<FMT, LAYOUT, true>), dim3(G), dim3(kAdvThreads), 0, s, vv, p.x, p.y, p.z, p.n,
                           p.n_dev, fitness, st, K, nv);
    else
        hipLaunchKernelGGL((k_adv<FMT, LAYOUT, false>), dim3(G), dim3(kAdvThreads), 0, s, vv, p.x, p.y, p.z, p.n,
                           p.n_dev, fitness, st, K, nv);
    return check_launch("particles_update");
}

// adv = true: advantage set, P^(i) and the partials of E*; false: partials of the pending pose.
// With a next view, also the partials of that pose on it (the next iteration's E_0).
int32_t launch_adv(bool adv, const VolView& vv, const Points& p, int G, const float* fitness, pf_track_state* st,
                   int K, hipStream_t s, const NextView& nv = NextView{nullptr, nullptr, nullptr, nullptr}) {
    return with_volume(vv.format, vv.layout, [&](auto fmt, auto layout) {
        return launch_adv_t<decltype(fmt)::value, decltype(layout)::value>(adv, vv, p, G, fitness, st, K, nv, s);
    });
}

// e0_partials > 0: also turns the second partials into the drawn iteration's E_0 at fit0[0] / nv0[0].
int32_t launch_next(int format, bool first, pf_track_state* st, int K, int G, bool draw, float* next_poses,
                    IterRec* recs, hipStream_t s, int e0_partials = 0, float* fit0 = nullptr, int* nv0 = nullptr) {
    const int blocks = draw ? (K + 1 + 255) / 256 : 1;
    const int d = draw ? 1 : 0;
#define PF_NEXT(F)                                                                                             \
    if (first)                                                                                                 \
        hipLaunchKernelGGL((k_next<F, true>), dim3(blocks), dim3(256), 0, s, st, K, G, d, next_poses, recs,   \
                           e0_partials, fit0, nv0);                                                            \
    else                                                                                                       \
        hipLaunchKernelGGL((k_next<F, false>), dim3(blocks), dim3(256), 0, s, st, K, G, d, next_poses, recs,  \
                           e0_partials, fit0, nv0);
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
    h.alt_K = p->alt_K;
    h.n_rates = p->n_rates;
    for (int r = 0; r < 3; ++r) h.Ks[r] = p->Ks[r];
    h.K_cur = p->alt_K ? p->Ks[0] : p->K;
    h.done = 0;
    h.stop_rad = p->stop_deg * (M_PI / 180.0);
    h.stop_m = p->stop_m;
    return h;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
    size_t pts, pix, counts, views[3], tiles_mask[3], tiles_start[3], vcount, poses, fit, nv, state, recs, polish, fin,
        rb, fuse, total;
};

WsLayout ws_layout(const pf_intrinsics* K, const pf_track_params* p) {
    WsLayout L;
    const size_t npix = (size_t)K->width * K->height;
    size_t off = 0;
    L.pts = off;
    off += align_up(3 * npix * sizeof(float));
    L.pix = off;
    off += align_up(npix * sizeof(int));
    L.counts = off;
    off += align_up(((npix + kBpChunk - 1) / kBpChunk + 1) * sizeof(int));
    // views, then the views' tile masks back to back (cleared as one range), then the tile starts
    size_t nt[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r) {
        L.views[r] = off;
        if (r < p->n_rates && p->rates[r] > 1) {
            const size_t m = (npix + p->rates[r] - 1) / p->rates[r];
            off += align_up(3 * m * sizeof(float));
            nt[r] = (size_t)view_n_tiles(K->width, K->height, p->rates[r]);
        }
    }
    for (int r = 0; r < 3; ++r) {
        L.tiles_mask[r] = off;
        off += nt[r] * sizeof(unsigned long long);
    }
    off = align_up(off);
    for (int r = 0; r < 3; ++r) {
        L.tiles_start[r] = off;
        off += nt[r] * sizeof(int);
    }
    off = align_up(off);
    L.vcount = off;
    off += align_up(8 * sizeof(int));
    L.poses = off;
    off += align_up((size_t)(p->K + 1) * 12 * sizeof(float));
    L.fit = off;
    off += align_up((size_t)(p->K + 1) * sizeof(float));
    L.nv = off;
    off += align_up((size_t)(p->K + 1) * sizeof(int));
    L.state = off;
    off += align_up(partials_offset(p->K) + 2 * kMaxPartials * sizeof(Partial));
    L.recs = off;
    off += align_up(PF_MAX_ITERS * sizeof(IterRec) + 2 * sizeof(int));
    L.polish = off;
    off += align_up(polish_scratch_bytes(kMaxPartials));
    L.fin = off;
    off += align_up(256 + kMaxPartials * 8);
    L.rb = off;
    off += align_up(sizeof(Readback));
    L.fuse = off;   // the arguments of the fusion at the tracked pose (track_frame_fuse)
    off += align_up(fuse_args_bytes());
    L.total = off;
    return L;
}

}  // namespace

size_t state_bytes(int K) { return partials_offset(K) + 2 * kMaxPartials * sizeof(Partial); }

pf_track_state initial_state(const pf_pose* init, const pf_track_params* p) { return make_state(init, p); }

int32_t launch_backproject(const float* depth, const pf_intrinsics* K, int stride, float* px, float* py, float* pz,
                           int* n_out, int* block_counts, hipStream_t s, int* pix, unsigned long long* masks,
                           int n_masks) {
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
    a.pix = pix;
    a.masks = masks;
    a.n_masks = n_masks;
    a.nblocks = nb;
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

namespace {

// The spread regime of every iteration of the last call on this thread, and the parameters it ran
// with. The search size contracts along much the same path frame after frame, so a call with the
// same parameters launches, per iteration, only the scoring launch of the regime that iteration had
// last time, instead of one regime-gated launch per regime (all but one of which return at once).
// A wrong forecast costs speed only: the sums are exact whatever the launch.
struct RegimeForecast {
    bool valid = false;
    int K = 0, n_iters = 0, n_rates = 0, alt_K = 0, rates[3] = {}, Ks[3] = {};
    float inv_vs = 0.0f;
    int regime[PF_MAX_ITERS] = {};
};
thread_local RegimeForecast g_forecast;

bool forecast_matches(const RegimeForecast& f, const pf_track_params* p, float inv_vs) {
    if (!f.valid || f.K != p->K || f.n_iters != p->n_iters || f.n_rates != p->n_rates || f.alt_K != p->alt_K ||
        f.inv_vs != inv_vs)
        return false;
    for (int r = 0; r < 3; ++r)
        if (f.rates[r] != p->rates[r] || f.Ks[r] != p->Ks[r]) return false;
    return true;
}

}  // namespace

// The read-back of a call that fuses: pinned host memory (a copy into it does not wait for the host)
// and an event after the copy, both per host thread, allocated on the first such call and kept.
thread_local Readback* g_pinned_rb = nullptr;
thread_local hipEvent_t g_rb_event[64] = {};

int32_t fuse_readback(Readback** rb, hipEvent_t* ev) {
    if (!g_pinned_rb && hipHostMalloc(reinterpret_cast<void**>(&g_pinned_rb), sizeof(Readback), hipHostMallocDefault) !=
                            hipSuccess) {
        g_pinned_rb = nullptr;
        return set_error(PF_EHIP, "track_frame_fuse: pinned read-back buffer: %s", hipGetErrorString(hipGetLastError()));
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return set_error(PF_EHIP, "track_frame_fuse: no current device below 64");
    if (!g_rb_event[dev] && hipEventCreateWithFlags(&g_rb_event[dev], hipEventDisableTiming) != hipSuccess) {
        g_rb_event[dev] = nullptr;
        return set_error(PF_EHIP, "track_frame_fuse: event: %s", hipGetErrorString(hipGetLastError()));
    }
    *rb = g_pinned_rb;
    *ev = g_rb_event[dev];
    return PF_OK;
}

int32_t track(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* init,
              const pf_track_params* p, pf_pose* out, pf_track_stats* stats, void* workspace, size_t ws_bytes,
              hipStream_t s, bool fuse) {
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

    // the views' tile masks sit one after another, so the count step clears them as one range
    int* pixv = reinterpret_cast<int*>(ws + L.pix);
    ViewSet vs{};
    Points views[3];
    int nviews = 0, max_blocks = 0, n_masks = 0;
    for (int r = 0; r < p->n_rates; ++r) {
        const int rate = p->rates[r];
        if (rate == 1) {
            views[r] = Points{px, py, pz, 0, vcount};
            continue;
        }
        const int cap = (int)((npix + rate - 1) / rate);
        float* vx = reinterpret_cast<float*>(ws + L.views[r]);
        const int y = nviews++;
        vs.rate[y] = rate;
        vs.t[y] = ViewTiles{reinterpret_cast<unsigned long long*>(ws + L.tiles_mask[r]),
                            reinterpret_cast<int*>(ws + L.tiles_start[r]), view_tiles_x(K->width, rate),
                            view_n_tiles(K->width, K->height, rate)};
        vs.vx[y] = vx;
        vs.vy[y] = vx + cap;
        vs.vz[y] = vx + 2 * cap;
        vs.n_view[y] = vcount + 1 + r;
        max_blocks = max_blocks > (cap + 255) / 256 ? max_blocks : (cap + 255) / 256;
        n_masks += vs.t[y].n_tiles;
        views[r] = Points{vs.vx[y], vs.vy[y], vs.vz[y], 0, vs.n_view[y]};
    }
    int32_t rc = launch_backproject(depth, K, p->pixel_stride, px, py, pz, vcount, counts, s, pixv,
                                    reinterpret_cast<unsigned long long*>(ws + L.tiles_mask[0]), n_masks);
    if (rc) return rc;
    if (nviews) {
        hipLaunchKernelGGL(k_view_mark, dim3(max_blocks, nviews), dim3(256), 0, s, pixv, vcount, K->width, vs);
        hipLaunchKernelGGL(k_view_scan, dim3(nviews), dim3(256), 0, s, vs);
        hipLaunchKernelGGL(k_view_scatter, dim3(max_blocks, nviews), dim3(256), 0, s, px, py, pz, pixv, vcount,
                           K->width, vs);
        if ((rc = check_launch("track_frame views"))) return rc;
    }
    // Iterations whose particle launch draws its own particles: those with a regime forecast and
    // the automatic 4 x 256 shape (the others keep the separate draw launch)
    const bool forecast = forecast_matches(g_forecast, p, vv.inv_vs);
    bool fused[PF_MAX_ITERS + 2] = {};
    for (int i = 1; i <= p->n_iters; ++i) {
        const int K_i = p->alt_K ? p->Ks[(i - 1) % p->n_rates] : p->K;
        fused[i] = forecast && g_forecast.regime[i - 1] >= 0 && score_auto_4x256(K_i);
    }
    if (score_auto_4x256(p->K)) warm_draw_score(vv.format, vv.layout);
    // the initial state, the initial pose scored on the first view (slot 0 of iteration 1) and
    // the particles of iteration 1
    const int G1 = n_partials_for((int)((npix + p->rates[0] - 1) / p->rates[0]));
    {
        pf_track_state h = make_state(init, p);
        hipLaunchKernelGGL(k_state_set, dim3(1), dim3(1), 0, s, st, h);
        if ((rc = check_launch("track_frame"))) return rc;
        const Points& S1 = views[0];
        const NextView nv1{S1.x, S1.y, S1.z, S1.n_dev};
        if ((rc = launch_adv(false, vv, S1, G1, fit, st, p->K, s, nv1))) return rc;
        if (!fused[1] && (rc = launch_next(vv.format, true, st, p->K, 0, true, poses, nullptr, s, G1, fit, nv)))
            return rc;
    }
    const bool timed = g_timing.on;
    int Gv[3];
    for (int r = 0; r < p->n_rates; ++r) Gv[r] = n_partials_for((int)((npix + p->rates[r] - 1) / p->rates[r]));
    int densest = 0;
    for (int r = 1; r < p->n_rates; ++r)
        if (p->rates[r] < p->rates[densest]) densest = r;
    float* ef_dev = reinterpret_cast<float*>(recs + PF_MAX_ITERS);
    int* nvf_dev = reinterpret_cast<int*>(ef_dev + 1);
    // With no polish and no stop rule the returned pose is P^(I): the last update step scores it on
    // the densest view as it goes (E_final), instead of a separate pass after the loop.
    const bool final_in_loop = p->polish_steps == 0 && !(p->stop_deg > 0.0 && p->stop_m > 0.0);
    int G_prev = G1;   // partials of the previous update step: its E* and this iteration's E_0
    for (int i = 1; i <= p->n_iters; ++i) {
        const int r = (i - 1) % p->n_rates;
        const Points& S = views[r];
        const int K_i = p->alt_K ? p->Ks[r] : p->K;
        if (timed) (void)hipEventRecord(g_timing.ev[2 * (i - 1)], s);
        const int expect = forecast ? g_forecast.regime[i - 1] : -1;
        // the particles 1..K_i; slot 0 (E_0, the current pose on this view) was scored by the
        // previous update step
        const Points Sp{S.x, S.y, S.z, S.n, S.n_dev};
        if (fused[i])
            rc = launch_draw_score(vv, Sp, st, p->K, K_i, G_prev, i == 1, recs, G_prev, poses, fit, nv, expect, s);
        else
            rc = launch_score(vv, Sp, poses + 12, K_i, fit + 1, nv + 1, s, st, expect);
        if (rc) return rc;
        if (timed) (void)hipEventRecord(g_timing.ev[2 * (i - 1) + 1], s);
        // the update also scores the new pose on the next iteration's view (its slot 0); the last
        // iteration only completes (E*, s), its particles stay in `poses` / `fit`
        const bool more = i < p->n_iters;
        const int rn = more ? i % p->n_rates : densest;
        const bool second = more || final_in_loop;
        const int G = second ? (Gv[r] > Gv[rn] ? Gv[r] : Gv[rn]) : Gv[r];
        const NextView nvn = second ? NextView{views[rn].x, views[rn].y, views[rn].z, views[rn].n_dev}
                                    : NextView{nullptr, nullptr, nullptr, nullptr};
        if ((rc = launch_adv(true, vv, S, G, fit, st, p->K, s, nvn))) return rc;
        // (the next iteration's particle launch completes this one itself when it draws)
        if (!(more && fused[i + 1]) &&
            (rc = launch_next(vv.format, false, st, p->K, G, more, poses, recs, s, second ? G : 0,
                              more ? fit : ef_dev, more ? nv : nvf_dev)))
            return rc;
        G_prev = G;
    }
    // optional gradient polish of the best candidate, on the densest view
    if (p->polish_steps > 0 &&
        (rc = launch_polish(vv, views[densest], Gv[densest], st, p->K, fit, p->compose_mode, v->voxel_size,
                            p->polish_steps, ws + L.polish, s)))
        return rc;
    // fitness of the returned pose on the densest view
    if (!final_in_loop &&
        (rc = launch_state_fitness(vv, views[densest], Gv[densest], st, ws + L.fin, ef_dev, nvf_dev, s)))
        return rc;

    Readback* rb = reinterpret_cast<Readback*>(ws + L.rb);
    hipLaunchKernelGGL(k_readback, dim3(1), dim3(256), 0, s, st, recs, ef_dev, nvf_dev, vcount,
                       p->polish_steps > 0 ? reinterpret_cast<const int*>(ws + L.polish + polish_accepted_offset())
                                           : nullptr,
                       rb);
    if ((rc = check_launch("track_frame read-back"))) return rc;
    // Fusing a dense volume: the fusion at the tracked pose (read by the device from the state) is
    // enqueued right after the read-back copy, and the host waits for the copy only, so the GPU
    // fuses while the host reads the result (a sparse volume is fused from the host afterwards).
    Readback local;
    Readback* hp = &local;
    hipEvent_t ev = nullptr;
    const bool fuse_here = fuse && v->layout != PF_LAYOUT_BRICKS;
    if (fuse && (rc = fuse_readback(&hp, &ev))) return rc;
    if (hipMemcpyAsync(hp, rb, sizeof(Readback), hipMemcpyDeviceToHost, s) != hipSuccess)
        return set_error(PF_EHIP, "track_frame: read-back failed: %s", hipGetErrorString(hipGetLastError()));
    hipError_t e;
    if (fuse_here) {
        if (hipEventRecord(ev, s) != hipSuccess)
            return set_error(PF_EHIP, "track_frame_fuse: %s", hipGetErrorString(hipGetLastError()));
        if ((rc = launch_tsdf_integrate_at(v, depth, K, st->R, st->t, ws + L.fuse, s))) return rc;
        e = hipEventSynchronize(ev);
    } else {
        e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return set_error(PF_EHIP, "track_frame: %s", hipGetErrorString(e));
    const Readback hrb = *hp;
    const pf_track_state& hs = hrb.st;
    const IterRec* hr = hrb.recs;
    const float ef = hrb.ef;
    const int nvf = hrb.nvf, nall = hrb.nall, accepted = hrb.accepted;
    if (hs.flags) return set_error(PF_EINVAL, "track_frame: inconsistent optimizer state (flags %d)", hs.flags);
    // iterations that ran (all n_iters unless the stop rule ended the optimization)
    const int n_run = hs.iter_done;
    g_forecast.valid = true;
    g_forecast.K = p->K;
    g_forecast.n_iters = p->n_iters;
    g_forecast.n_rates = p->n_rates;
    g_forecast.alt_K = p->alt_K;
    for (int r = 0; r < 3; ++r) {
        g_forecast.rates[r] = p->rates[r];
        g_forecast.Ks[r] = p->Ks[r];
    }
    g_forecast.inv_vs = vv.inv_vs;
    // iterations after an early exit take the last regime that ran (their launches return at once
    // while the optimization stays stopped)
    int last = -1;
    for (int i = 0; i < PF_MAX_ITERS; ++i) {
        if (i < n_run && i < p->n_iters) last = spread_regime_of(hr[i].s_rad, hr[i].s_m, vv.inv_vs);
        g_forecast.regime[i] = last;
    }
    if (timed) {
        for (int i = 0; i < n_run; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, g_timing.ev[2 * i], g_timing.ev[2 * i + 1]) == hipSuccess) g_timing.ms += ms;
            g_timing.launches += 1;
            g_timing.evals += (int64_t)hr[i].n_particles * hr[i].n_sub;
        }
    }
    for (int q = 0; q < 9; ++q) out->R[q] = hs.R[q];
    for (int q = 0; q < 3; ++q) out->t[q] = hs.t[q];
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->n_points = nall;
        stats->n_iters = n_run;
        for (int i = 0; i < n_run; ++i) {
            stats->E0[i] = hr[i].E0;
            stats->Estar[i] = hr[i].Estar;
            stats->n_adv[i] = hr[i].n_adv;
            stats->n_sub[i] = hr[i].n_sub;
            stats->n_valid[i] = hr[i].n_valid;
            stats->s_rad[i] = hr[i].s_rad;
            stats->s_m[i] = hr[i].s_m;
            stats->n_particles[i] = hr[i].n_particles;
        }
        stats->E_final = ef;
        stats->polish_accepted = accepted;
        stats->n_valid_final = nvf;
        stats->lost = nvf < p->min_valid ? 1 : 0;
    }
    if (fuse && !fuse_here) return launch_tsdf_integrate(v, depth, K, out, s);
    return PF_OK;
}

}  // namespace pf
