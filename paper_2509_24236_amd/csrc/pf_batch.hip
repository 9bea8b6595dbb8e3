// Batched tracking of many independent problems (frames or sequences with their own volumes,
// resolutions and particle counts). Every step of the frame optimization, and of the gradient
// polish, is one launch over all problems; the scoring launch is persistent (a fixed grid strides
// over the list of (problem, pose group) items, longest problems first). The step bodies are the
// same device functions the single-problem kernels run, so each problem reproduces track_frame
// bit for bit. The host
// record holds the grid sizes, which makes track_batch_run a fixed kernel sequence: no host
// synchronisation, copy or allocation, and therefore capturable into a HIP graph.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <type_traits>
#include <vector>

#include "pf_polish.hpp"
#include "pf_steps.hpp"

namespace pf {

size_t state_bytes(int K);
pf_track_state initial_state(const pf_pose* init, const pf_track_params* p);
int32_t check_problem(const pf_batch_problem& q, int idx);

struct BatchProb {
    VolView vv;
    BpArgs bp;
    int bp_blocks;
    int K;
    float* px;
    float* py;
    float* pz;
    int* counts;
    int* ncount;            // [0] = |M|, [1 + r] = |S_r|
    int* pix;               // pixel index of every point of M
    ViewTiles tiles[3];
    float* vx[3];
    float* vy[3];
    float* vz[3];
    int caps[3];
    int rates[3];
    int G[3];               // E* partial workgroups per rate
    int densest;
    float* poses;
    float* fit;
    int* nv;
    pf_track_state* st;
    IterRec* recs;
    float* efin;
    int* nfin;
    // gradient polish (polish_steps > 0): state, gradient partials [S], candidate partials [6][S]
    PolishState* ps;
    GradPartial* gp;
    Partial2* cp;
    double vs;
    int mode;
};

namespace {

__device__ inline void view_of(const BatchProb& P, int r, const float*& x, const float*& y, const float*& z,
                               const int*& nd) {
    if (P.rates[r] == 1) {
        x = P.px;
        y = P.py;
        z = P.pz;
        nd = P.ncount;
    } else {
        x = P.vx[r];
        y = P.vy[r];
        z = P.vz[r];
        nd = P.ncount + 1 + r;
    }
}

__global__ __launch_bounds__(kBpThreads) void kb_bp_count(const BatchProb* tab, const int4* items) {
    const int4 w = items[blockIdx.x];
    bp_count_step(tab[w.x].bp, tab[w.x].counts, w.y);
}

__global__ __launch_bounds__(kBpThreads) void kb_bp_scatter(const BatchProb* tab, const int4* items) {
    const int4 w = items[blockIdx.x];
    const BatchProb& P = tab[w.x];
    bp_scatter_step(P.bp, P.counts, P.bp_blocks, P.px, P.py, P.pz, P.ncount, w.y);
}

__global__ __launch_bounds__(256) void kb_view_mark(const BatchProb* tab, const int4* items) {
    const int4 w = items[blockIdx.x];
    const BatchProb& P = tab[w.x];
    view_mark_step(P.pix, P.ncount, P.rates[w.y], P.bp.width, P.tiles[w.y], w.z);
}

// one workgroup per (problem, view); views with rate 1 have no tiles
__global__ __launch_bounds__(256) void kb_view_scan(const BatchProb* tab) {
    const BatchProb& P = tab[blockIdx.x / 3];
    const int r = blockIdx.x % 3;
    if (P.tiles[r].n_tiles > 0) view_scan_step(P.tiles[r]);
}

__global__ __launch_bounds__(256) void kb_view_scatter(const BatchProb* tab, const int4* items) {
    const int4 w = items[blockIdx.x];
    const BatchProb& P = tab[w.x];
    const int r = w.y;
    view_scatter_step(P.px, P.py, P.pz, P.pix, P.ncount, P.rates[r], P.bp.width, P.tiles[r], P.vx[r], P.vy[r],
                      P.vz[r], P.ncount + 1 + r, w.z);
}

__global__ void kb_state_set(const BatchProb* tab, const pf_track_state* init, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) *tab[p].st = init[p];
}

template <int FMT, bool FIRST>
__global__ __launch_bounds__(256) void kb_next(const BatchProb* tab, const int4* items, int phase, int draw) {
    const int4 w = items[blockIdx.x];
    const BatchProb& P = tab[w.x];
    next_step<FMT, FIRST>(P.st, P.K, P.G[phase], draw, P.poses, P.recs, w.y);
}

// Persistent over the (problem, pose group) items. Only the items of problems whose particles are
// in one of the spread regimes `regimes` (bit r for regime r) are scored; the others are skipped at
// the cost of one state read. PATH 0: a problem in a regime of kMaskRegimes reads its cells
// through the mask, the others take the per-lane path, in one kernel; PATH 1 / 2: the masked
// (compacting) path or the per-lane path only, each a kernel with its own register and LDS
// footprint (the automatic plan launches the two, one per regime, as track_frame does). NARROW: every
// problem's volume passes narrow_grid (score_step). The batched kernels leave the scoring paths'
// raised-priority windows off (PRIO = false here and in the update and polish steps): with waves of
// several problems on every CU, a raised wave delays other problems' work instead of its own
// arithmetic, and a 64-problem batch ran 4% slower with them.
template <int FMT, int LAYOUT, int TK, int BLOCK, int PATH = 0, bool NARROW = false>
__global__ __launch_bounds__(BLOCK) void kb_score(const BatchProb* tab, const int4* items, int n_items, int phase,
                                                  int regimes) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int4 w = items[it];
        const BatchProb& P = tab[w.x];
        const int regime = spread_regime(P.st, P.vv.inv_vs);
        if (!((regimes >> regime) & 1)) continue;
        const float *x, *y, *z;
        const int* nd;
        view_of(P, phase, x, y, z, nd);
        if constexpr (PATH == 0)
            score_step_regime<FMT, LAYOUT, TK, BLOCK, false>(P.vv, x, y, z, *nd, P.poses, P.K + 1, w.y * TK, P.fit, P.nv,
                                                      regime);
        else
            score_step<FMT, LAYOUT, TK, BLOCK, PATH == 1 && LAYOUT != PF_LAYOUT_LINEAR, NARROW, false>(
                P.vv, x, y, z, *nd, P.poses, P.K + 1, w.y * TK, P.fit, P.nv);
    }
}

template <int FMT, int LAYOUT, bool ADV>
__global__ __launch_bounds__(256) void kb_adv(const BatchProb* tab, const int4* items, int phase) {
    const int4 w = items[blockIdx.x];
    const BatchProb& P = tab[w.x];
    const float *x, *y, *z;
    const int* nd;
    view_of(P, ADV ? phase : P.densest, x, y, z, nd);
    adv_step<FMT, LAYOUT, ADV, false>(P.vv, x, y, z, 0, nd, P.fit, P.st, P.K, w.y, w.z);
}

template <int FMT>
__global__ void kb_final(const BatchProb* tab, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const BatchProb& P = tab[p];
    const Partial* pt = state_partials(P.st, P.K);
    FixSum sum = 0;
    int cnt = 0;
    for (int b = 0; b < P.G[P.densest]; ++b) {
        sum += pt[b].sum;
        cnt += pt[b].cnt;
    }
    *P.efin = fitness_from<FMT>(sum, cnt);
    *P.nfin = cnt;
}

// ---- gradient polish of every problem's best candidate (track_frame's launch_polish, batched)
__global__ __launch_bounds__(256) void kb_best(const BatchProb* tab) {
    const BatchProb& P = tab[blockIdx.x];
    best_step(P.st, P.fit, P.ps);
}

template <int FMT, int LAYOUT>
__global__ __launch_bounds__(kGradThreads) void kb_grad(const BatchProb* tab, const int4* items) {
    const int4 w = items[blockIdx.x];
    const BatchProb& P = tab[w.x];
    if (P.ps->stop) return;   // a stopped polish ignores the gradient
    const float *x, *y, *z;
    const int* nd;
    view_of(P, P.densest, x, y, z, nd);
    grad_step<FMT, LAYOUT>(P.vv, x, y, z, *nd, P.ps->P, nullptr, P.mode, nullptr, nullptr, nullptr, P.gp, 0,
                           P.G[P.densest], w.y);
}

template <int FMT>
__global__ void kb_polish_prep(const BatchProb* tab) {
    const BatchProb& P = tab[blockIdx.x];
    polish_prep_step<FMT>(P.ps, P.gp, P.G[P.densest], P.mode, P.vs);
}

template <int FMT, int LAYOUT>
__global__ __launch_bounds__(kGradThreads) void kb_pose_partials(const BatchProb* tab, const int4* items) {
    const int4 w = items[blockIdx.x];
    const BatchProb& P = tab[w.x];
    if (P.ps->stop) return;
    const float *x, *y, *z;
    const int* nd;
    view_of(P, P.densest, x, y, z, nd);
    pose_partials_step<FMT, LAYOUT, false>(P.vv, x, y, z, *nd, &P.ps->cand[0][0], P.cp, w.y, P.G[P.densest], w.z);
}

template <int FMT>
__global__ void kb_polish_pick(const BatchProb* tab) {
    const BatchProb& P = tab[blockIdx.x];
    polish_pick_step<FMT>(P.ps, P.cp, P.G[P.densest]);
}

__global__ void kb_polish_commit(const BatchProb* tab) {
    const BatchProb& P = tab[blockIdx.x];
    polish_commit_step(P.ps, P.st);
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

int rate_or_1(const pf_track_params& p, int r) { return r < p.n_rates ? p.rates[r] : 1; }

struct ProbLayout {
    size_t pts, pix, counts, ncount, views[3], tiles_mask[3], tiles_start[3], n_tiles[3], poses, fit, nv, state, recs,
        fin, polish, end;
};

ProbLayout prob_layout(const pf_batch_problem& q, size_t off) {
    ProbLayout L;
    const size_t npix = (size_t)q.K.width * q.K.height;
    const pf_track_params& p = q.params;
    L.pts = off;
    off += al(3 * npix * sizeof(float));
    L.pix = off;
    off += al(npix * sizeof(int));
    L.counts = off;
    off += al(((npix + kBpChunk - 1) / kBpChunk + 1) * sizeof(int));
    L.ncount = off;
    off += al(8 * sizeof(int));
    for (int r = 0; r < 3; ++r) {
        L.views[r] = off;
        L.n_tiles[r] = 0;
        if (r < p.n_rates && p.rates[r] > 1) {
            off += al(3 * ((npix + p.rates[r] - 1) / p.rates[r]) * sizeof(float));
            L.n_tiles[r] = (size_t)view_n_tiles(q.K.width, q.K.height, p.rates[r]);
        }
    }
    // the tile masks back to back, cleared as one range by the count step
    for (int r = 0; r < 3; ++r) {
        L.tiles_mask[r] = off;
        off += L.n_tiles[r] * sizeof(unsigned long long);
    }
    off = al(off);
    for (int r = 0; r < 3; ++r) {
        L.tiles_start[r] = off;
        off += L.n_tiles[r] * sizeof(int);
    }
    off = al(off);
    L.poses = off;
    off += al((size_t)(p.K + 1) * 12 * sizeof(float));
    L.fit = off;
    off += al((size_t)(p.K + 1) * sizeof(float));
    L.nv = off;
    off += al((size_t)(p.K + 1) * sizeof(int));
    L.state = off;
    off += al(state_bytes(p.K));
    L.recs = off;
    off += al(PF_MAX_ITERS * sizeof(IterRec));
    L.fin = off;
    off += al(2 * sizeof(int));
    L.polish = off;
    if (p.polish_steps > 0) {
        int rmin = p.rates[0];
        for (int r = 1; r < p.n_rates; ++r) rmin = p.rates[r] < rmin ? p.rates[r] : rmin;
        off += al(polish_scratch_bytes(n_partials_for((int)((npix + rmin - 1) / rmin))));
    }
    L.end = off;
    return L;
}

}  // namespace
}  // namespace pf

using namespace pf;

struct pf_batch {
    int n = 0, n_iters = 0, n_rates = 0, format = 0, layout = 0, polish_steps = 0;
    pf_batch_plan plan{};
    char* ws = nullptr;
    BatchProb* tab = nullptr;
    pf_track_state* init = nullptr;
    int4* items = nullptr;                  // all lists, back to back
    size_t off_bp = 0, off_view = 0, off_next = 0, off_score = 0, off_fin = 0, off_adv[3] = {0, 0, 0};
    size_t off_grad = 0, off_pp = 0;
    int n_bp = 0, n_view = 0, n_next = 0, n_score = 0, n_fin = 0, n_adv[3] = {0, 0, 0}, n_grad = 0,
        n_pp = 0;
    std::vector<BatchProb> host;
    std::vector<int> min_valid;
    bool narrow = false;   // every problem's volume passes narrow_grid
};

namespace {

size_t table_bytes(int n) { return al(sizeof(BatchProb) * n) + al(sizeof(pf_track_state) * n); }

template <int FMT, int LAYOUT, int TK>
void launch_score_batch(pf_batch* b, int phase, hipStream_t s) {
    const int grid = std::min(b->plan.score_grid, b->n_score);
    hipLaunchKernelGGL((kb_score<FMT, LAYOUT, TK, 256>), dim3(grid), dim3(256), 0, s, b->tab,
                       b->items + b->off_score, b->n_score, phase, (1 << kRegimes) - 1);
}

// The automatic plan: track_frame's launches, 4 poses x 256 threads, one kernel per spread regime
// (the masked, compacting one for the problems still spread, the per-lane one for the others), each
// persistent over the item list.
template <int FMT, int LAYOUT>
void launch_score_batch_auto(pf_batch* b, int phase, hipStream_t s) {
    const int g = std::min(b->plan.score_grid, b->n_score);
    auto go = [&](auto narrow) {
        constexpr bool N = decltype(narrow)::value;
        hipLaunchKernelGGL((kb_score<FMT, LAYOUT, 4, 256, 1, N>), dim3(g), dim3(256), 0, s, b->tab,
                           b->items + b->off_score, b->n_score, phase, kMaskRegimes);
        hipLaunchKernelGGL((kb_score<FMT, LAYOUT, 4, 256, 2, N>), dim3(g), dim3(256), 0, s, b->tab,
                           b->items + b->off_score, b->n_score, phase, ((1 << kRegimes) - 1) & ~kMaskRegimes);
    };
    if (b->narrow)
        go(std::true_type{});
    else
        go(std::false_type{});
}

template <int FMT, int LAYOUT>
int32_t run_t(pf_batch* b, hipStream_t s) {
    hipLaunchKernelGGL(kb_bp_count, dim3(b->n_bp), dim3(kBpThreads), 0, s, b->tab, b->items + b->off_bp);
    hipLaunchKernelGGL(kb_bp_scatter, dim3(b->n_bp), dim3(kBpThreads), 0, s, b->tab, b->items + b->off_bp);
    if (b->n_view) {
        hipLaunchKernelGGL(kb_view_mark, dim3(b->n_view), dim3(256), 0, s, b->tab, b->items + b->off_view);
        hipLaunchKernelGGL(kb_view_scan, dim3(3 * b->n), dim3(256), 0, s, b->tab);
        hipLaunchKernelGGL(kb_view_scatter, dim3(b->n_view), dim3(256), 0, s, b->tab, b->items + b->off_view);
    }
    hipLaunchKernelGGL(kb_state_set, dim3((b->n + 63) / 64), dim3(64), 0, s, b->tab, b->init, b->n);
    hipLaunchKernelGGL((kb_next<FMT, true>), dim3(b->n_next), dim3(256), 0, s, b->tab, b->items + b->off_next, 0, 1);
    for (int i = 1; i <= b->n_iters; ++i) {
        const int ph = (i - 1) % b->n_rates;
        switch (b->plan.score_tk) {
            case 0: launch_score_batch_auto<FMT, LAYOUT>(b, ph, s); break;
            case 1: launch_score_batch<FMT, LAYOUT, 1>(b, ph, s); break;
            case 2: launch_score_batch<FMT, LAYOUT, 2>(b, ph, s); break;
            case 8: launch_score_batch<FMT, LAYOUT, 8>(b, ph, s); break;
            default: launch_score_batch<FMT, LAYOUT, 4>(b, ph, s); break;
        }
        hipLaunchKernelGGL((kb_adv<FMT, LAYOUT, true>), dim3(b->n_adv[ph]), dim3(256), 0, s, b->tab,
                           b->items + b->off_adv[ph], ph);
        hipLaunchKernelGGL((kb_next<FMT, false>), dim3(b->n_next), dim3(256), 0, s, b->tab, b->items + b->off_next,
                           ph, i < b->n_iters ? 1 : 0);
    }
    if (b->polish_steps > 0) {
        hipLaunchKernelGGL(kb_best, dim3(b->n), dim3(256), 0, s, b->tab);
        for (int it = 0; it < b->polish_steps; ++it) {
            hipLaunchKernelGGL((kb_grad<FMT, LAYOUT>), dim3(b->n_grad), dim3(kGradThreads), 0, s, b->tab,
                               b->items + b->off_grad);
            hipLaunchKernelGGL(kb_polish_prep<FMT>, dim3(b->n), dim3(1), 0, s, b->tab);
            hipLaunchKernelGGL((kb_pose_partials<FMT, LAYOUT>), dim3(b->n_pp), dim3(kGradThreads), 0, s, b->tab,
                               b->items + b->off_pp);
            hipLaunchKernelGGL(kb_polish_pick<FMT>, dim3(b->n), dim3(1), 0, s, b->tab);
        }
        hipLaunchKernelGGL(kb_polish_commit, dim3(b->n), dim3(1), 0, s, b->tab);
    }
    hipLaunchKernelGGL((kb_adv<FMT, LAYOUT, false>), dim3(b->n_fin), dim3(256), 0, s, b->tab, b->items + b->off_fin,
                       0);
    hipLaunchKernelGGL(kb_final<FMT>, dim3((b->n + 63) / 64), dim3(64), 0, s, b->tab, b->n);
    return check_launch("track_batch_run");
}

}  // namespace

extern "C" {

size_t track_batch_workspace_bytes(const pf_batch_problem* problems, int32_t n) {
    if (!problems || n < 1) return 0;
    size_t off = table_bytes(n);
    for (int p = 0; p < n; ++p) {
        if (check_problem(problems[p], p)) return 0;
        off = prob_layout(problems[p], off).end;
    }
    size_t items = 0;
    for (int p = 0; p < n; ++p) {
        const pf_batch_problem& q = problems[p];
        const size_t npix = (size_t)q.K.width * q.K.height;
        items += 2 * ((npix + kBpChunk - 1) / kBpChunk);
        for (int r = 0; r < q.params.n_rates; ++r)
            items += (npix / q.params.rates[r] + 256) / 256 + (size_t)kMaxPartials;
        items += 2 * ((size_t)q.params.K + 256) / 256 + (size_t)q.params.K + 1 + kMaxPartials;
        items += 7 * (size_t)kMaxPartials;   // polish: gradient and candidate chunks
    }
    return off + al(items * sizeof(int4));
}

pf_batch* track_batch_create(const pf_batch_problem* problems, int32_t n, const pf_batch_plan* plan, void* workspace,
                             size_t ws_bytes, void* stream) {
    if (!problems || n < 1 || !plan || !workspace) {
        set_error(PF_EINVAL, "track_batch_create: null argument or n < 1");
        return nullptr;
    }
    if (plan->score_tk != 0 && plan->score_tk != 1 && plan->score_tk != 2 && plan->score_tk != 4 &&
        plan->score_tk != 8) {
        set_error(PF_EINVAL, "track_batch_create: score_tk %d not in {0, 1, 2, 4, 8}", plan->score_tk);
        return nullptr;
    }
    if (plan->score_grid < 1 || plan->reserved != 0 || (plan->order != 0 && plan->order != 1)) {
        set_error(PF_EINVAL, "track_batch_create: bad plan (grid %d, order %d)", plan->score_grid, plan->order);
        return nullptr;
    }
    for (int p = 0; p < n; ++p)
        if (check_problem(problems[p], p)) return nullptr;
    const pf_batch_problem& q0 = problems[0];
    for (int p = 1; p < n; ++p) {
        const pf_batch_problem& q = problems[p];
        if (q.params.n_iters != q0.params.n_iters || q.params.n_rates != q0.params.n_rates ||
            q.params.polish_steps != q0.params.polish_steps || q.vol.format != q0.vol.format ||
            q.vol.layout != q0.vol.layout) {
            set_error(PF_EINVAL, "track_batch_create: problem %d differs from problem 0 in n_iters, n_rates, "
                                 "polish_steps, format or layout", p);
            return nullptr;
        }
    }
    const size_t need = track_batch_workspace_bytes(problems, n);
    if (ws_bytes < need) {
        set_error(PF_ENOMEM, "track_batch_create: workspace of %zu bytes, %zu needed", ws_bytes, need);
        return nullptr;
    }
    pf_batch* b = new (std::nothrow) pf_batch();
    if (!b) {
        set_error(PF_ENOMEM, "track_batch_create: host allocation failed");
        return nullptr;
    }
    b->n = n;
    b->n_iters = q0.params.n_iters;
    b->n_rates = q0.params.n_rates;
    b->format = q0.vol.format;
    b->layout = q0.vol.layout;
    b->polish_steps = q0.params.polish_steps;
    b->plan = *plan;
    b->ws = static_cast<char*>(workspace);
    b->tab = reinterpret_cast<BatchProb*>(b->ws);
    b->init = reinterpret_cast<pf_track_state*>(b->ws + al(sizeof(BatchProb) * n));
    std::vector<pf_track_state> init(n);
    size_t off = table_bytes(n);
    b->host.resize(n);
    b->narrow = true;
    for (int p = 0; p < n; ++p) {
        const pf_batch_problem& q = problems[p];
        const ProbLayout L = prob_layout(q, off);
        off = L.end;
        BatchProb& P = b->host[p];
        memset(&P, 0, sizeof P);
        P.vv = make_view(&q.vol);
        b->narrow = b->narrow && narrow_grid(P.vv);
        const size_t npix = (size_t)q.K.width * q.K.height;
        P.bp.depth = q.depth;
        P.bp.width = q.K.width;
        P.bp.height = q.K.height;
        P.bp.stride = q.params.pixel_stride;
        P.bp.fx = (float)q.K.fx;
        P.bp.fy = (float)q.K.fy;
        P.bp.cx = (float)q.K.cx;
        P.bp.cy = (float)q.K.cy;
        P.bp_blocks = (int)((npix + kBpChunk - 1) / kBpChunk);
        P.bp.nblocks = P.bp_blocks;
        P.pix = reinterpret_cast<int*>(b->ws + L.pix);
        P.bp.pix = P.pix;
        P.bp.masks = reinterpret_cast<unsigned long long*>(b->ws + L.tiles_mask[0]);
        P.bp.n_masks = (int)(L.n_tiles[0] + L.n_tiles[1] + L.n_tiles[2]);
        for (int r = 0; r < 3; ++r)
            P.tiles[r] = ViewTiles{reinterpret_cast<unsigned long long*>(b->ws + L.tiles_mask[r]),
                                   reinterpret_cast<int*>(b->ws + L.tiles_start[r]),
                                   view_tiles_x(q.K.width, rate_or_1(q.params, r)), (int)L.n_tiles[r]};
        P.K = q.params.K;
        P.px = reinterpret_cast<float*>(b->ws + L.pts);
        P.py = P.px + npix;
        P.pz = P.py + npix;
        P.counts = reinterpret_cast<int*>(b->ws + L.counts);
        P.ncount = reinterpret_cast<int*>(b->ws + L.ncount);
        P.densest = 0;
        for (int r = 0; r < 3; ++r) {
            const int rate = r < q.params.n_rates ? q.params.rates[r] : 1;
            P.rates[r] = rate;
            P.caps[r] = (int)((npix + rate - 1) / rate);
            P.G[r] = n_partials_for(P.caps[r]);
            P.vx[r] = reinterpret_cast<float*>(b->ws + L.views[r]);
            P.vy[r] = P.vx[r] + P.caps[r];
            P.vz[r] = P.vy[r] + P.caps[r];
            if (r < q.params.n_rates && rate < P.rates[P.densest]) P.densest = r;
        }
        P.poses = reinterpret_cast<float*>(b->ws + L.poses);
        P.fit = reinterpret_cast<float*>(b->ws + L.fit);
        P.nv = reinterpret_cast<int*>(b->ws + L.nv);
        P.st = reinterpret_cast<pf_track_state*>(b->ws + L.state);
        P.recs = reinterpret_cast<IterRec*>(b->ws + L.recs);
        P.efin = reinterpret_cast<float*>(b->ws + L.fin);
        P.nfin = reinterpret_cast<int*>(b->ws + L.fin + sizeof(float));
        P.vs = q.vol.voxel_size;
        P.mode = q.params.compose_mode;
        if (q.params.polish_steps > 0) {
            // the same scratch layout as track_frame's polish
            char* pb = b->ws + L.polish;
            P.ps = reinterpret_cast<PolishState*>(pb);
            P.gp = reinterpret_cast<GradPartial*>(pb + al(sizeof(PolishState)));
            P.cp = reinterpret_cast<Partial2*>(reinterpret_cast<char*>(P.gp) + al(P.G[P.densest] * sizeof(GradPartial)));
        }
        init[p] = initial_state(&q.init, &q.params);
        b->min_valid.push_back(q.params.min_valid);
    }
    // item lists
    std::vector<int> order(n);
    for (int p = 0; p < n; ++p) order[p] = p;
    if (plan->order == 1)
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
            const size_t na = (size_t)problems[a].K.width * problems[a].K.height * (problems[a].params.K + 1);
            const size_t nc = (size_t)problems[c].K.width * problems[c].K.height * (problems[c].params.K + 1);
            return na > nc;
        });
    std::vector<int4> items;
    auto mark = [&](size_t& o) { o = items.size(); };
    mark(b->off_bp);
    for (int p = 0; p < n; ++p)
        for (int k = 0; k < b->host[p].bp_blocks; ++k) items.push_back(make_int4(p, k, 0, 0));
    b->n_bp = (int)(items.size() - b->off_bp);
    mark(b->off_view);
    for (int p = 0; p < n; ++p)
        for (int r = 0; r < b->n_rates; ++r)
            if (b->host[p].rates[r] > 1)
                for (int k = 0; k < (b->host[p].caps[r] + 255) / 256; ++k) items.push_back(make_int4(p, r, k, 0));
    b->n_view = (int)(items.size() - b->off_view);
    mark(b->off_next);
    for (int p = 0; p < n; ++p)
        for (int k = 0; k < (b->host[p].K + 1 + 255) / 256; ++k) items.push_back(make_int4(p, k, 0, 0));
    b->n_next = (int)(items.size() - b->off_next);
    mark(b->off_score);
    const int tk = plan->score_tk == 0 ? 4 : plan->score_tk;
    for (int p : order)
        for (int g = 0; g < (b->host[p].K + 1 + tk - 1) / tk; ++g) items.push_back(make_int4(p, g, 0, 0));
    b->n_score = (int)(items.size() - b->off_score);
    for (int ph = 0; ph < b->n_rates; ++ph) {
        mark(b->off_adv[ph]);
        for (int p = 0; p < n; ++p)
            for (int k = 0; k < b->host[p].G[ph]; ++k) items.push_back(make_int4(p, k, b->host[p].G[ph], 0));
        b->n_adv[ph] = (int)(items.size() - b->off_adv[ph]);
    }
    mark(b->off_fin);
    for (int p = 0; p < n; ++p) {
        const int G = b->host[p].G[b->host[p].densest];
        for (int k = 0; k < G; ++k) items.push_back(make_int4(p, k, G, 0));
    }
    b->n_fin = (int)(items.size() - b->off_fin);
    if (b->polish_steps > 0) {
        mark(b->off_grad);
        for (int p = 0; p < n; ++p)
            for (int k = 0; k < b->host[p].G[b->host[p].densest]; ++k) items.push_back(make_int4(p, k, 0, 0));
        b->n_grad = (int)(items.size() - b->off_grad);
        mark(b->off_pp);
        for (int p = 0; p < n; ++p)
            for (int h = 0; h < 6; ++h)
                for (int k = 0; k < b->host[p].G[b->host[p].densest]; ++k) items.push_back(make_int4(p, h, k, 0));
        b->n_pp = (int)(items.size() - b->off_pp);
    }
    b->items = reinterpret_cast<int4*>(b->ws + off);
    if (off + items.size() * sizeof(int4) > ws_bytes) {
        delete b;
        set_error(PF_ENOMEM, "track_batch_create: item lists exceed the workspace");
        return nullptr;
    }
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(b->tab, b->host.data(), sizeof(BatchProb) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->init, init.data(), sizeof(pf_track_state) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        delete b;
        set_error(PF_EHIP, "track_batch_create: upload failed: %s", hipGetErrorString(hipGetLastError()));
        return nullptr;
    }
    return b;
}

int32_t track_batch_run(pf_batch* b, void* stream) {
    if (!b) return set_error(PF_EINVAL, "track_batch_run: null batch");
    hipStream_t s = (hipStream_t)stream;
    return with_volume(b->format, b->layout, [&](auto fmt, auto layout) {
        return run_t<decltype(fmt)::value, decltype(layout)::value>(b, s);
    });
}

int32_t track_batch_results(pf_batch* b, pf_pose* out, pf_track_stats* stats, void* stream) {
    if (!b || !out) return set_error(PF_EINVAL, "track_batch_results: null argument");
    hipStream_t s = (hipStream_t)stream;
    const int n = b->n;
    std::vector<pf_track_state> st(n);
    std::vector<IterRec> recs((size_t)n * PF_MAX_ITERS);
    std::vector<float> ef(n);
    std::vector<int> nf(n), na(n), acc(n, 0);
    for (int p = 0; p < n; ++p) {
        const BatchProb& P = b->host[p];
        if (b->polish_steps > 0 &&
            hipMemcpyAsync(&acc[p], reinterpret_cast<char*>(P.ps) + offsetof(PolishState, accepted), sizeof(int),
                           hipMemcpyDeviceToHost, s) != hipSuccess)
            return set_error(PF_EHIP, "track_batch_results: read-back failed");
        if (hipMemcpyAsync(&st[p], P.st, sizeof(pf_track_state), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&recs[(size_t)p * PF_MAX_ITERS], P.recs, sizeof(IterRec) * b->n_iters, hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipMemcpyAsync(&ef[p], P.efin, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&nf[p], P.nfin, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&na[p], P.ncount, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
            return set_error(PF_EHIP, "track_batch_results: read-back failed");
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(PF_EHIP, "track_batch_results: %s", hipGetErrorString(e));
    for (int p = 0; p < n; ++p) {
        if (st[p].flags) return set_error(PF_EINVAL, "track_batch_results: problem %d state flags %d", p, st[p].flags);
        for (int q = 0; q < 9; ++q) out[p].R[q] = st[p].R[q];
        for (int q = 0; q < 3; ++q) out[p].t[q] = st[p].t[q];
        if (stats) {
            pf_track_stats& S = stats[p];
            memset(&S, 0, sizeof S);
            S.n_points = na[p];
            S.n_iters = b->n_iters;
            for (int i = 0; i < b->n_iters; ++i) {
                const IterRec& r = recs[(size_t)p * PF_MAX_ITERS + i];
                S.E0[i] = r.E0;
                S.Estar[i] = r.Estar;
                S.n_adv[i] = r.n_adv;
                S.n_sub[i] = r.n_sub;
                S.n_valid[i] = r.n_valid;
                S.s_rad[i] = r.s_rad;
                S.s_m[i] = r.s_m;
            }
            S.E_final = ef[p];
            S.n_valid_final = nf[p];
            S.polish_accepted = acc[p];
            S.lost = nf[p] < b->min_valid[p] ? 1 : 0;
        }
    }
    return PF_OK;
}

void track_batch_destroy(pf_batch* b) { delete b; }

}  // extern "C"
