// C ABI of the library (include/profusion.h): argument validation before any launch, error
// codes and thread-local messages, and dispatch to the launchers. No entry point allocates or
// frees device memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "pf_internal.hpp"

namespace pf {

size_t state_bytes(int K);
int32_t state_init(void* state, const pf_pose* init, const pf_track_params* p, int format, float* next_poses,
                   hipStream_t s);
int32_t update(const VolView& vv, const Points& pts, const float* fitness, void* state, int K, float* next_poses,
               hipStream_t s);
size_t workspace_bytes(const pf_intrinsics* K, const pf_track_params* p);
int32_t track(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* init,
              const pf_track_params* p, pf_pose* out, pf_track_stats* stats, void* workspace, size_t ws_bytes,
              hipStream_t s, bool fuse);
int32_t timing_enable(int on);
int32_t score_config(int tk, int block);
int32_t score_mask(int mode);
int32_t timing_read(double* ms, int64_t* launches, int64_t* evals, int reset);

namespace {
thread_local char g_err[512] = "";
}

int32_t set_error(int32_t code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int32_t check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(PF_EHIP, "%s: %s", what, hipGetErrorString(e));
    return PF_OK;
}

size_t t_elem_bytes(int format) { return format == PF_F32_W_F32 ? 4 : 2; }

size_t cells_offset_bytes(const pf_tsdf* v) {
    if (v->layout != PF_LAYOUT_CELLS) return 0;
    const size_t n = (size_t)v->nx * v->ny * v->nz;
    return (n * t_elem_bytes(v->format) + 255) & ~(size_t)255;
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

CellMask cell_mask_layout(const pf_tsdf* v) {
    CellMask M;
    M.mwx = (v->nx - 1 + 3) / 4;
    M.mwy = (v->ny - 1 + 3) / 4;
    M.mwz = (v->nz - 1 + 3) / 4;
    M.words = (size_t)M.mwx * M.mwy * M.mwz;
    const size_t cells = (size_t)(v->nx - 1) * (v->ny - 1) * (v->nz - 1);
    M.mask = al256(cells_offset_bytes(v) + cells * 8 * t_elem_bytes(v->format));
    M.flags = al256(M.mask + M.words * sizeof(unsigned long long));
    M.t_total = al256(M.flags + M.words);
    return M;
}

BrickLayout brick_layout(const pf_tsdf* v) {
    BrickLayout L;
    L.nbx = v->nx / kBrickEdge;
    L.nby = v->ny / kBrickEdge;
    L.nbz = v->nz / kBrickEdge;
    const size_t nb = (size_t)L.nbx * L.nby * L.nbz, slots = (size_t)v->max_bricks, tb = t_elem_bytes(v->format);
    L.index = 256;
    L.cand = L.index + al256(nb * sizeof(int));
    L.coords = L.cand + al256(nb * sizeof(int));
    L.pool_t = L.coords + al256(slots * 4 * sizeof(int));
    L.pool_cells = L.pool_t + al256(slots * kBrickVox * tb);
    L.pool_mask = L.pool_cells + al256(slots * kBrickVox * 8 * tb);
    L.t_total = L.pool_mask + slots * kBrickMaskWords * sizeof(unsigned long long);
    L.w_total = slots * kBrickVox * (v->format == PF_F32_W_F32 ? 4 : 1);
    return L;
}

VolView make_view(const pf_tsdf* v) {
    VolView vv;
    vv.T = v->tsdf;
    vv.bindex = nullptr;
    vv.ones = nullptr;
    vv.nbx = vv.nby = 0;
    vv.cells = v->layout == PF_LAYOUT_CELLS ? static_cast<const char*>(v->tsdf) + cells_offset_bytes(v) : nullptr;
    vv.mask = nullptr;
    vv.mwx = vv.mwy = 0;
    if (v->layout == PF_LAYOUT_CELLS) {
        const CellMask M = cell_mask_layout(v);
        vv.mask = reinterpret_cast<const unsigned long long*>(static_cast<const char*>(v->tsdf) + M.mask);
        vv.mwx = M.mwx;
        vv.mwy = M.mwy;
    }
    if (v->layout == PF_LAYOUT_BRICKS) {
        const BrickLayout L = brick_layout(v);
        const char* base = static_cast<const char*>(v->tsdf);
        vv.T = base + L.pool_t;
        vv.cells = base + L.pool_cells;
        vv.bindex = reinterpret_cast<const int*>(base + L.index);
        vv.ones = base + kBrickOnes;
        vv.mask = reinterpret_cast<const unsigned long long*>(base + L.pool_mask);
        vv.nbx = L.nbx;
        vv.nby = L.nby;
    }
    vv.nx = v->nx;
    vv.ny = v->ny;
    vv.nz = v->nz;
    vv.format = v->format;
    vv.layout = v->layout;
    vv.inv_vs = (float)(1.0 / v->voxel_size);
    vv.gx0 = (float)(-v->origin[0] / v->voxel_size);
    vv.gy0 = (float)(-v->origin[1] / v->voxel_size);
    vv.gz0 = (float)(-v->origin[2] / v->voxel_size);
    return vv;
}

namespace {

int32_t check_tsdf(const pf_tsdf* v, const char* fn, bool need_weight = true) {
    if (!v) return set_error(PF_EINVAL, "%s: null volume", fn);
    if (v->nx < 2 || v->ny < 2 || v->nz < 2)
        return set_error(PF_EINVAL, "%s: volume dims %d x %d x %d (each must be >= 2)", fn, v->nx, v->ny, v->nz);
    if (v->reserved != 0) return set_error(PF_EINVAL, "%s: reserved field must be 0", fn);
    if (v->layout == PF_LAYOUT_BRICKS) {
        if (v->nx % kBrickEdge || v->ny % kBrickEdge || v->nz % kBrickEdge)
            return set_error(PF_EINVAL, "%s: BRICKS needs dims that are multiples of 8", fn);
        if (v->ny / kBrickEdge > 65535 || v->nz / kBrickEdge > 65535)
            return set_error(PF_EINVAL, "%s: ny/8 and nz/8 must be <= 65535", fn);
        if ((int64_t)(v->nx / kBrickEdge) * (v->ny / kBrickEdge) * (v->nz / kBrickEdge) >= ((int64_t)1 << 31))
            return set_error(PF_EINVAL, "%s: brick-index grid exceeds 2^31 - 1 entries", fn);
        if ((int64_t)(v->nx / kBrickEdge) * (v->ny / kBrickEdge) >= ((int64_t)1 << 24))
            return set_error(PF_EINVAL, "%s: (nx/8)(ny/8) must be below 2^24", fn);
        if (v->max_bricks < 1) return set_error(PF_EINVAL, "%s: BRICKS needs max_bricks >= 1", fn);
        if (v->max_bricks > kMaxBricks)
            return set_error(PF_EINVAL, "%s: BRICKS max_bricks %d > %d (a pool cell's index must fit 32 bits)", fn,
                             v->max_bricks, kMaxBricks);
    } else {
        if (v->max_bricks != 0) return set_error(PF_EINVAL, "%s: max_bricks must be 0 for a dense layout", fn);
        if (v->ny > 65535 || v->nz > 65535)
            return set_error(PF_EINVAL, "%s: ny and nz must be <= 65535", fn);
        if ((int64_t)v->nx * v->ny * v->nz >= ((int64_t)1 << 31))
            return set_error(PF_EINVAL, "%s: volume of %lld voxels exceeds 2^31 - 1", fn,
                             (long long)v->nx * v->ny * v->nz);
        if ((int64_t)v->nx * v->ny >= ((int64_t)1 << 24))
            return set_error(PF_EINVAL, "%s: nx * ny must be below 2^24 for a dense layout", fn);
    }
    if (v->format != PF_F32_W_F32 && v->format != PF_F16_W_U8 && v->format != PF_I16_W_U8)
        return set_error(PF_EINVAL, "%s: unknown format %d", fn, v->format);
    if (!(v->voxel_size > 0.0) || !isfinite(v->voxel_size))
        return set_error(PF_EINVAL, "%s: voxel_size must be finite and > 0", fn);
    if (!(v->trunc > 0.0) || !isfinite(v->trunc)) return set_error(PF_EINVAL, "%s: trunc must be finite and > 0", fn);
    for (int a = 0; a < 3; ++a)
        if (!isfinite(v->origin[a])) return set_error(PF_EINVAL, "%s: origin must be finite", fn);
    if (v->w_max < 1 || v->w_max > 255) return set_error(PF_EINVAL, "%s: w_max %d not in 1..255", fn, v->w_max);
    if (v->layout != PF_LAYOUT_LINEAR && v->layout != PF_LAYOUT_CELLS && v->layout != PF_LAYOUT_BRICKS)
        return set_error(PF_EINVAL, "%s: unknown layout %d", fn, v->layout);
    if (!v->tsdf) return set_error(PF_EINVAL, "%s: null tsdf pointer", fn);
    if (need_weight && !v->weight) return set_error(PF_EINVAL, "%s: null weight pointer", fn);
    return PF_OK;
}

int32_t check_pose(const pf_pose* P, const char* fn) {
    if (!P) return set_error(PF_EINVAL, "%s: null pose", fn);
    for (int q = 0; q < 9; ++q)
        if (!isfinite(P->R[q])) return set_error(PF_EINVAL, "%s: non-finite rotation", fn);
    for (int q = 0; q < 3; ++q)
        if (!isfinite(P->t[q])) return set_error(PF_EINVAL, "%s: non-finite translation", fn);
    double worst = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += P->R[a * 3 + c] * P->R[b * 3 + c];
            worst = fmax(worst, fabs(s - (a == b ? 1.0 : 0.0)));
        }
    const double* R = P->R;
    double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) + R[2] * (R[3] * R[7] - R[4] * R[6]);
    if (worst > 1e-9 || det <= 0.0)
        return set_error(PF_EINVAL, "%s: R is not a rotation (|R R^T - I| = %.3g, det = %.6g)", fn, worst, det);
    return PF_OK;
}

int32_t check_intr(const pf_intrinsics* K, const char* fn) {
    if (!K) return set_error(PF_EINVAL, "%s: null intrinsics", fn);
    if (!(K->fx > 0.0) || !(K->fy > 0.0) || !isfinite(K->fx) || !isfinite(K->fy) || !isfinite(K->cx) ||
        !isfinite(K->cy))
        return set_error(PF_EINVAL, "%s: bad focal lengths or principal point", fn);
    if (K->width < 1 || K->height < 1 || (int64_t)K->width * K->height >= ((int64_t)1 << 30))
        return set_error(PF_EINVAL, "%s: bad image size %d x %d", fn, K->width, K->height);
    return PF_OK;
}

int32_t check_params(const pf_track_params* p, const char* fn) {
    if (!p) return set_error(PF_EINVAL, "%s: null parameters", fn);
    if (p->n_iters < 1 || p->n_iters > PF_MAX_ITERS)
        return set_error(PF_EINVAL, "%s: n_iters %d not in 1..%d", fn, p->n_iters, PF_MAX_ITERS);
    if (p->K < 1 || p->K > PF_MAX_K) return set_error(PF_EINVAL, "%s: K %d not in 1..%d", fn, p->K, PF_MAX_K);
    if (p->n_rates < 1 || p->n_rates > 3) return set_error(PF_EINVAL, "%s: n_rates %d not in 1..3", fn, p->n_rates);
    for (int r = 0; r < p->n_rates; ++r)
        if (p->rates[r] < 1) return set_error(PF_EINVAL, "%s: rate %d must be >= 1", fn, p->rates[r]);
    if (p->pixel_stride < 1) return set_error(PF_EINVAL, "%s: pixel_stride must be >= 1", fn);
    if (!(p->s1_deg >= 0.0) || !(p->s1_m >= 0.0) || !isfinite(p->s1_deg) || !isfinite(p->s1_m))
        return set_error(PF_EINVAL, "%s: the initial search size must be finite and >= 0", fn);
    if (!(p->beta >= 0.0 && p->beta <= 1.0)) return set_error(PF_EINVAL, "%s: beta must be in [0, 1]", fn);
    if (p->compose_mode != PF_COMPOSE_DECOUPLED && p->compose_mode != PF_COMPOSE_LITERAL)
        return set_error(PF_EINVAL, "%s: unknown compose_mode %d", fn, p->compose_mode);
    if (p->frame_index < 0 || p->frame_index >= (1 << 24))
        return set_error(PF_EINVAL, "%s: frame_index must be in 0..2^24-1", fn);
    if (p->polish_steps < 0 || p->polish_steps > 64) return set_error(PF_EINVAL, "%s: polish_steps not in 0..64", fn);
    if (p->alt_K != 0 && p->alt_K != 1) return set_error(PF_EINVAL, "%s: alt_K must be 0 or 1", fn);
    if (p->alt_K)
        for (int r = 0; r < p->n_rates; ++r)
            if (p->Ks[r] < 1 || p->Ks[r] > p->K)
                return set_error(PF_EINVAL, "%s: Ks[%d] = %d not in 1..K (%d)", fn, r, p->Ks[r], p->K);
    if (!(p->stop_deg >= 0.0) || !(p->stop_m >= 0.0) || !isfinite(p->stop_deg) || !isfinite(p->stop_m))
        return set_error(PF_EINVAL, "%s: the stop size must be finite and >= 0", fn);
    if (p->reserved != 0) return set_error(PF_EINVAL, "%s: reserved field must be 0", fn);
    return PF_OK;
}

}  // namespace

int32_t check_problem(const pf_batch_problem& q, int idx) {
    char fn[64];
    snprintf(fn, sizeof fn, "track_batch problem %d", idx);
    int32_t rc;
    if ((rc = check_tsdf(&q.vol, fn, false))) return rc;
    if ((rc = check_intr(&q.K, fn))) return rc;
    if ((rc = check_pose(&q.init, fn))) return rc;
    if ((rc = check_params(&q.params, fn))) return rc;
    if (!q.depth) return set_error(PF_EINVAL, "%s: null depth", fn);
    if (q.params.alt_K != 0 || q.params.stop_deg != 0.0 || q.params.stop_m != 0.0)
        return set_error(PF_EUNSUPPORTED, "%s: the alternating particle count and the stop rule are not batched", fn);
    if (q.params.K < 64) return set_error(PF_EINVAL, "%s: K %d < 64", fn, q.params.K);
    return PF_OK;
}

// Workspace of track_frame_noalloc: one array per GPU, held until the process ends. In host code
// `scratch` names a host-side stand-in, not device memory: its device address is looked up once
// per device (with that device current) and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[PF_NOALLOC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's `scratch`, looked up on the first call on that device.
int32_t scratch_of_current_device(void** ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(PF_EHIP, "track_frame_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(PF_EUNSUPPORTED, "track_frame_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(PF_EHIP, "track_frame_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return PF_OK;
}
}  // namespace

}  // namespace pf

using namespace pf;

extern "C" {

const char* pf_last_error(void) { return g_err; }

size_t tsdf_bytes(const pf_tsdf* v, size_t* weight_bytes) {
    if (weight_bytes) *weight_bytes = 0;
    if (!v || v->nx < 2 || v->ny < 2 || v->nz < 2) return 0;
    if (v->format != PF_F32_W_F32 && v->format != PF_F16_W_U8 && v->format != PF_I16_W_U8) return 0;
    if (v->layout == PF_LAYOUT_BRICKS) {
        if (v->nx % kBrickEdge || v->ny % kBrickEdge || v->nz % kBrickEdge || v->max_bricks < 1 ||
            v->max_bricks > kMaxBricks || v->reserved)
            return 0;
        if ((int64_t)(v->nx / kBrickEdge) * (v->ny / kBrickEdge) * (v->nz / kBrickEdge) >= ((int64_t)1 << 31)) return 0;
        if ((int64_t)(v->nx / kBrickEdge) * (v->ny / kBrickEdge) >= ((int64_t)1 << 24)) return 0;
        const BrickLayout L = brick_layout(v);
        if (weight_bytes) *weight_bytes = L.w_total;
        return L.t_total;
    }
    if (v->max_bricks != 0 || v->reserved) return 0;
    const int64_t n = (int64_t)v->nx * v->ny * v->nz;
    if (n >= ((int64_t)1 << 31) || (int64_t)v->nx * v->ny >= ((int64_t)1 << 24)) return 0;
    if (v->layout != PF_LAYOUT_LINEAR && v->layout != PF_LAYOUT_CELLS) return 0;
    const size_t tb = t_elem_bytes(v->format), wb = v->format == PF_F32_W_F32 ? 4 : 1;
    if (weight_bytes) *weight_bytes = (size_t)n * wb;
    if (v->layout == PF_LAYOUT_LINEAR) return (size_t)n * tb;
    return cell_mask_layout(v).t_total;
}

size_t tsdf_cells_offset(const pf_tsdf* v) {
    if (!v || tsdf_bytes(v, nullptr) == 0) return 0;
    return cells_offset_bytes(v);
}

size_t tsdf_mask_offset(const pf_tsdf* v) {
    if (!v || tsdf_bytes(v, nullptr) == 0) return 0;
    if (v->layout == PF_LAYOUT_CELLS) return cell_mask_layout(v).mask;
    if (v->layout == PF_LAYOUT_BRICKS) return brick_layout(v).pool_mask;
    return 0;
}

int32_t tsdf_brick_offsets(const pf_tsdf* v, size_t* index, size_t* coords, size_t* pool_t, size_t* pool_cells) {
    if (!v || v->layout != PF_LAYOUT_BRICKS || tsdf_bytes(v, nullptr) == 0)
        return set_error(PF_EINVAL, "tsdf_brick_offsets: not a valid BRICKS description");
    const BrickLayout L = brick_layout(v);
    if (index) *index = L.index;
    if (coords) *coords = L.coords;
    if (pool_t) *pool_t = L.pool_t;
    if (pool_cells) *pool_cells = L.pool_cells;
    return PF_OK;
}

int32_t tsdf_bricks_used(const pf_tsdf* v, int32_t* n_bricks, int32_t* overflow, void* stream) {
    int32_t rc = check_tsdf(v, "tsdf_bricks_used", false);
    if (rc) return rc;
    if (v->layout != PF_LAYOUT_BRICKS) return set_error(PF_EINVAL, "tsdf_bricks_used: not a BRICKS volume");
    BrickHeader h;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&h, v->tsdf, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return set_error(PF_EHIP, "tsdf_bricks_used: read-back failed");
    if (n_bricks) *n_bricks = h.n < v->max_bricks ? h.n : v->max_bricks;
    if (overflow) *overflow = h.overflow;
    return PF_OK;
}

int32_t tsdf_init(const pf_tsdf* v, void* stream) {
    int32_t rc = check_tsdf(v, "tsdf_init");
    if (rc) return rc;
    return launch_tsdf_init(v, (hipStream_t)stream);
}

int32_t tsdf_integrate(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* cam_to_world,
                       void* stream) {
    int32_t rc;
    if ((rc = check_tsdf(v, "tsdf_integrate"))) return rc;
    if (!depth) return set_error(PF_EINVAL, "tsdf_integrate: null depth");
    if ((rc = check_intr(K, "tsdf_integrate"))) return rc;
    if ((rc = check_pose(cam_to_world, "tsdf_integrate"))) return rc;
    return launch_tsdf_integrate(v, depth, K, cam_to_world, (hipStream_t)stream);
}

int32_t tsdf_export_linear(const pf_tsdf* v, float* T_out, float* W_out, void* stream) {
    int32_t rc = check_tsdf(v, "tsdf_export_linear", W_out != nullptr);
    if (rc) return rc;
    if (!T_out) return set_error(PF_EINVAL, "tsdf_export_linear: null T_out");
    if ((int64_t)v->nx * v->ny * v->nz >= ((int64_t)1 << 31))
        return set_error(PF_EUNSUPPORTED, "tsdf_export_linear: a linear copy needs < 2^31 voxels");
    return launch_tsdf_export(v, T_out, W_out, (hipStream_t)stream);
}

int32_t tsdf_import_linear(const pf_tsdf* v, const float* T_in, const float* W_in, void* stream) {
    int32_t rc = check_tsdf(v, "tsdf_import_linear");
    if (rc) return rc;
    if (!T_in) return set_error(PF_EINVAL, "tsdf_import_linear: null T_in");
    if ((int64_t)v->nx * v->ny * v->nz >= ((int64_t)1 << 31))
        return set_error(PF_EUNSUPPORTED, "tsdf_import_linear: a linear copy needs < 2^31 voxels");
    return launch_tsdf_import(v, T_in, W_in, (hipStream_t)stream);
}

int32_t backproject(const float* depth, const pf_intrinsics* K, int32_t pixel_stride, float* px, float* py, float* pz,
                    int32_t* n_out, void* stream) {
    (void)depth;
    int32_t rc = check_intr(K, "backproject");
    if (rc) return rc;
    if (!depth || !px || !py || !pz || !n_out) return set_error(PF_EINVAL, "backproject: null pointer");
    if (pixel_stride < 1) return set_error(PF_EINVAL, "backproject: pixel_stride must be >= 1");
    // the per-workgroup counts live after the count itself: n_out must hold
    // 1 + ceil(width*height / 1024) int32 values
    return launch_backproject(depth, K, pixel_stride, px, py, pz, n_out, n_out + 1, (hipStream_t)stream);
}

int32_t particles_score(const pf_tsdf* v, const float* px, const float* py, const float* pz, int32_t n_pts,
                        const float* poses, int32_t K, float* fitness, int32_t* n_valid, void* stream) {
    int32_t rc = check_tsdf(v, "particles_score", false);
    if (rc) return rc;
    if (!px || !py || !pz || !poses || !fitness || !n_valid)
        return set_error(PF_EINVAL, "particles_score: null pointer");
    if (n_pts < 1 || n_pts >= (1 << 30))
        return set_error(PF_EINVAL, "particles_score: n_pts %d not in 1 .. 2^30 - 1", n_pts);
    if (K < 1) return set_error(PF_EINVAL, "particles_score: K %d must be >= 1", K);
    Points p{px, py, pz, n_pts, nullptr};
    return launch_score(make_view(v), p, poses, K, fitness, n_valid, (hipStream_t)stream);
}

int32_t particles_score_grad(const pf_tsdf* v, const float* px, const float* py, const float* pz, int32_t n_pts,
                             const double* base, const double* xi, int32_t B, int32_t compose_mode, float* fitness,
                             float* grad, int32_t* n_valid, void* stream) {
    int32_t rc = check_tsdf(v, "particles_score_grad", false);
    if (rc) return rc;
    if (!px || !py || !pz || !base || !fitness || !grad)
        return set_error(PF_EINVAL, "particles_score_grad: null pointer");
    if (n_pts < 1) return set_error(PF_EINVAL, "particles_score_grad: n_pts %d must be >= 1", n_pts);
    if (B < 1 || B > 65535) return set_error(PF_EINVAL, "particles_score_grad: B %d not in 1..65535", B);
    if (compose_mode != PF_COMPOSE_DECOUPLED && compose_mode != PF_COMPOSE_LITERAL)
        return set_error(PF_EINVAL, "particles_score_grad: unknown compose_mode %d", compose_mode);
    Points p{px, py, pz, n_pts, nullptr};
    return launch_grad(make_view(v), p, base, xi, B, 1, compose_mode, fitness, grad, n_valid, nullptr,
                       (hipStream_t)stream);
}

int32_t pf_score_config(int32_t poses_per_group, int32_t group_size) {
    return score_config(poses_per_group, group_size);
}

int32_t pf_score_mask(int32_t mode) { return score_mask(mode); }

size_t particles_state_bytes(int32_t K) {
    if (K < 1 || K > PF_MAX_K) return 0;
    return state_bytes(K);
}

int32_t particles_state_init(void* state, const pf_pose* init, const pf_track_params* p, float* next_poses,
                             void* stream) {
    int32_t rc;
    if (!state || !next_poses) return set_error(PF_EINVAL, "particles_state_init: null pointer");
    if ((rc = check_pose(init, "particles_state_init"))) return rc;
    if ((rc = check_params(p, "particles_state_init"))) return rc;
    return state_init(state, init, p, PF_F32_W_F32, next_poses, (hipStream_t)stream);
}

int32_t particles_update(const pf_tsdf* v, const float* px, const float* py, const float* pz, int32_t n_pts,
                         const float* fitness, const int32_t* n_valid, void* state, int32_t K, float* next_poses,
                         void* stream) {
    (void)n_valid;
    int32_t rc = check_tsdf(v, "particles_update", false);
    if (rc) return rc;
    if (!px || !py || !pz || !fitness || !state || !next_poses)
        return set_error(PF_EINVAL, "particles_update: null pointer");
    if (n_pts < 1) return set_error(PF_EINVAL, "particles_update: n_pts %d must be >= 1", n_pts);
    if (K < 1 || K > PF_MAX_K) return set_error(PF_EINVAL, "particles_update: K %d not in 1..%d", K, PF_MAX_K);
    Points p{px, py, pz, n_pts, nullptr};
    return update(make_view(v), p, fitness, state, K, next_poses, (hipStream_t)stream);
}

size_t track_workspace_bytes(const pf_intrinsics* K, const pf_track_params* p) {
    if (check_intr(K, "track_workspace_bytes") || check_params(p, "track_workspace_bytes")) return 0;
    return workspace_bytes(K, p);
}

int32_t track_frame(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* init,
                    const pf_track_params* p, pf_pose* out, pf_track_stats* stats, void* workspace, size_t ws_bytes,
                    void* stream) {
    int32_t rc;
    if ((rc = check_tsdf(v, "track_frame", false))) return rc;
    if ((rc = check_intr(K, "track_frame"))) return rc;
    if ((rc = check_pose(init, "track_frame"))) return rc;
    if ((rc = check_params(p, "track_frame"))) return rc;
    if (!depth || !out || !workspace) return set_error(PF_EINVAL, "track_frame: null pointer");
    return track(v, depth, K, init, p, out, stats, workspace, ws_bytes, (hipStream_t)stream, false);
}

int32_t track_frame_fuse(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* init,
                         const pf_track_params* p, pf_pose* out, pf_track_stats* stats, void* workspace,
                         size_t ws_bytes, void* stream) {
    int32_t rc;
    if ((rc = check_tsdf(v, "track_frame_fuse"))) return rc;
    if ((rc = check_intr(K, "track_frame_fuse"))) return rc;
    if ((rc = check_pose(init, "track_frame_fuse"))) return rc;
    if ((rc = check_params(p, "track_frame_fuse"))) return rc;
    if (!depth || !out || !workspace) return set_error(PF_EINVAL, "track_frame_fuse: null pointer");
    return track(v, depth, K, init, p, out, stats, workspace, ws_bytes, (hipStream_t)stream, true);
}

int32_t track_frame_noalloc(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* init,
                            const pf_track_params* p, pf_pose* out, pf_track_stats* stats, void* stream) {
    int32_t rc;
    if ((rc = check_tsdf(v, "track_frame_noalloc", false))) return rc;
    if ((rc = check_intr(K, "track_frame_noalloc"))) return rc;
    if ((rc = check_pose(init, "track_frame_noalloc"))) return rc;
    if ((rc = check_params(p, "track_frame_noalloc"))) return rc;
    if (!depth || !out) return set_error(PF_EINVAL, "track_frame_noalloc: null pointer");
    const size_t need = workspace_bytes(K, p);
    if (need > (size_t)PF_NOALLOC_WORKSPACE_BYTES)
        return set_error(PF_ENOMEM, "track_frame_noalloc: needs %zu bytes of workspace, the library's array holds %zu",
                         need, (size_t)PF_NOALLOC_WORKSPACE_BYTES);
    void* ws = nullptr;
    if ((rc = scratch_of_current_device(&ws))) return rc;
    return track(v, depth, K, init, p, out, stats, ws, (size_t)PF_NOALLOC_WORKSPACE_BYTES, (hipStream_t)stream, false);
}

int32_t pf_timing_enable(int32_t on) { return timing_enable(on); }

int32_t pf_timing_read(double* score_ms, int64_t* score_launches, int64_t* score_evals, int32_t reset) {
    return timing_read(score_ms, score_launches, score_evals, reset);
}

}  // extern "C"
