// TSDF volume kernels for gfx950: initialisation, KinectFusion-style fusion of one depth frame
// (Sec. III "Method overview"; Fig. 2), conversion to / from a linear FP32 form, and upkeep of the
// cell-major replica that particle scoring reads (PF_LAYOUT_CELLS).
//
// Layout: x-fastest dense grid, T[(k*ny + j)*nx + i]. One thread owns one voxel, so the
// read-modify-write of fusion needs no atomics. Consecutive threads own consecutive x, so the
// T/W traffic of updated voxels is coalesced; voxels that are not updated are never read,
// because the decision depends only on the voxel index, the pose and the depth image. A voxel is
// corner (dx, dy, dz) of the cells (i-dx, j-dy, k-dz); its replica entries are rewritten only
// when its stored value changes, which outside the truncation band (free space stays at +1) is
// rare, so the replica costs little fusion traffic.
#include <math.h>

#include "pf_sample.hpp"

namespace pf {
namespace {

constexpr int kBlock = 256;

template <int FMT>
struct Store;

template <>
struct Store<PF_F32_W_F32> {
    using T = float;
    using W = float;
    __device__ static inline T enc(float v) { return v; }
    __device__ static inline float dec(T v) { return v; }
    __device__ static inline W encw(float w) { return w; }
    __device__ static inline float decw(W w) { return w; }
    __device__ static inline bool same(T a, T b) { return __float_as_uint(a) == __float_as_uint(b); }
    // replica value of a stored T: itself inside the band, NaN outside it
    __device__ static inline T cell(T v) { return fabsf(v) < 1.0f ? v : __uint_as_float(0x7fc00000u); }
};

template <>
struct Store<PF_F16_W_U8> {
    using T = __half;
    using W = uint8_t;
    __device__ static inline T enc(float v) { return __float2half_rn(v); }
    __device__ static inline float dec(T v) { return __half2float(v); }
    __device__ static inline W encw(float w) { return (uint8_t)fminf(255.0f, fmaxf(0.0f, rintf(w))); }
    __device__ static inline float decw(W w) { return (float)w; }
    __device__ static inline bool same(T a, T b) { return __half_as_ushort(a) == __half_as_ushort(b); }
    __device__ static inline T cell(T v) { return fabsf(__half2float(v)) < 1.0f ? v : __ushort_as_half(0x7e00u); }
};

template <>
struct Store<PF_I16_W_U8> {
    using T = int16_t;
    using W = uint8_t;
    // RNE(T * 32767) clamped to +-32767; +-32767 are the out-of-band values
    __device__ static inline T enc(float v) { return (int16_t)fminf(32767.0f, fmaxf(-32767.0f, rintf(v * 32767.0f))); }
    __device__ static inline float dec(T v) { return (float)v * (1.0f / 32767.0f); }
    __device__ static inline W encw(float w) { return (uint8_t)fminf(255.0f, fmaxf(0.0f, rintf(w))); }
    __device__ static inline float decw(W w) { return (float)w; }
    __device__ static inline bool same(T a, T b) { return a == b; }
    __device__ static inline T cell(T v) { return v; }   // no NaN: the scoring tests the corners
};

struct Dims {
    int nx, ny, nz;
    int64_t n;        // voxels
    int64_t ncells;   // (nx-1)(ny-1)(nz-1)
};

Dims dims_of(const pf_tsdf* v) {
    Dims d;
    d.nx = v->nx;
    d.ny = v->ny;
    d.nz = v->nz;
    d.n = (int64_t)v->nx * v->ny * v->nz;
    d.ncells = (int64_t)(v->nx - 1) * (v->ny - 1) * (v->nz - 1);
    return d;
}

// Writes voxel (i, j, k)'s replica value (Store::cell of its stored value) into every cell that has
// it as a corner.
template <typename T>
__device__ inline void write_corners(T* cells, const Dims& d, int i, int j, int k, T val) {
    const int cnx = d.nx - 1, cny = d.ny - 1, cnz = d.nz - 1;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int ci = i - dx, cj = j - dy, ck = k - dz;
                if (ci < 0 || cj < 0 || ck < 0 || ci >= cnx || cj >= cny || ck >= cnz) continue;
                const int64_t c = ((int64_t)ck * cny + cj) * cnx + ci;
                cells[(c << 3) + (dx + 2 * dy + 4 * dz)] = val;
            }
}

// The cell-validity mask of a CELLS volume (64-bit words of 4x4x4 cells) and the per-word bytes
// that fusion sets when a voxel of the word's cells enters or leaves the band.
struct MaskArgs {
    unsigned long long* mask;
    uint8_t* flags;
    int mwx, mwy, mwz;
};

MaskArgs mask_args(const pf_tsdf* v) {
    MaskArgs m{nullptr, nullptr, 0, 0, 0};
    if (v->layout != PF_LAYOUT_CELLS) return m;
    const CellMask M = cell_mask_layout(v);
    m.mask = reinterpret_cast<unsigned long long*>(static_cast<char*>(v->tsdf) + M.mask);
    m.flags = reinterpret_cast<uint8_t*>(static_cast<char*>(v->tsdf) + M.flags);
    m.mwx = M.mwx;
    m.mwy = M.mwy;
    m.mwz = M.mwz;
    return m;
}

// The band test of the scoring kernels on a stored value.
template <int FMT>
__device__ inline bool stored_in_band(typename Store<FMT>::T v) {
    return Fmt<FMT>::in_band(Fmt<FMT>::val(v));
}

// Flags the mask words of the (up to 8) cells that have voxel (i, j, k) as a corner.
__device__ inline void flag_cells_of(const MaskArgs& m, const Dims& d, int i, int j, int k) {
    const int x0 = max(i - 1, 0) >> 2, x1 = min(i, d.nx - 2) >> 2;
    const int y0 = max(j - 1, 0) >> 2, y1 = min(j, d.ny - 2) >> 2;
    const int z0 = max(k - 1, 0) >> 2, z1 = min(k, d.nz - 2) >> 2;
    for (int z = z0; z <= z1; ++z)
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) m.flags[((int64_t)z * m.mwy + y) * m.mwx + x] = 1;
}

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_init(void* Tv, void* Wv, void* Cv, Dims d, MaskArgs m) {
    using S = Store<FMT>;
    auto* T = static_cast<typename S::T*>(Tv);
    auto* W = static_cast<typename S::W*>(Wv);
    auto* C = static_cast<typename S::T*>(Cv);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const typename S::T one = S::enc(1.0f);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < d.n; i += stride) {
        T[i] = one;
        W[i] = S::encw(0.0f);
    }
    const typename S::T one_cell = S::cell(one);
    if (C)
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (d.ncells << 3); i += stride) C[i] = one_cell;
    // no voxel is in the band: every mask word is 0 and none is flagged
    const int64_t words = (int64_t)m.mwx * m.mwy * m.mwz;
    for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < words; w += stride) {
        m.mask[w] = 0;
        m.flags[w] = 0;
    }
}

// Rebuilds the flagged mask words (every word when `all`) from the x-fastest storage and clears
// their flags. A wave scans 64 consecutive words' flags, then rebuilds the flagged words together,
// kMaskWords at a time so that their corner loads are in flight at once: lane l takes cell l of a
// word's 4x4x4 block (bit l of the word), tests its 8 corners, and the wave's ballot is the word.
// Cells past the last one of the grid have no corners there: bit 0 (their loads read the grid's
// first cell instead, in bounds, and are ignored).
constexpr int kMaskWords = 4;

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_mask_update(const void* Tv, Dims d, MaskArgs m, int all) {
    const auto* T = static_cast<const typename Store<FMT>::T*>(Tv);
    const int64_t words = (int64_t)m.mwx * m.mwy * m.mwz;
    const int lane = threadIdx.x & (kWave - 1);
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int64_t nxy = (int64_t)d.nx * d.ny;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) - lane; base < words; base += stride) {
        const int64_t own = base + lane;
        unsigned long long todo = __ballot(own < words && (all || m.flags[own]));
        while (todo) {   // uniform: the same words for every lane
            int64_t w[kMaskWords];
            bool inside[kMaskWords];
            typename Store<FMT>::T c[kMaskWords][8];
#pragma unroll
            for (int q = 0; q < kMaskWords; ++q) {
                w[q] = todo ? base + (__ffsll((long long)todo) - 1) : -1;   // -1: no word left
                todo &= todo - 1;
                // 32-bit: a dense grid holds under 2^31 voxels, so under 2^25 words (64-bit division
                // is a long emulated sequence, and this runs once per flagged word)
                const unsigned wu = w[q] < 0 ? 0u : (unsigned)w[q], row = wu / (unsigned)m.mwx;
                const int wx = (int)(wu - row * (unsigned)m.mwx), wy = (int)(row % (unsigned)m.mwy);
                const int wz = (int)(row / (unsigned)m.mwy);
                const int cx = wx * 4 + lx, cy = wy * 4 + ly, cz = wz * 4 + lz;
                inside[q] = cx < d.nx - 1 && cy < d.ny - 1 && cz < d.nz - 1;
                const int64_t b = inside[q] ? ((int64_t)cz * d.ny + cy) * d.nx + cx : 0;
                c[q][0] = T[b];
                c[q][1] = T[b + 1];
                c[q][2] = T[b + d.nx];
                c[q][3] = T[b + d.nx + 1];
                c[q][4] = T[b + nxy];
                c[q][5] = T[b + nxy + 1];
                c[q][6] = T[b + nxy + d.nx];
                c[q][7] = T[b + nxy + d.nx + 1];
            }
#pragma unroll
            for (int q = 0; q < kMaskWords; ++q) {
                bool valid = inside[q];
#pragma unroll
                for (int r = 0; r < 8; ++r) valid &= stored_in_band<FMT>(c[q][r]);
                const unsigned long long word = __ballot(valid);
                if (lane == 0 && w[q] >= 0) {
                    m.mask[w[q]] = word;
                    m.flags[w[q]] = 0;
                }
            }
        }
    }
}

struct FuseArgs {
    void* T;
    void* W;
    void* C;
    MaskArgs m;   // CELLS: the validity mask, else null
    Dims d;
    double vs, tau, ox, oy, oz;
    double R[9], t[3];
    double fx, fy, cx, cy;
    int width, height;
    float w_max;
    const float* depth;
    // FP32 copies for the conservative pre-test: camera-frame depth and pixel coordinates of
    // voxel (i, j, k) are q = Q0 + i Qi + j Qj + k Qk with Q0 = R^T (origin - t), Qi = R^T e_x vs, ...
    float q0[3], qi[3], qj[3], qk[3];
    double zfar;   // largest camera depth of a grid corner: no voxel lies deeper
};

// The fields of a fusion that depend on the camera pose (R, t): the pose itself and the FP32 copies
// of its projection for the pre-tests. The same code on the host and on the device (this file is
// compiled without contraction on both), so a pose read from device memory gives the same fields
// as the same pose passed from the host.
__host__ __device__ inline void fuse_pose_fields(FuseArgs& a, const double* R, const double* t) {
    for (int q = 0; q < 9; ++q) a.R[q] = R[q];
    for (int q = 0; q < 3; ++q) a.t[q] = t[q];
    for (int r = 0; r < 3; ++r) {   // camera axis r = column r of R
        a.q0[r] = (float)(a.R[r] * (a.ox - a.t[0]) + a.R[3 + r] * (a.oy - a.t[1]) + a.R[6 + r] * (a.oz - a.t[2]));
        a.qi[r] = (float)(a.R[r] * a.vs);
        a.qj[r] = (float)(a.R[3 + r] * a.vs);
        a.qk[r] = (float)(a.R[6 + r] * a.vs);
    }
    a.zfar = -1e300;
    for (int c = 0; c < 8; ++c) {
        const double p[3] = {a.ox + a.vs * ((c & 1) ? a.d.nx - 1 : 0), a.oy + a.vs * ((c & 2) ? a.d.ny - 1 : 0),
                             a.oz + a.vs * ((c & 4) ? a.d.nz - 1 : 0)};
        a.zfar = fmax(a.zfar, a.R[2] * (p[0] - a.t[0]) + a.R[5] * (p[1] - a.t[1]) + a.R[8] * (p[2] - a.t[2]));
    }
    a.zfar += 1e-6 * (fabs(a.zfar) + 1.0);
}

// The projection is evaluated in FP64 with the same operation order as the plain definition,
// and this file is compiled without multiply-add contraction, so the per-voxel decisions
// (updated or not, which pixel) are those of an FP64 evaluation of the formula as written; the
// running average is FP32.
// Conservative FP32 pre-tests drop most voxels of the grid (behind the camera, or outside the image
// by more than two pixels) before any FP64 work; each drops only voxels the FP64 test drops too.
// Returns whether voxel (i, j, k) is updated by this frame, and its observation phi.
__device__ inline bool fuse_decide(const FuseArgs& a, int i, int j, int k, double& phi_out) {
    {
        // FP32 pre-test, conservative: it drops only voxels the FP64 test below drops too. The FP32
        // camera coordinates carry at most ~1e-5 m of error here (|q| < 10 m), so a voxel is
        // dropped as behind the camera only at qz < -1e-3 m, and as outside the image only at
        // qz > 0.2 m (pixel error < 0.5) and more than two pixels beyond the border. The
        // reciprocal is the hardware's (1 ulp): for a pixel within reach of the border its error is
        // below 1e-3 pixel.
        const float fi = (float)i, fj = (float)j, fk = (float)k;
        const float z32 = a.q0[2] + fi * a.qi[2] + fj * a.qj[2] + fk * a.qk[2];
        if (z32 < -1e-3f) return false;
        if (z32 > 0.2f) {
            const float x32 = a.q0[0] + fi * a.qi[0] + fj * a.qj[0] + fk * a.qk[0];
            const float y32 = a.q0[1] + fi * a.qi[1] + fj * a.qj[1] + fk * a.qk[1];
            const float iz = __builtin_amdgcn_rcpf(z32);
            const float u32 = (float)a.fx * x32 * iz + (float)a.cx;
            const float v32 = (float)a.fy * y32 * iz + (float)a.cy;
            if (!(u32 > -2.5f && u32 < (float)a.width + 1.5f && v32 > -2.5f && v32 < (float)a.height + 1.5f)) return false;
        }
    }
    const double px = a.ox + a.vs * (double)i;
    const double py = a.oy + a.vs * (double)j;
    const double pz = a.oz + a.vs * (double)k;
    const double dx = px - a.t[0], dy = py - a.t[1], dz = pz - a.t[2];
    const double qz = a.R[2] * dx + a.R[5] * dy + a.R[8] * dz;
    if (!(qz > 0.0)) return false;
    const double qx = a.R[0] * dx + a.R[3] * dy + a.R[6] * dz;
    const double qy = a.R[1] * dx + a.R[4] * dy + a.R[7] * dz;
    if (qz > 1e-6) {   // (below, FP32 could overflow; the FP64 test decides alone)
        const float iz = __builtin_amdgcn_rcpf((float)qz);
        const float uf32 = (float)a.fx * (float)qx * iz + (float)a.cx;
        const float vf32 = (float)a.fy * (float)qy * iz + (float)a.cy;
        if (!(uf32 > -2.5f && uf32 < (float)a.width + 1.5f && vf32 > -2.5f && vf32 < (float)a.height + 1.5f)) return false;
    }
    const double u = a.fx * qx / qz + a.cx;
    const double v = a.fy * qy / qz + a.cy;
    const double uf = floor(u + 0.5), vf = floor(v + 0.5);
    if (uf < 0.0 || uf >= (double)a.width || vf < 0.0 || vf >= (double)a.height) return false;
    const int ui = (int)uf, vi = (int)vf;
    const double D = (double)a.depth[(int64_t)vi * a.width + ui];
    if (!(isfinite(D) && D > 0.0)) return false;
    const double eta = D - qz;
    if (eta < -a.tau) return false;
    double phi = eta / a.tau;
    if (phi > 1.0) phi = 1.0;
    phi_out = phi;
    return true;
}

// The running-average update of one stored voxel (T[e], W[e]); returns whether T changed.
template <int FMT>
__device__ inline bool fuse_apply(const FuseArgs& a, int64_t e, double phi, typename Store<FMT>::T& told,
                                  typename Store<FMT>::T& tnew) {
    using S = Store<FMT>;
    auto* T = static_cast<typename S::T*>(a.T);
    auto* W = static_cast<typename S::W*>(a.W);
    told = T[e];
    const float w = S::decw(W[e]);
    const float tn = (S::dec(told) * w + (float)phi) / (w + 1.0f);
    tnew = S::enc(tn);
    const bool changed = !S::same(told, tnew);
    if (changed) T[e] = tnew;
    W[e] = S::encw(fminf(w + 1.0f, a.w_max));
    return changed;
}

// Grid: a workgroup owns a brick of kFuseX x kFuseY x kFuseZ voxels (a wave per x row, each thread
// walking kFuseZ slices, kFuseU at a time, so no index division and each wave lives long enough to
// amortise its start). A brick whose 8 corners all lie behind the camera, or all beyond one side of the image
// (a plane through the camera centre, two pixels out, with a margin far above the FP32 error), is
// skipped as a whole: every voxel in it is a convex combination of the corners, so the per-voxel
// tests would drop it too. Lane l of each wave evaluates corner l mod 8 and ballots combine the
// corners (the test is the same for every wave of the workgroup), instead of every lane walking all
// eight: most workgroups of a frame end here.
constexpr int kFuseX = 64, kFuseY = kBlock / kFuseX, kFuseZ = 32;

__device__ inline bool brick_outside(const FuseArgs& a, int i0, int j0, int k0, int i1, int j1, int k1) {
    // the four side planes n . q >= 0 of the image widened by two pixels, q in camera coordinates
    const float fx = (float)a.fx, fy = (float)a.fy, cx = (float)a.cx, cy = (float)a.cy;
    const float W = (float)a.width, H = (float)a.height;
    const float n[4][3] = {{fx, 0.0f, cx + 2.5f}, {-fx, 0.0f, W + 1.5f - cx},
                           {0.0f, fy, cy + 2.5f}, {0.0f, -fy, H + 1.5f - cy}};
    const int c = (int)threadIdx.x & 7;
    const float fi = (float)((c & 1) ? i1 : i0), fj = (float)((c & 2) ? j1 : j0), fk = (float)((c & 4) ? k1 : k0);
    float q[3];
    for (int r = 0; r < 3; ++r) q[r] = a.q0[r] + fi * a.qi[r] + fj * a.qj[r] + fk * a.qk[r];
    // a test holds for the brick when it holds at all 8 corners (lanes 0..7 of the wave)
    bool outside = (__ballot(q[2] < -1e-3f) & 0xffull) == 0xffull;
    for (int p = 0; p < 4; ++p) {
        const float d = n[p][0] * q[0] + n[p][1] * q[1] + n[p][2] * q[2];
        const float tol = 1e-3f * (fabsf(n[p][0]) + fabsf(n[p][1]) + fabsf(n[p][2]));
        outside |= (__ballot(d < -tol) & 0xffull) == 0xffull;
    }
    return outside;
}

// The voxels (i, j, k0..k1) of one thread, kFuseU slices at a time in phases, so that each phase's
// loads are in flight together instead of one voxel's dependent rounds after another's: the T and W
// of all kFuseU voxels (their addresses do not depend on the image, so these loads are issued first
// and run under the projection arithmetic; a voxel that is not updated wastes its 8 bytes), the
// projections (fuse_decide's FP64 formula, with the same operations in the same order; its FP32
// pre-tests only skip work and are left out), then their depth pixels (a voxel outside the image
// reads pixel 0 and is dropped), the decisions and the updates. One dependent memory round per
// phase (the depth pixel) is left exposed instead of two.
constexpr int kFuseU = 4;

template <int FMT>
__device__ inline void fuse_column(const FuseArgs& a, int i, int j, int k0, int k1) {
    using S = Store<FMT>;
    auto* T = static_cast<typename S::T*>(a.T);
    auto* W = static_cast<typename S::W*>(a.W);
    const double px = a.ox + a.vs * (double)i;
    const double py = a.oy + a.vs * (double)j;
    const double dx = px - a.t[0], dy = py - a.t[1];
    for (int kb = k0; kb <= k1; kb += kFuseU) {
        const int64_t e0 = ((int64_t)kb * a.d.ny + j) * a.d.nx + i, slice = (int64_t)a.d.ny * a.d.nx;
        typename S::T told[kFuseU];
        typename S::W wold[kFuseU];
#pragma unroll
        for (int u = 0; u < kFuseU; ++u) {
            if (kb + u <= k1) {
                told[u] = T[e0 + u * slice];
                wold[u] = W[e0 + u * slice];
            }
        }
        double qz[kFuseU];
        unsigned pix[kFuseU];   // below 2^30: the boundary rejects larger images
        bool in[kFuseU];
#pragma unroll
        for (int u = 0; u < kFuseU; ++u) {
            const int k = kb + u;
            const double pz = a.oz + a.vs * (double)k;
            const double dz = pz - a.t[2];
            qz[u] = a.R[2] * dx + a.R[5] * dy + a.R[8] * dz;
            const double qx = a.R[0] * dx + a.R[3] * dy + a.R[6] * dz;
            const double qy = a.R[1] * dx + a.R[4] * dy + a.R[7] * dz;
            const double uu = a.fx * qx / qz[u] + a.cx;
            const double vv = a.fy * qy / qz[u] + a.cy;
            const double uf = floor(uu + 0.5), vf = floor(vv + 0.5);
            in[u] = k <= k1 && qz[u] > 0.0 && uf >= 0.0 && uf < (double)a.width && vf >= 0.0 &&
                    vf < (double)a.height;
            pix[u] = in[u] ? (unsigned)vf * (unsigned)a.width + (unsigned)uf : 0u;
        }
        float Dp[kFuseU];
#pragma unroll
        for (int u = 0; u < kFuseU; ++u) Dp[u] = a.depth[pix[u]];
        double phi[kFuseU];
        bool go[kFuseU];
#pragma unroll
        for (int u = 0; u < kFuseU; ++u) {
            const double D = (double)Dp[u];
            const double eta = D - qz[u];
            go[u] = in[u] && isfinite(D) && D > 0.0 && !(eta < -a.tau);
            double ph = eta / a.tau;
            if (ph > 1.0) ph = 1.0;
            phi[u] = ph;
        }
#pragma unroll
        for (int u = 0; u < kFuseU; ++u) {
            if (!go[u]) continue;
            const float w = S::decw(wold[u]);
            const float tn = (S::dec(told[u]) * w + (float)phi[u]) / (w + 1.0f);
            const typename S::T tnew = S::enc(tn);
            const bool changed = !S::same(told[u], tnew);
            if (changed) T[e0 + u * slice] = tnew;
            W[e0 + u * slice] = S::encw(fminf(w + 1.0f, a.w_max));
            if (changed && a.C) {
                write_corners(static_cast<typename S::T*>(a.C), a.d, i, j, kb + u, S::cell(tnew));
                if (stored_in_band<FMT>(told[u]) != stored_in_band<FMT>(tnew)) flag_cells_of(a.m, a.d, i, j, kb + u);
            }
        }
    }
}

// Fills the pose fields of a fusion from a pose in device memory (the tracker's state).
__global__ void k_fuse_pose(FuseArgs* out, FuseArgs base, const double* R, const double* t) {
    fuse_pose_fields(base, R, t);
    *out = base;
}

template <int FMT>
__attribute__((always_inline)) __device__ inline void fuse_brick(const FuseArgs& a) {
    const int i0 = blockIdx.x * kFuseX, j0 = blockIdx.y * kFuseY, k0 = blockIdx.z * kFuseZ;
    const int i1 = min(a.d.nx, i0 + kFuseX) - 1, j1 = min(a.d.ny, j0 + kFuseY) - 1, k1 = min(a.d.nz, k0 + kFuseZ) - 1;
    if (brick_outside(a, i0, j0, k0, i1, j1, k1)) return;
    const int i = i0 + (int)(threadIdx.x % kFuseX), j = j0 + (int)(threadIdx.x / kFuseX);
    if (i > i1 || j > j1) return;
    fuse_column<FMT>(a, i, j, k0, k1);
}

// DEV: the fusion's arguments come from device memory (a pose the device computed), else from the
// kernel arguments. Two instantiations rather than a run-time choice: selecting between the two
// sources made the compiler copy the whole argument block into vector registers (122 per lane).
template <int FMT, bool DEV>
__global__ __launch_bounds__(kBlock) void k_integrate(FuseArgs a0, const FuseArgs* __restrict__ ap) {
    if constexpr (DEV) {
        const FuseArgs a = *ap;   // read before any store, into scalar registers
        fuse_brick<FMT>(a);
    } else {
        fuse_brick<FMT>(a0);
    }
}

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_export(const void* Tv, const void* Wv, Dims d, float* To, float* Wo) {
    using S = Store<FMT>;
    const auto* T = static_cast<const typename S::T*>(Tv);
    const auto* W = static_cast<const typename S::W*>(Wv);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < d.n; i += stride) {
        To[i] = S::dec(T[i]);
        if (Wo) Wo[i] = S::decw(W[i]);
    }
}

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_import(void* Tv, void* Wv, Dims d, const float* Ti, const float* Wi) {
    using S = Store<FMT>;
    auto* T = static_cast<typename S::T*>(Tv);
    auto* W = static_cast<typename S::W*>(Wv);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < d.n; i += stride) {
        T[i] = S::enc(Ti[i]);
        W[i] = S::encw(Wi ? Wi[i] : 0.0f);
    }
}

// Rebuilds the whole cell replica from the x-fastest storage.
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_build_cells(const void* Tv, void* Cv, Dims d) {
    using S = Store<FMT>;
    const auto* T = static_cast<const typename S::T*>(Tv);
    auto* C = static_cast<typename S::T*>(Cv);
    const int cnx = d.nx - 1, cny = d.ny - 1;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < d.ncells; c += stride) {
        const int ck = (int)(c / ((int64_t)cnx * cny));
        const int64_t rem = c - (int64_t)ck * cnx * cny;
        const int cj = (int)(rem / cnx), ci = (int)(rem - (int64_t)cj * cnx);
        const int64_t b = ((int64_t)ck * d.ny + cj) * d.nx + ci;
        const int64_t nxy = (int64_t)d.nx * d.ny;
        typename S::T* o = C + (c << 3);
        o[0] = S::cell(T[b]);
        o[1] = S::cell(T[b + 1]);
        o[2] = S::cell(T[b + d.nx]);
        o[3] = S::cell(T[b + d.nx + 1]);
        o[4] = S::cell(T[b + nxy]);
        o[5] = S::cell(T[b + nxy + 1]);
        o[6] = S::cell(T[b + nxy + d.nx]);
        o[7] = S::cell(T[b + nxy + d.nx + 1]);
    }
}

// ---------------------------------------------------------------- sparse bricks (PF_LAYOUT_BRICKS)
// Bricks of 8x8x8 voxels in a pool behind a dense brick-index grid. A fusion first lists candidate
// bricks from the depth image, gives a pool slot to every candidate the frame puts a band voxel into
// (the same FP64 decision per voxel as the update), initialises the new slots, and then updates
// every allocated brick exactly as the dense layouts update a voxel.
struct BrickArgs {
    BrickHeader* hdr;
    int* index;     // brick-index grid: slot or -1 (kCandidate while a fusion lists candidates)
    int* cand;      // candidate list, one entry per brick at most
    int4* coords;   // slot -> brick coordinates
    void* T;        // slots' T, 512 each
    void* C;        // slots' cells, 512 x 8 each
    unsigned long long* M;   // slots' cell-validity words, 8 each
    void* W;        // slots' W
    int nbx, nby, nbz, max_bricks;
};

BrickArgs brick_args(const pf_tsdf* v) {
    const BrickLayout L = brick_layout(v);
    char* base = static_cast<char*>(v->tsdf);
    BrickArgs b;
    b.hdr = reinterpret_cast<BrickHeader*>(base);
    b.index = reinterpret_cast<int*>(base + L.index);
    b.cand = reinterpret_cast<int*>(base + L.cand);
    b.coords = reinterpret_cast<int4*>(base + L.coords);
    b.T = base + L.pool_t;
    b.C = base + L.pool_cells;
    b.M = reinterpret_cast<unsigned long long*>(base + L.pool_mask);
    b.W = v->weight;
    b.nbx = L.nbx;
    b.nby = L.nby;
    b.nbz = L.nbz;
    b.max_bricks = v->max_bricks;
    return b;
}

__device__ inline int brick_slot(const BrickArgs& b, int bx, int by, int bz) {
    if (bx < 0 || by < 0 || bz < 0 || bx >= b.nbx || by >= b.nby || bz >= b.nbz) return -1;
    return b.index[((int64_t)bz * b.nby + by) * b.nbx + bx];
}

__device__ inline int brick_local(int i, int j, int k) { return (i & 7) | ((j & 7) << 3) | ((k & 7) << 6); }

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_bricks_reset(BrickArgs b, int64_t n_index) {
    if (blockIdx.x == 0 && threadIdx.x < 8) {
        if (threadIdx.x == 0) *b.hdr = BrickHeader{0, 0, 0, 0};
        reinterpret_cast<typename Store<FMT>::T*>(reinterpret_cast<char*>(b.hdr) + kBrickOnes)[threadIdx.x] =
            Store<FMT>::cell(Store<FMT>::enc(1.0f));
    }
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_index; i += stride) b.index[i] = -1;
}

// Start of a fusion: the count comes back to the pool size after an overflow, the slots in use so
// far are recorded, and the candidate list is emptied.
__global__ void k_bricks_prep(BrickArgs b) {
    const int n = min(b.hdr->n, b.max_bricks);
    b.hdr->n = n;
    b.hdr->n_prev = n;
    b.hdr->ncand = 0;
}

// Candidates for new slots, found from the depth image. A voxel the frame puts in the band has a
// nearest pixel (u, v) with valid depth D and a camera depth qz in (D - tau, D + tau], so its
// centre lies in the frustum segment of that pixel's footprint [u - 1/2, u + 1/2] x
// [v - 1/2, v + 1/2] between those depths. The grid coordinates are an affine function of the
// camera coordinates, so the segment's 8 corners bound the voxel's index; one thread per pixel
// lists every brick without a slot that this box (widened by kCandMargin voxels against rounding)
// touches, each brick once (its entry is claimed from -1 to kCandidate). The exact per-voxel test
// then runs on the listed bricks only.
constexpr int kCandidate = -2;
constexpr double kCandMargin = 0.01;   // voxels

__global__ __launch_bounds__(kBlock) void k_bricks_candidates(FuseArgs a, BrickArgs b) {
    const int64_t pix = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pix >= (int64_t)a.width * a.height) return;
    const int u = (int)(pix % a.width), v = (int)(pix / a.width);
    const double D = (double)a.depth[pix];
    if (!(isfinite(D) && D > 0.0)) return;
    const double z0 = fmax(D - a.tau, 0.0), z1 = D + a.tau;
    if (z0 > a.zfar) return;   // the segment lies beyond every voxel (and its footprint stays bounded)
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    const double org[3] = {a.ox, a.oy, a.oz};
    for (int c = 0; c < 8; ++c) {
        const double z = (c & 4) ? z1 : z0;
        const double x = ((double)u + ((c & 1) ? 0.5 : -0.5) - a.cx) / a.fx * z;
        const double y = ((double)v + ((c & 2) ? 0.5 : -0.5) - a.cy) / a.fy * z;
        for (int r = 0; r < 3; ++r) {
            const double p = a.t[r] + a.R[3 * r] * x + a.R[3 * r + 1] * y + a.R[3 * r + 2] * z;
            const double g = (p - org[r]) / a.vs;
            lo[r] = fmin(lo[r], g);
            hi[r] = fmax(hi[r], g);
        }
    }
    const int nv[3] = {a.d.nx, a.d.ny, a.d.nz};
    int b0[3], b1[3];
    for (int r = 0; r < 3; ++r) {
        const double l = ceil(lo[r] - kCandMargin), h = floor(hi[r] + kCandMargin);
        if (h < 0.0 || l > (double)(nv[r] - 1)) return;   // the segment misses the grid
        b0[r] = (int)fmax(l, 0.0) >> 3;
        b1[r] = (int)fmin(h, (double)(nv[r] - 1)) >> 3;
    }
    for (int bz = b0[2]; bz <= b1[2]; ++bz)
        for (int by = b0[1]; by <= b1[1]; ++by)
            for (int bx = b0[0]; bx <= b1[0]; ++bx) {
                const int64_t e = ((int64_t)bz * b.nby + by) * b.nbx + bx;
                if (b.index[e] == -1 && atomicCAS(&b.index[e], -1, kCandidate) == -1)
                    b.cand[atomicAdd(&b.hdr->ncand, 1)] = (int)e;
            }
}

// Gives a slot to every listed candidate that holds a voxel this frame puts in the band
// (-tau <= eta < tau: updated with phi < 1), and returns the others to -1. Persistent over the list;
// only the workgroup of a candidate touches its entry.
__global__ __launch_bounds__(kBlock) void k_bricks_mark(FuseArgs a, BrickArgs b) {
    const int nc = b.hdr->ncand;
    for (int c = blockIdx.x; c < nc; c += gridDim.x) {
        const int e_idx = b.cand[c];
        const int bx = e_idx % b.nbx, by = (e_idx / b.nbx) % b.nby, bz = e_idx / (b.nbx * b.nby);
        const int i0 = bx * kBrickEdge, j0 = by * kBrickEdge, k0 = bz * kBrickEdge;
        int band = 0;
        for (int e = threadIdx.x; e < kBrickVox; e += kBlock) {
            double phi;
            if (fuse_decide(a, i0 + (e & 7), j0 + ((e >> 3) & 7), k0 + (e >> 6), phi) && phi < 1.0) band = 1;
        }
        band = __syncthreads_or(band);
        if (threadIdx.x == 0) {
            int entry = -1;
            if (band) {
                const int slot = atomicAdd(&b.hdr->n, 1);
                if (slot < b.max_bricks) {
                    b.coords[slot] = make_int4(bx, by, bz, 0);
                    entry = slot;
                } else {
                    atomicOr(&b.hdr->overflow, 1);
                }
            }
            b.index[e_idx] = entry;
        }
    }
}

// Replica value of voxel (i, j, k) as a cell corner: from slot s < src_limit, +1 elsewhere.
template <int FMT>
__device__ inline typename Store<FMT>::T brick_voxel(const BrickArgs& b, const Dims& d, int i, int j, int k,
                                                     int src_limit) {
    using S = Store<FMT>;
    if (i >= d.nx || j >= d.ny || k >= d.nz) return S::cell(S::enc(1.0f));
    const int s2 = brick_slot(b, i >> 3, j >> 3, k >> 3);
    if (s2 < 0 || s2 >= src_limit) return S::cell(S::enc(1.0f));
    return S::cell(static_cast<const typename S::T*>(b.T)[((int64_t)s2 << 9) + brick_local(i, j, k)]);
}

// Cells of slots [begin, end), corners read from slots below src_limit (+1 elsewhere). With
// init, the slots' own T and W are first set to +1 and 0 (their corners read +1 either way).
template <int FMT, bool INIT>
__global__ __launch_bounds__(kBlock) void k_bricks_cells(BrickArgs b, Dims d, int first_new) {
    using S = Store<FMT>;
    const int n_now = min(b.hdr->n, b.max_bricks);
    const int begin = first_new ? b.hdr->n_prev : 0, src_limit = INIT ? b.hdr->n_prev : n_now;
    auto* T = static_cast<typename S::T*>(b.T);
    auto* W = static_cast<typename S::W*>(b.W);
    auto* C = static_cast<typename S::T*>(b.C);
    for (int slot = begin + blockIdx.x; slot < n_now; slot += gridDim.x) {
        const int4 c = b.coords[slot];
        for (int e = threadIdx.x; e < kBrickVox; e += kBlock) {
            if (INIT) {
                T[((int64_t)slot << 9) + e] = S::enc(1.0f);
                W[((int64_t)slot << 9) + e] = S::encw(0.0f);
            }
            const int i = c.x * kBrickEdge + (e & 7), j = c.y * kBrickEdge + ((e >> 3) & 7), k = c.z * kBrickEdge + (e >> 6);
            typename S::T* o = C + ((((int64_t)slot << 9) + e) << 3);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                o[q] = brick_voxel<FMT>(b, d, i + (q & 1), j + ((q >> 1) & 1), k + (q >> 2), src_limit);
        }
    }
}

// Writes voxel (i, j, k)'s replica value into every allocated cell that has it as a corner.
template <typename T>
__device__ inline void write_corners_bricks(const BrickArgs& b, const Dims& d, int i, int j, int k, T val) {
    T* C = static_cast<T*>(b.C);
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int ci = i - dx, cj = j - dy, ck = k - dz;
                if (ci < 0 || cj < 0 || ck < 0 || ci >= d.nx - 1 || cj >= d.ny - 1 || ck >= d.nz - 1) continue;
                const int s2 = brick_slot(b, ci >> 3, cj >> 3, ck >> 3);
                if (s2 < 0) continue;
                C[((((int64_t)s2 << 9) + brick_local(ci, cj, ck)) << 3) + (dx + 2 * dy + 4 * dz)] = val;
            }
}

// Fusion of every allocated brick (persistent over the slots in use).
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_bricks_integrate(FuseArgs a, BrickArgs b) {
    const int n_now = min(b.hdr->n, b.max_bricks);
    for (int slot = blockIdx.x; slot < n_now; slot += gridDim.x) {
        const int4 c = b.coords[slot];
        const int i0 = c.x * kBrickEdge, j0 = c.y * kBrickEdge, k0 = c.z * kBrickEdge;
        if (brick_outside(a, i0, j0, k0, i0 + 7, j0 + 7, k0 + 7)) continue;
        for (int e = threadIdx.x; e < kBrickVox; e += kBlock) {
            const int i = i0 + (e & 7), j = j0 + ((e >> 3) & 7), k = k0 + (e >> 6);
            double phi;
            if (!fuse_decide(a, i, j, k, phi)) continue;
            typename Store<FMT>::T told, tnew;
            if (fuse_apply<FMT>(a, ((int64_t)slot << 9) + e, phi, told, tnew))
                write_corners_bricks(b, a.d, i, j, k, Store<FMT>::cell(tnew));
        }
    }
}

// Rebuilds the cell-validity words of every slot in use from its cell blocks: bit (local & 63) of
// word (local >> 6) is set iff all 8 corners of the cell are in the band (the test of the scoring;
// a NaN-marked corner fails it). A wave covers 64 consecutive cells of a slot, so its ballot is a
// word.
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_bricks_mask(BrickArgs b) {
    using ST = typename Store<FMT>::T;
    const ST* C = static_cast<const ST*>(b.C);
    const int n_now = min(b.hdr->n, b.max_bricks);
    const int lane = threadIdx.x & (kWave - 1);
    for (int slot = blockIdx.x; slot < n_now; slot += gridDim.x) {
        for (int e = threadIdx.x; e < kBrickVox; e += kBlock) {
            float c[8];
            load_cell8<FMT>(C + ((((size_t)slot << 9) | (size_t)e) << 3), c);
            bool valid = true;
#pragma unroll
            for (int q = 0; q < 8; ++q) valid &= Fmt<FMT>::in_band(c[q]);
            const unsigned long long word = __ballot(valid);
            if (lane == 0) b.M[(size_t)slot * kBrickMaskWords + (e >> 6)] = word;
        }
    }
}

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_bricks_export(BrickArgs b, Dims d, float* To, float* Wo) {
    using S = Store<FMT>;
    const auto* T = static_cast<const typename S::T*>(b.T);
    const auto* W = static_cast<const typename S::W*>(b.W);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < d.n; v += stride) {
        const int i = (int)(v % d.nx), j = (int)((v / d.nx) % d.ny), k = (int)(v / ((int64_t)d.nx * d.ny));
        const int s2 = brick_slot(b, i >> 3, j >> 3, k >> 3);
        const int64_t e = ((int64_t)max(s2, 0) << 9) + brick_local(i, j, k);   // slot 0 always exists
        To[v] = s2 < 0 ? 1.0f : S::dec(T[e]);
        if (Wo) Wo[v] = s2 < 0 ? 0.0f : S::decw(W[e]);
    }
}

// Import: one workgroup per brick gives a slot to bricks holding any voxel other than
// (T, W) = (+1, 0), then the slots are filled from the linear arrays.
__global__ __launch_bounds__(kBlock) void k_bricks_import_mark(BrickArgs b, Dims d, const float* Ti, const float* Wi) {
    const int bx = blockIdx.x, by = blockIdx.y, bz = blockIdx.z;
    int need = 0;
    for (int e = threadIdx.x; e < kBrickVox; e += kBlock) {
        const int i = bx * kBrickEdge + (e & 7), j = by * kBrickEdge + ((e >> 3) & 7), k = bz * kBrickEdge + (e >> 6);
        const int64_t v = ((int64_t)k * d.ny + j) * d.nx + i;
        if (Ti[v] != 1.0f || (Wi && Wi[v] != 0.0f)) need = 1;
    }
    if (!__syncthreads_or(need)) return;
    if (threadIdx.x == 0) {
        const int slot = atomicAdd(&b.hdr->n, 1);
        if (slot < b.max_bricks) {
            b.coords[slot] = make_int4(bx, by, bz, 0);
            b.index[((int64_t)bz * b.nby + by) * b.nbx + bx] = slot;
        } else {
            atomicOr(&b.hdr->overflow, 1);
        }
    }
}

template <int FMT>
__global__ __launch_bounds__(kBlock) void k_bricks_import_fill(BrickArgs b, Dims d, const float* Ti, const float* Wi) {
    using S = Store<FMT>;
    auto* T = static_cast<typename S::T*>(b.T);
    auto* W = static_cast<typename S::W*>(b.W);
    const int n_now = min(b.hdr->n, b.max_bricks);
    for (int slot = blockIdx.x; slot < n_now; slot += gridDim.x) {
        const int4 c = b.coords[slot];
        for (int e = threadIdx.x; e < kBrickVox; e += kBlock) {
            const int i = c.x * kBrickEdge + (e & 7), j = c.y * kBrickEdge + ((e >> 3) & 7), k = c.z * kBrickEdge + (e >> 6);
            const int64_t v = ((int64_t)k * d.ny + j) * d.nx + i;
            T[((int64_t)slot << 9) + e] = S::enc(Ti[v]);
            W[((int64_t)slot << 9) + e] = S::encw(Wi ? Wi[v] : 0.0f);
        }
    }
}

constexpr int kBrickGrid = 4096;   // persistent workgroups over the slots

int grid_for(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < 65536 ? b : 65536);
}

void* cells_ptr(const pf_tsdf* v) {
    return v->layout == PF_LAYOUT_CELLS ? static_cast<char*>(v->tsdf) + cells_offset_bytes(v) : nullptr;
}

template <int FMT>
int32_t bricks_reset(const pf_tsdf* v, hipStream_t s) {
    const BrickArgs b = brick_args(v);
    const int64_t n_index = (int64_t)b.nbx * b.nby * b.nbz;
    hipLaunchKernelGGL(k_bricks_reset<FMT>, dim3(grid_for(n_index)), dim3(kBlock), 0, s, b, n_index);
    return check_launch("tsdf_init (bricks)");
}

template <int FMT>
int32_t init_t(const pf_tsdf* v, hipStream_t s) {
    if (v->layout == PF_LAYOUT_BRICKS) return bricks_reset<FMT>(v, s);
    const Dims d = dims_of(v);
    hipLaunchKernelGGL(k_init<FMT>, dim3(grid_for(d.n * 8)), dim3(kBlock), 0, s, v->tsdf, v->weight, cells_ptr(v), d,
                       mask_args(v));
    return check_launch("tsdf_init");
}

// The fields of a fusion that do not depend on the pose.
FuseArgs fuse_base(const pf_tsdf* v, const float* depth, const pf_intrinsics* K) {
    FuseArgs a;
    a.T = v->tsdf;
    a.W = v->weight;
    a.C = cells_ptr(v);
    a.m = mask_args(v);
    a.d = dims_of(v);
    a.vs = v->voxel_size;
    a.tau = v->trunc;
    a.ox = v->origin[0];
    a.oy = v->origin[1];
    a.oz = v->origin[2];
    a.fx = K->fx;
    a.fy = K->fy;
    a.cx = K->cx;
    a.cy = K->cy;
    a.width = K->width;
    a.height = K->height;
    a.w_max = (float)v->w_max;
    a.depth = depth;
    return a;
}

// The dense fusion's launches; ap != nullptr: the arguments (pose fields included) are read from
// that device copy instead of `a`.
template <int FMT>
int32_t integrate_dense(const pf_tsdf* v, const FuseArgs& a, const FuseArgs* ap, hipStream_t s) {
    const dim3 grid((unsigned)((a.d.nx + kFuseX - 1) / kFuseX), (unsigned)((a.d.ny + kFuseY - 1) / kFuseY),
                    (unsigned)((a.d.nz + kFuseZ - 1) / kFuseZ));
    if (ap)
        hipLaunchKernelGGL((k_integrate<FMT, true>), grid, dim3(kBlock), 0, s, a, ap);
    else
        hipLaunchKernelGGL((k_integrate<FMT, false>), grid, dim3(kBlock), 0, s, a, ap);
    if (v->layout == PF_LAYOUT_CELLS) {
        const int64_t words = (int64_t)a.m.mwx * a.m.mwy * a.m.mwz;
        hipLaunchKernelGGL(k_mask_update<FMT>, dim3(grid_for(words)), dim3(kBlock), 0, s, v->tsdf, a.d, a.m, 0);
    }
    return check_launch("tsdf_integrate");
}

template <int FMT>
int32_t integrate_t(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* P, hipStream_t s) {
    FuseArgs a = fuse_base(v, depth, K);
    fuse_pose_fields(a, P->R, P->t);
    if (v->layout == PF_LAYOUT_BRICKS) {
        const BrickArgs b = brick_args(v);
        a.T = b.T;
        a.W = b.W;
        a.C = nullptr;
        hipLaunchKernelGGL(k_bricks_prep, dim3(1), dim3(1), 0, s, b);
        const int64_t npix = (int64_t)a.width * a.height;
        hipLaunchKernelGGL(k_bricks_candidates, dim3((unsigned)((npix + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a, b);
        hipLaunchKernelGGL(k_bricks_mark, dim3(kBrickGrid), dim3(kBlock), 0, s, a, b);
        hipLaunchKernelGGL((k_bricks_cells<FMT, true>), dim3(kBrickGrid), dim3(kBlock), 0, s, b, a.d, 1);
        hipLaunchKernelGGL(k_bricks_integrate<FMT>, dim3(kBrickGrid), dim3(kBlock), 0, s, a, b);
        hipLaunchKernelGGL(k_bricks_mask<FMT>, dim3(kBrickGrid), dim3(kBlock), 0, s, b);
        return check_launch("tsdf_integrate (bricks)");
    }
    return integrate_dense<FMT>(v, a, nullptr, s);
}

template <int FMT>
int32_t integrate_at_t(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const double* R_dev,
                       const double* t_dev, void* args_dev, hipStream_t s) {
    const FuseArgs a = fuse_base(v, depth, K);
    FuseArgs* ap = static_cast<FuseArgs*>(args_dev);
    hipLaunchKernelGGL(k_fuse_pose, dim3(1), dim3(1), 0, s, ap, a, R_dev, t_dev);
    return integrate_dense<FMT>(v, a, ap, s);
}

template <int FMT>
int32_t export_t(const pf_tsdf* v, float* T, float* W, hipStream_t s) {
    const Dims d = dims_of(v);
    if (v->layout == PF_LAYOUT_BRICKS) {
        hipLaunchKernelGGL(k_bricks_export<FMT>, dim3(grid_for(d.n)), dim3(kBlock), 0, s, brick_args(v), d, T, W);
        return check_launch("tsdf_export_linear (bricks)");
    }
    hipLaunchKernelGGL(k_export<FMT>, dim3(grid_for(d.n)), dim3(kBlock), 0, s, v->tsdf, v->weight, d, T, W);
    return check_launch("tsdf_export_linear");
}

template <int FMT>
int32_t import_t(const pf_tsdf* v, const float* T, const float* W, hipStream_t s) {
    const Dims d = dims_of(v);
    if (v->layout == PF_LAYOUT_BRICKS) {
        int32_t rc = bricks_reset<FMT>(v, s);
        if (rc) return rc;
        const BrickArgs b = brick_args(v);
        hipLaunchKernelGGL(k_bricks_import_mark, dim3((unsigned)b.nbx, (unsigned)b.nby, (unsigned)b.nbz), dim3(kBlock),
                           0, s, b, d, T, W);
        hipLaunchKernelGGL(k_bricks_import_fill<FMT>, dim3(kBrickGrid), dim3(kBlock), 0, s, b, d, T, W);
        hipLaunchKernelGGL((k_bricks_cells<FMT, false>), dim3(kBrickGrid), dim3(kBlock), 0, s, b, d, 0);
        hipLaunchKernelGGL(k_bricks_mask<FMT>, dim3(kBrickGrid), dim3(kBlock), 0, s, b);
        return check_launch("tsdf_import_linear (bricks)");
    }
    hipLaunchKernelGGL(k_import<FMT>, dim3(grid_for(d.n)), dim3(kBlock), 0, s, v->tsdf, v->weight, d, T, W);
    int32_t rc = check_launch("tsdf_import_linear");
    if (rc || v->layout != PF_LAYOUT_CELLS) return rc;
    hipLaunchKernelGGL(k_build_cells<FMT>, dim3(grid_for(d.ncells)), dim3(kBlock), 0, s, v->tsdf, cells_ptr(v), d);
    const MaskArgs m = mask_args(v);
    const int64_t words = (int64_t)m.mwx * m.mwy * m.mwz;
    hipLaunchKernelGGL(k_mask_update<FMT>, dim3(grid_for(words)), dim3(kBlock), 0, s, v->tsdf, d, m, 1);
    return check_launch("tsdf_import_linear (cells)");
}

}  // namespace

int32_t launch_tsdf_init(const pf_tsdf* v, hipStream_t s) {
    switch (v->format) {
        case PF_F32_W_F32: return init_t<PF_F32_W_F32>(v, s);
        case PF_F16_W_U8: return init_t<PF_F16_W_U8>(v, s);
        case PF_I16_W_U8: return init_t<PF_I16_W_U8>(v, s);
        default: return set_error(PF_EUNSUPPORTED, "unsupported format %d", v->format);
    }
}

int32_t launch_tsdf_integrate(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* P,
                              hipStream_t s) {
    switch (v->format) {
        case PF_F32_W_F32: return integrate_t<PF_F32_W_F32>(v, depth, K, P, s);
        case PF_F16_W_U8: return integrate_t<PF_F16_W_U8>(v, depth, K, P, s);
        case PF_I16_W_U8: return integrate_t<PF_I16_W_U8>(v, depth, K, P, s);
        default: return set_error(PF_EUNSUPPORTED, "unsupported format %d", v->format);
    }
}

int32_t launch_tsdf_integrate_at(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const double* R_dev,
                                 const double* t_dev, void* args_dev, hipStream_t s) {
    if (v->layout == PF_LAYOUT_BRICKS)
        return set_error(PF_EUNSUPPORTED, "tsdf_integrate at a device pose: dense layouts only");
    switch (v->format) {
        case PF_F32_W_F32: return integrate_at_t<PF_F32_W_F32>(v, depth, K, R_dev, t_dev, args_dev, s);
        case PF_F16_W_U8: return integrate_at_t<PF_F16_W_U8>(v, depth, K, R_dev, t_dev, args_dev, s);
        case PF_I16_W_U8: return integrate_at_t<PF_I16_W_U8>(v, depth, K, R_dev, t_dev, args_dev, s);
        default: return set_error(PF_EUNSUPPORTED, "unsupported format %d", v->format);
    }
}

size_t fuse_args_bytes() { return sizeof(FuseArgs); }

int32_t launch_tsdf_export(const pf_tsdf* v, float* T, float* W, hipStream_t s) {
    switch (v->format) {
        case PF_F32_W_F32: return export_t<PF_F32_W_F32>(v, T, W, s);
        case PF_F16_W_U8: return export_t<PF_F16_W_U8>(v, T, W, s);
        case PF_I16_W_U8: return export_t<PF_I16_W_U8>(v, T, W, s);
        default: return set_error(PF_EUNSUPPORTED, "unsupported format %d", v->format);
    }
}

int32_t launch_tsdf_import(const pf_tsdf* v, const float* T, const float* W, hipStream_t s) {
    switch (v->format) {
        case PF_F32_W_F32: return import_t<PF_F32_W_F32>(v, T, W, s);
        case PF_F16_W_U8: return import_t<PF_F16_W_U8>(v, T, W, s);
        case PF_I16_W_U8: return import_t<PF_I16_W_U8>(v, T, W, s);
        default: return set_error(PF_EUNSUPPORTED, "unsupported format %d", v->format);
    }
}

}  // namespace pf
