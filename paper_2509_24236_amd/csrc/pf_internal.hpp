// Internal declarations of the gfx950 library: device helpers shared by the kernels and the
// launchers the C ABI calls. Nothing here is part of the public ABI (include/profusion.h).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/profusion.h"

namespace pf {

constexpr int kWave = 64;

// ------------------------------------------------------------------ error plumbing (pf_capi.hip)
int32_t set_error(int32_t code, const char* fmt, ...);
int32_t check_launch(const char* what);

// ------------------------------------------------------------------ device helpers
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): n-th output of the generator whose state
// starts at `seed` is mix(seed + (n + 1) * 0x9E3779B97F4A7C15).
__device__ __host__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t n) {
    uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Draw for (frame t, iteration i, particle k, dimension d): counter t<<40 | i<<32 | k<<3 | d,
// top 53 bits scaled to [0, 1), then 2u - 1 in [-1, 1); every step is exact in FP64.
__device__ inline double draw_pm1(uint64_t seed, uint32_t t, uint32_t i, uint32_t k, uint32_t d) {
    uint64_t n = ((uint64_t)t << 40) | ((uint64_t)i << 32) | ((uint64_t)k << 3) | (uint64_t)d;
    uint64_t x = splitmix64_at(seed, n);
    double u = (double)(x >> 11) * 0x1.0p-53;
    return 2.0 * u - 1.0;
}

// The FP64 pose functions below round every multiplication and addition on its own, in source
// order (no fused multiply-add): with contraction the compiler may fuse them differently wherever
// they are inlined, and every kernel that draws or composes a pose (the separate draw launch, the
// particle launch that draws its own particles, the update step, the batched kernels, the polish)
// must get the same bits from the same inputs.
//
// Rotation matrix of a rotation vector w (radians), row-major: I + a [w]x + b [w]x^2 with
// a = sin(th)/th and b = (1 - cos th)/th^2, series a = 1 - th^2/6, b = 1/2 - th^2/24 below 1e-6.
__device__ inline void rotvec_to_matrix(const double w[3], double M[9]) {
#pragma clang fp contract(off)
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double a, b;
    if (th < 1e-6) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
    } else {
        double s, c;
        sincos(th, &s, &c);
        a = s / th;
        b = (1.0 - c) / th2;
    }
    // [w]x^2 = w w^T - th^2 I
    M[0] = 1.0 + b * (w[0] * w[0] - th2);
    M[4] = 1.0 + b * (w[1] * w[1] - th2);
    M[8] = 1.0 + b * (w[2] * w[2] - th2);
    M[1] = -a * w[2] + b * w[0] * w[1];
    M[3] = a * w[2] + b * w[0] * w[1];
    M[2] = a * w[1] + b * w[0] * w[2];
    M[6] = -a * w[1] + b * w[0] * w[2];
    M[5] = -a * w[0] + b * w[1] * w[2];
    M[7] = a * w[0] + b * w[1] * w[2];
}

// Delta pose (rotation vector r, translation tau) applied to (R, t); see PF_COMPOSE_*.
__device__ inline void apply_delta(int mode, const double r[3], const double tau[3], const double R[9],
                                   const double t[3], double Ro[9], double to[3]) {
#pragma clang fp contract(off)
    double D[9];
    rotvec_to_matrix(r, D);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Ro[a * 3 + b] = D[a * 3 + 0] * R[0 * 3 + b] + D[a * 3 + 1] * R[1 * 3 + b] + D[a * 3 + 2] * R[2 * 3 + b];
    if (mode == PF_COMPOSE_LITERAL) {
        for (int a = 0; a < 3; ++a) to[a] = D[a * 3 + 0] * t[0] + D[a * 3 + 1] * t[1] + D[a * 3 + 2] * t[2] + tau[a];
    } else {
        for (int a = 0; a < 3; ++a) to[a] = t[a] + tau[a];
    }
}

__device__ inline void store_pose12(float* dst, const double R[9], const double t[3]) {
    dst[0] = (float)R[0]; dst[1] = (float)R[1]; dst[2] = (float)R[2];  dst[3] = (float)t[0];
    dst[4] = (float)R[3]; dst[5] = (float)R[4]; dst[6] = (float)R[5];  dst[7] = (float)t[1];
    dst[8] = (float)R[6]; dst[9] = (float)R[7]; dst[10] = (float)R[8]; dst[11] = (float)t[2];
}

// ------------------------------------------------------------------ volume view for kernels
struct VolView {
    const void* T;       // x-fastest storage (dense layouts) or the slots' T (BRICKS)
    const void* cells;   // cell-major replica (PF_LAYOUT_CELLS) or the slots' cells (BRICKS), else nullptr
    const int* bindex;   // BRICKS: brick-index grid, else nullptr
    const unsigned long long* mask;   // CELLS: cell-validity words (4x4x4 cells each), else nullptr
    int mwx, mwy;        // CELLS: mask words along x and y
    const void* ones;    // BRICKS: one cell block of +1 (read for cells of bricks without a slot)
    int nbx, nby;        // BRICKS: bricks along x and y
    int nx, ny, nz, format, layout;
    float inv_vs;        // 1 / voxel_size
    float gx0, gy0, gz0; // -origin / voxel_size: grid coordinate of the world origin
};

VolView make_view(const pf_tsdf* v);

// Whether the scoring launches may take their narrow form for this volume (one instantiation each
// way, chosen at launch): a cubic grid (the in-grid test is one three-way maximum and a compare)
// and, for the cell replica, blocks that 32-bit byte offsets address, with row and slice strides
// below 2^24 bytes (24-bit multiplies). A 512^3 FP32 replica (511^3 blocks of 32 B) just fits.
inline bool narrow_grid(const VolView& v) {
    if (v.nx != v.ny || v.ny != v.nz) return false;
    if (v.layout != PF_LAYOUT_CELLS) return true;
    const uint64_t block = v.format == PF_F32_W_F32 ? 32 : 16, c = (uint64_t)(v.nx - 1);
    return c * c * c * block <= (1ull << 32) && c * c * block < (1ull << 24);
}

// Cell-validity mask of a CELLS T buffer: after the replica, one 64-bit word per block of 4x4x4
// cells (bit (x&3) + 4 (y&3) + 16 (z&3) of word ((z/4) mwy + y/4) mwx + x/4 is set iff all 8
// corners of cell (x, y, z) are in the band), then one byte per word that fusion sets when a
// voxel of the word's cells enters or leaves the band (the word is rebuilt and the byte cleared
// right after).
struct CellMask {
    int mwx, mwy, mwz;
    size_t words;
    size_t mask, flags, t_total;   // byte offsets from v->tsdf, and the whole T buffer (a multiple of 256)
};
CellMask cell_mask_layout(const pf_tsdf* v);

// Byte layout of a BRICKS T buffer (offsets from v->tsdf) and of its W buffer.
constexpr int kBrickEdge = 8, kBrickVox = 512;
struct BrickLayout {
    int nbx, nby, nbz;
    size_t index, cand, coords, pool_t, pool_cells, pool_mask, t_total, w_total;
};
constexpr int kBrickMaskWords = 8;   // cell-validity words per slot: 64 cells (local 64w .. 64w+63) each
constexpr int kMaxBricks = 1 << 23;  // slots: a pool cell's index (slot * 512 + local) fits 32 bits
BrickLayout brick_layout(const pf_tsdf* v);

// Header at the start of a BRICKS T buffer; a cell block of +1 follows at kBrickOnes.
struct BrickHeader {
    int n;          // slots in use
    int overflow;   // 1 once an allocation found the pool full
    int n_prev;     // slots in use before the current fusion
    int ncand;      // bricks listed as candidates by the current fusion
};
constexpr size_t kBrickOnes = 64;

// Calls fn(fmt, layout) with the volume's format and layout as std::integral_constant values,
// so one generic lambda reaches the kernel instantiation of every supported pair.
template <int V>
using IC = std::integral_constant<int, V>;

template <int FMT, typename Fn>
inline int32_t with_layout(int layout, Fn&& fn) {
    switch (layout) {
        case PF_LAYOUT_LINEAR: return fn(IC<FMT>{}, IC<PF_LAYOUT_LINEAR>{});
        case PF_LAYOUT_CELLS: return fn(IC<FMT>{}, IC<PF_LAYOUT_CELLS>{});
        case PF_LAYOUT_BRICKS: return fn(IC<FMT>{}, IC<PF_LAYOUT_BRICKS>{});
        default: return set_error(PF_EUNSUPPORTED, "unsupported layout %d", layout);
    }
}

template <typename Fn>
inline int32_t with_volume(int format, int layout, Fn&& fn) {
    switch (format) {
        case PF_F32_W_F32: return with_layout<PF_F32_W_F32>(layout, fn);
        case PF_F16_W_U8: return with_layout<PF_F16_W_U8>(layout, fn);
        case PF_I16_W_U8: return with_layout<PF_I16_W_U8>(layout, fn);
        default: return set_error(PF_EUNSUPPORTED, "unsupported format %d", format);
    }
}

// Element size of T and W for a format, and the byte offset of the cell replica in the T buffer.
size_t t_elem_bytes(int format);
size_t cells_offset_bytes(const pf_tsdf* v);

// Per-lane point block used by the scoring launchers: SoA camera coordinates.
struct Points {
    const float* x;
    const float* y;
    const float* z;
    int n;              // used when n_dev == nullptr
    const int* n_dev;   // device count (track_frame's compacted views)
};

// ------------------------------------------------------------------ launchers
int32_t launch_tsdf_init(const pf_tsdf* v, hipStream_t s);
int32_t launch_tsdf_integrate(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* P,
                              hipStream_t s);
// Dense layouts: the same fusion at the camera pose R_dev [9], t_dev [3] (FP64, device memory,
// e.g. the tracker's state), without the pose passing through the host; args_dev: device scratch of
// fuse_args_bytes() bytes (the arguments the kernels read). PF_EUNSUPPORTED for BRICKS.
int32_t launch_tsdf_integrate_at(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const double* R_dev,
                                 const double* t_dev, void* args_dev, hipStream_t s);
size_t fuse_args_bytes();
int32_t launch_tsdf_export(const pf_tsdf* v, float* T, float* W, hipStream_t s);
int32_t launch_tsdf_import(const pf_tsdf* v, const float* T, const float* W, hipStream_t s);

// Scores poses [K][12] (camera -> world float32) into fitness / n_valid. With an optimizer state,
// the launch shape follows the spread of the search size that drew the poses.
int32_t launch_score(const VolView& vv, const Points& p, const float* poses, int K, float* fitness, int* n_valid,
                     hipStream_t s, const pf_track_state* st = nullptr, int expect = -1);
// Spread regime (0 wide, 1 mid, 2 tight) of particles drawn with search size (s_rad, s_m): the
// host-side twin of the test the scoring launches make on the device.
int spread_regime_of(double s_rad, double s_m, float inv_vs);
// Whether the automatic launch for the K particles of an optimizer state has 4 poses x 256 threads
// per workgroup (the shape of the particle launch that draws its own particles), and whether a
// launch of spread regime `regime` reads the cell-validity mask of a volume of this layout.
bool score_auto_4x256(int K);
bool score_regime_masked(int layout, int regime);

// Largest number of per-workgroup partial sums the single-pose passes use.
constexpr int kMaxPartials = 256;

// Adjoint and polish (pf_grad.hip).
struct GradPartial;
int32_t launch_grad(const VolView& vv, const Points& p, const double* base, const double* xi, int B, int S, int mode,
                    float* E, float* g, int* nv, GradPartial* partials, hipStream_t s);
size_t polish_scratch_bytes(int S);
int polish_accepted_offset();
int32_t launch_polish(const VolView& vv, const Points& p, int S, pf_track_state* st, int K, const float* fit,
                      int mode, double vs, int steps, void* scratch, hipStream_t s);
int32_t launch_state_fitness(const VolView& vv, const Points& p, int S, const pf_track_state* st, void* scratch,
                             float* E_out, int* n_out, hipStream_t s);

int32_t launch_backproject(const float* depth, const pf_intrinsics* K, int stride, float* px, float* py, float* pz,
                           int* n_out, int* block_counts, hipStream_t s, int* pix = nullptr,
                           unsigned long long* masks = nullptr, int n_masks = 0);
size_t backproject_scratch_ints(const pf_intrinsics* K);

}  // namespace pf
