// Per-sample evaluation of the fitness equation (Sec. III-B) for the three storage formats and
// the two layouts, and the workgroup reduction of (sum, count) pairs. Shared by the scoring,
// update and gradient kernels so every path evaluates a pose identically.
//
// Sums of |T| are exact: each FP32 sample value is converted to a 32-bit fixed-point integer
// (2^-32 units of the normalised TSDF; 2^-17 stored units for int16) and added in 64-bit
// integers. Integer addition is associative, so a pose's fitness does not depend on how the
// points were split over lanes, waves, workgroups or launches: every launch shape, the batched
// path and the single-problem path give the same bits. The conversion error is below 2^-32 per
// sample, far under FP32 accumulation error.
#pragma once

#include <hip/hip_fp16.h>
#include <math.h>

#include "pf_internal.hpp"

namespace pf {

// Storage element of each format and its band test (|T| < 1 in stored units: the +1 sentinel
// of unobserved voxels, and its negative, fail it).
template <int FMT>
struct Fmt;

// `fix` maps a valid |value| (in stored units, always below the band limit) into [0, 2^32);
// `unfix` maps the fixed-point sum back to normalised TSDF units.
// `nan_cells`: the cell replica marks corners outside the band as NaN, so a sample is valid exactly
// when its interpolated value is a number (the x-fastest storage keeps the +1 sentinel).
template <>
struct Fmt<PF_F32_W_F32> {
    using T = float;
    static constexpr bool nan_cells = true;
    __device__ static inline float val(float a) { return a; }
    __device__ static inline bool in_band(float a) { return fabsf(a) < 1.0f; }
    static constexpr float scale = 1.0f;
    static constexpr float fix = 4294967296.0f;                  // 2^32
    static constexpr double unfix = 1.0 / 4294967296.0;
};

template <>
struct Fmt<PF_F16_W_U8> {
    using T = __half;
    static constexpr bool nan_cells = true;
    __device__ static inline float val(__half a) { return __half2float(a); }
    __device__ static inline bool in_band(float a) { return fabsf(a) < 1.0f; }
    static constexpr float scale = 1.0f;
    static constexpr float fix = 4294967296.0f;
    static constexpr double unfix = 1.0 / 4294967296.0;
};

template <>
struct Fmt<PF_I16_W_U8> {
    using T = int16_t;
    static constexpr bool nan_cells = false;
    __device__ static inline float val(int16_t a) { return (float)a; }
    __device__ static inline bool in_band(float a) { return fabsf(a) < 32767.0f; }
    static constexpr float scale = 1.0f / 32767.0f;
    static constexpr float fix = 131072.0f;                      // 2^17: 32767 * 2^17 < 2^32
    static constexpr double unfix = 1.0 / (131072.0 * 32767.0);
};

using FixSum = unsigned long long;

// Fixed-point value of a valid sample. Each lerp of the interpolation is one fused multiply-add
// with a fraction below 1, whose exact value lies between its two endpoints, so rounding keeps it
// there: |value| is at most the largest |corner|, below 1 (32767 stored units for int16), and the
// product with `fix` is at most (1 - 2^-24) 2^32 (32766 * 2^17), inside the unsigned range.
template <int FMT>
__device__ inline unsigned fixed_point(float v) {
    return (unsigned)(fabsf(v) * Fmt<FMT>::fix);
}

// E from an exact (sum, count) pair; E = 1 for an empty valid set.
template <int FMT>
__device__ inline float fitness_from(FixSum sum, int cnt) {
    return cnt > 0 ? (float)((double)sum * Fmt<FMT>::unfix / (double)cnt) : 1.0f;
}

// Gathers the 8 stencil corners of cell (cx, cy, cz) (already clamped into the grid) in the order
// (dx, dy, dz) = 000 100 010 110 001 101 011 111.
template <int FMT, int LAYOUT>
struct Gather;

template <int FMT>
struct Gather<FMT, PF_LAYOUT_LINEAR> {
    using ST = typename Fmt<FMT>::T;
    const ST* __restrict__ T;
    int nx, nxy;
    // (nx * ny < 2^24 for the dense layouts, so the products are full-rate 24-bit multiplies)
    __device__ inline const ST* addr(int cx, int cy, int cz) const {
        return T + (__umul24((unsigned)cz, (unsigned)nxy) + __umul24((unsigned)cy, (unsigned)nx) + (unsigned)cx);
    }
    __device__ inline void load(const ST* p, float (&c)[8]) const {
        c[0] = Fmt<FMT>::val(p[0]);
        c[1] = Fmt<FMT>::val(p[1]);
        c[2] = Fmt<FMT>::val(p[nx]);
        c[3] = Fmt<FMT>::val(p[nx + 1]);
        c[4] = Fmt<FMT>::val(p[nxy]);
        c[5] = Fmt<FMT>::val(p[nxy + 1]);
        c[6] = Fmt<FMT>::val(p[nxy + nx]);
        c[7] = Fmt<FMT>::val(p[nxy + nx + 1]);
    }
};

// The 8 corners of a cell stored as one aligned block (32 B in FP32, 16 B otherwise).
template <int FMT>
__device__ inline void load_cell8(const typename Fmt<FMT>::T* p, float (&c)[8]) {
    using ST = typename Fmt<FMT>::T;
    if constexpr (FMT == PF_F32_W_F32) {
        const float4 a = reinterpret_cast<const float4*>(p)[0];
        const float4 b = reinterpret_cast<const float4*>(p)[1];
        c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w;
        c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
    } else {
        const uint4 w = reinterpret_cast<const uint4*>(p)[0];
        const uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            ST lo, hi;
            const uint16_t l16 = (uint16_t)(q[e] & 0xffffu), h16 = (uint16_t)(q[e] >> 16);
            __builtin_memcpy(&lo, &l16, 2);
            __builtin_memcpy(&hi, &h16, 2);
            c[2 * e] = Fmt<FMT>::val(lo);
            c[2 * e + 1] = Fmt<FMT>::val(hi);
        }
    }
}

// a * b + c on 24-bit a and b (b uniform, in a scalar register), one full-rate instruction: the
// compiler forms such sums as two multiplies and a three-way add, one instruction more
__device__ inline unsigned mad_u24(unsigned a, unsigned b, unsigned c) {
    unsigned r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// Cell-major replica: the 8 corners of a cell are one aligned block.
template <int FMT>
struct Gather<FMT, PF_LAYOUT_CELLS> {
    using ST = typename Fmt<FMT>::T;
    const ST* __restrict__ C;   // cells
    int cnx, cnxy;              // (nx-1), (nx-1)*(ny-1)
    const unsigned long long* __restrict__ M;   // cell-validity mask: one word per 4x4x4 cells
    int mwx, mwxy;
    // cell index (below 2^31 for the dense layouts), unsigned so that its widening is a zero
    // extension and the address one shift-and-add; (nx - 1)(ny - 1) < 2^24 for the dense layouts, so
    // the products are 24-bit multiply-adds (full rate; a 32-bit multiply issues at a quarter rate)
    __device__ inline unsigned index(unsigned cx, unsigned cy, unsigned cz) const {
        return mad_u24(cz, (unsigned)cnxy, mad_u24(cy, (unsigned)cnx, cx));
    }
    __device__ inline const ST* at(unsigned idx) const { return C + ((size_t)idx << 3); }
    __device__ inline const ST* addr(int cx, int cy, int cz) const { return at(index(cx, cy, cz)); }
    // byte offset of a cell's block, for a replica that 32-bit offsets address (row and slice
    // strides in bytes below 2^24: 24-bit multiplies); the gather then adds it to the uniform base
    // in the load itself, with no 64-bit address arithmetic
    static constexpr unsigned kBlockShift = sizeof(ST) == 4 ? 5 : 4;
    unsigned rowb, sliceb;   // cnx, cnxy times the block's bytes (meaningful for such replicas only)
    // (the operands are 24-bit for any cell of such a replica; the result of a cell outside it is
    // not used)
    __device__ inline unsigned offset(unsigned cx, unsigned cy, unsigned cz) const {
        return mad_u24(cz, sliceb, mad_u24(cy, rowb, cx << kBlockShift));
    }
    __device__ inline const ST* at_offset(unsigned off) const {
        return reinterpret_cast<const ST*>(reinterpret_cast<const char*>(C) + off);
    }
    __device__ inline void load(const ST* p, float (&c)[8]) const { load_cell8<FMT>(p, c); }
    // the mask is below 2^28 bytes, so a 32-bit offset from the uniform base addresses a word
    __device__ inline const unsigned long long* mask_word(int cx, int cy, int cz) const {
        const unsigned w = __umul24((unsigned)(cz >> 2), (unsigned)mwxy) + __umul24((unsigned)(cy >> 2), (unsigned)mwx) +
                           (unsigned)(cx >> 2);
        return reinterpret_cast<const unsigned long long*>(reinterpret_cast<const char*>(M) + (w << 3));
    }
    __device__ static inline unsigned mask_bit(int cx, int cy, int cz) {
        return (unsigned)((cx & 3) | ((cy & 3) << 2) | ((cz & 3) << 4));
    }
    // the word's index for a cell of the grid (two 24-bit multiply-adds), and the word at an index
    __device__ inline unsigned mask_index(unsigned cx, unsigned cy, unsigned cz) const {
        return mad_u24(cz >> 2, (unsigned)mwxy, mad_u24(cy >> 2, (unsigned)mwx, cx >> 2));
    }
    __device__ inline unsigned long long mask_at(unsigned w) const {
        return *reinterpret_cast<const unsigned long long*>(reinterpret_cast<const char*>(M) + (w << 3));
    }
    // the same bit as a 64-bit shift amount, whose bits above the sixth the shift ignores, so z's
    // bits need no mask (one instruction fewer)
    __device__ static inline unsigned mask_shift(unsigned cx, unsigned cy, unsigned cz) {
        const unsigned xy = (cx & 3u) | ((cy << 2) & ~3u);
        return (xy & 15u) | ((cz << 4) & ~15u);
    }
};

// Sparse bricks: the brick-index grid names the slot of the cell's 8x8x8 brick, whose cell
// blocks are stored like the replica's; a cell of a brick without a slot reads a block of +1
// (outside the band, so the sample is not valid), as the dense layouts would.
template <int FMT>
struct Gather<FMT, PF_LAYOUT_BRICKS> {
    using ST = typename Fmt<FMT>::T;
    const ST* __restrict__ C;     // the slots' cells
    const ST* ones;               // one block of +1
    const int* __restrict__ idx;  // brick-index grid
    const unsigned long long* __restrict__ M;   // the slots' cell-validity words (8 per slot)
    int nbx, nbxy;
    // ((nx / 8)(ny / 8) < 2^24: 24-bit multiplies)
    __device__ inline int key(int cx, int cy, int cz) const {
        return (int)(__umul24((unsigned)(cz >> 3), (unsigned)nbxy) + __umul24((unsigned)(cy >> 3), (unsigned)nbx) +
                     (unsigned)(cx >> 3));
    }
    __device__ inline int slot(int k) const { return idx[k]; }
    __device__ static inline unsigned local(int cx, int cy, int cz) {
        return (unsigned)((cx & 7) | ((cy & 7) << 3) | ((cz & 7) << 6));
    }
    // a cell by its index in the pool (slot * 512 + local)
    __device__ inline const ST* at(unsigned cell) const { return C + ((size_t)cell << 3); }
    __device__ inline const ST* at(int s, int cx, int cy, int cz) const {
        const int local = (cx & 7) | ((cy & 7) << 3) | ((cz & 7) << 6);
        return s < 0 ? ones : C + ((((size_t)s << 9) | (size_t)local) << 3);
    }
    __device__ inline const ST* addr(int cx, int cy, int cz) const { return at(slot(key(cx, cy, cz)), cx, cy, cz); }
    __device__ inline void load(const ST* p, float (&c)[8]) const { load_cell8<FMT>(p, c); }
};

// Folds a float32 row-major 3x4 pose [R | t] into grid units: g = R (x / vs) + (t / vs + g0).
struct GridPose {
    float r[9];
    float t[3];
};

__device__ inline GridPose fold_pose(const float* P, float inv_vs, float gx0, float gy0, float gz0) {
    GridPose g;
    g.r[0] = P[0]; g.r[1] = P[1]; g.r[2] = P[2];
    g.r[3] = P[4]; g.r[4] = P[5]; g.r[5] = P[6];
    g.r[6] = P[8]; g.r[7] = P[9]; g.r[8] = P[10];
    g.t[0] = fmaf(P[3], inv_vs, gx0);
    g.t[1] = fmaf(P[7], inv_vs, gy0);
    g.t[2] = fmaf(P[11], inv_vs, gz0);
    return g;
}

// For the active lanes whose bit in `lanes` is set, `if_set`, else `if_clear` (one v_cndmask_b32 on
// the lane mask; opaque to the compiler, so it stays where it is written).
__device__ inline float select_lanes(unsigned long long lanes, float if_set, float if_clear) {
    float r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(lanes));
    return r;
}

// For the active lanes in `lanes`, a, else b (one v_cndmask_b32, which the compiler cannot turn into
// a branch around the computation of a).
__device__ inline unsigned select_u32(unsigned long long lanes, unsigned a, unsigned b) {
    unsigned r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(lanes));
    return r;
}

// Bit `bit` (only its low 6 bits count) of a 64-bit word, as 0 or 1.
__device__ inline unsigned word_bit(unsigned long long w, unsigned bit) {
    unsigned long long r;
    asm("v_lshrrev_b64 %0, %1, %2" : "=v"(r) : "v"(bit), "v"(w));
    return (unsigned)r & 1u;
}

// Whether cell (ux, uy, uz) (unsigned: a negative corner wraps to a large value) is inside the grid of
// cells below (lx, ly, lz); CUBIC (lx = ly = lz): one three-way maximum and one compare instead of
// three compares, the same answer.
template <bool CUBIC>
__device__ inline bool in_grid(unsigned ux, unsigned uy, unsigned uz, unsigned lx, unsigned ly, unsigned lz) {
    if constexpr (CUBIC)
        return max(ux, max(uy, uz)) < lx;
    else
        return (ux < lx) & (uy < ly) & (uz < lz);
}

// floor(x) as an int (v_cvt_flr_i32_f32; the compiler emits floor and convert separately). Values
// outside the int range only ever produce out-of-grid cells, which are clamped and rejected.
__device__ inline int floor_to_int(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// Trilinear interpolation of the 8 corners (order as in Gather) at fractions (f0, f1, f2): lerps
// along x, then y, then z, each as one fused multiply-add.
__device__ inline float trilerp(float f0, float f1, float f2, const float (&c)[8]) {
    const float a00 = fmaf(f0, c[1] - c[0], c[0]);
    const float a10 = fmaf(f0, c[3] - c[2], c[2]);
    const float a01 = fmaf(f0, c[5] - c[4], c[4]);
    const float a11 = fmaf(f0, c[7] - c[6], c[6]);
    const float b0 = fmaf(f1, a10 - a00, a00);
    const float b1 = fmaf(f1, a11 - a01, a01);
    return fmaf(f2, b1 - b0, b0);
}

// Evaluates one point (already divided by the voxel size) against NP poses in three phases:
// the cell of every pose, then all gathers, then validity and interpolation, so that the gathers
// of all poses are in flight together. The cell is clamped into the grid so every gather is in
// bounds, and an out-of-grid sample is rejected afterwards. Adds |value| (fixed point) and 1 to
// (sum[j], cnt[j]) for every valid sample.
//
// MASK (replica only): the cell-validity mask is read first, in one round of loads for all poses,
// and a cell block is gathered only for a sample whose cell the mask marks valid; the mask bit
// then stands in for the value test. Where most samples miss the band (a wide particle spread),
// this replaces most 32-byte gathers by reads of a mask that is 1/256 of the replica's size.
//
// NARROW (the caller checked narrow_grid): a cubic grid, so the in-grid test is one three-way
// maximum and one compare, whose replica 32-bit byte offsets address (no 64-bit address
// arithmetic). WAVE_COUNT: every lane of the wave calls together (uniform control flow; `active`
// false for a lane without a point), and cnt[j] grows by the number of the wave's valid samples in
// every lane (a scalar population count instead of a per-lane select and add).
//
// PRIO: the raised-priority window described below (the batched kernels leave it off).
template <int FMT, int LAYOUT, int NP, bool MASK = false, bool NARROW = false, bool WAVE_COUNT = false,
          bool PRIO = true>
__attribute__((always_inline))
__device__ inline void eval_poses(const Gather<FMT, LAYOUT>& G, unsigned lx, unsigned ly, unsigned lz,
                                  const GridPose (&g)[NP], float x, float y, float z, FixSum (&sum)[NP],
                                  int (&cnt)[NP], bool active = true) {
    static_assert(!MASK || LAYOUT == PF_LAYOUT_CELLS, "the mask exists for the replica only");
    using ST = typename Fmt<FMT>::T;
    const ST* p[NP];
    unsigned ci[NP];   // replica: cell index, compared instead of the 64-bit address
    float f[NP][3];
    bool inb[NP];
    unsigned long long minb[NP];   // WAVE_COUNT: the wave's lanes whose sample of pose j is in the grid
    const unsigned long long mact = WAVE_COUNT ? __builtin_amdgcn_ballot_w64(active) : 0ull;
    // The wave runs at a raised priority from its transforms until its gathers are issued, so that
    // its memory round starts before the other waves' interpolation takes the SIMD: -26 us per
    // frame on the headline sequence with the window around the gathers alone, -67 us more with
    // the transforms and cell arithmetic in it (balanced A/Bs). (In the batched kernels, whose
    // persistent workgroups take items of many problems, the window made a batch 3.5% slower.)
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
    int cl[NP][3];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const float gx = fmaf(g[j].r[0], x, fmaf(g[j].r[1], y, fmaf(g[j].r[2], z, g[j].t[0])));
        const float gy = fmaf(g[j].r[3], x, fmaf(g[j].r[4], y, fmaf(g[j].r[5], z, g[j].t[1])));
        const float gz = fmaf(g[j].r[6], x, fmaf(g[j].r[7], y, fmaf(g[j].r[8], z, g[j].t[2])));
        // lower corner and fraction: floor as an integer in one instruction, and x - floor(x), which
        // is exact in FP32, from the fract instruction
        const int ix = floor_to_int(gx), iy = floor_to_int(gy), iz = floor_to_int(gz);
        const unsigned ux = (unsigned)ix, uy = (unsigned)iy, uz = (unsigned)iz;
        inb[j] = in_grid<NARROW>(ux, uy, uz, lx, ly, lz);
        if constexpr (WAVE_COUNT) {
            minb[j] = __builtin_amdgcn_ballot_w64(inb[j]) & mact;
            inb[j] = inb[j] && active;
        }
        f[j][0] = __builtin_amdgcn_fractf(gx);
        f[j][1] = __builtin_amdgcn_fractf(gy);
        f[j][2] = __builtin_amdgcn_fractf(gz);
        if constexpr (LAYOUT == PF_LAYOUT_CELLS && !MASK && NARROW) {
            // (as below, by byte offset, formed for every lane and then selected)
            const unsigned off = G.offset(ux, uy, uz);
            ci[j] = inb[j] ? off : 0u;
            p[j] = G.at_offset(ci[j]);
        } else if constexpr (LAYOUT == PF_LAYOUT_CELLS && !MASK) {
            // a sample outside the grid (negative corners wrap to large values) reads cell 0
            // instead: the gather stays in bounds and the sample is rejected by inb
            ci[j] = inb[j] ? G.index(ux, uy, uz) : 0u;
            p[j] = G.at(ci[j]);
        } else {
            // any corner outside the grid is clamped to the last cell: the gather (and the mask
            // word) stay in bounds and the sample is rejected by inb
            const int cx = (int)min(ux, lx - 1u);
            const int cy = (int)min(uy, ly - 1u);
            const int cz = (int)min(uz, lz - 1u);
            cl[j][0] = cx;
            cl[j][1] = cy;
            cl[j][2] = cz;
            if constexpr (LAYOUT == PF_LAYOUT_CELLS) {
                ci[j] = G.index(cx, cy, cz);
                p[j] = G.at(ci[j]);
            } else if constexpr (LAYOUT == PF_LAYOUT_LINEAR) {
                p[j] = G.addr(cx, cy, cz);
            }
        }
    }
    if constexpr (LAYOUT == PF_LAYOUT_BRICKS) {
        // The brick of a cell comes from the index grid: a pose whose cell lies in the same brick
        // as the previous pose's takes that pose's slot instead of loading the entry again (the
        // same selection through an empty asm statement as for the corners below).
        int key[NP], slot[NP], kd[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) key[j] = G.key(cl[j][0], cl[j][1], cl[j][2]);
        slot[0] = G.slot(key[0]);
        kd[0] = 0;
#pragma unroll
        for (int j = 1; j < NP; ++j) {
            kd[j] = key[j] == key[j - 1] ? 1 : 0;
            slot[j] = -1;
            if (!kd[j]) slot[j] = G.slot(key[j]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 1; j < NP; ++j) {
            int d = kd[j];
            asm volatile("" : "+v"(d));
            slot[j] = d ? slot[j - 1] : slot[j];
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) p[j] = G.at(slot[j], cl[j][0], cl[j][1], cl[j][2]);
    }
    // keep the phases apart: the scheduler would otherwise interleave them pose by pose and
    // leave only one pose's gathers in flight
    __builtin_amdgcn_sched_barrier(0);
    // with the mask: whether each sample's cell is valid (a cell outside the grid was clamped onto
    // the last cell, whose bit may be set; such a sample is still rejected by inb)
    bool need[NP];
    if constexpr (MASK) {
        unsigned long long mw[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) mw[j] = *G.mask_word(cl[j][0], cl[j][1], cl[j][2]);
        __builtin_amdgcn_sched_barrier(0);
        // every bit is taken before the first gather is issued (an empty asm statement keeps the
        // tests out of the gathers' branches): a wait inside them would also wait for the gathers
        // already in flight
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            unsigned b = (unsigned)(mw[j] >> G.mask_bit(cl[j][0], cl[j][1], cl[j][2])) & 1u;
            asm volatile("" : "+v"(b));
            need[j] = b != 0;
        }
        __builtin_amdgcn_sched_barrier(0);
    } else {
#pragma unroll
        for (int j = 0; j < NP; ++j) need[j] = true;
    }
    // A pose that lands in the same cell as the previous pose reuses its corners instead of
    // gathering them again. Late in an optimization the search size has contracted so far that
    // neighbouring particles sample the same cells almost everywhere, and the loads of a whole
    // wavefront are then skipped; the values are identical either way.
    // The copy is made after all gathers were issued, by a lane select the compiler cannot see
    // through (select_lanes), so that it cannot fold the copy into the branch, where it would wait
    // for the previous pose's gather before issuing the next one.
    // (With the mask, a pose in the same cell as the previous one has the same bit, so the block it
    // copies was gathered whenever it needs one.)
    float c[NP][8];
    unsigned long long dup[NP];   // lanes whose pose j samples the same cell as pose j-1
    if (need[0]) G.load(p[0], c[0]);
#pragma unroll
    for (int j = 1; j < NP; ++j) {
        // (one compare: the lane mask of the lanes that differ, negated in scalar registers)
        bool nd;
        if constexpr (LAYOUT == PF_LAYOUT_CELLS)
            nd = ci[j] != ci[j - 1];
        else
            nd = p[j] != p[j - 1];
        dup[j] = ~__builtin_amdgcn_ballot_w64(nd);
        if (nd && need[j]) G.load(p[j], c[j]);
    }
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 1; j < NP; ++j)
#pragma unroll
        for (int q = 0; q < 8; ++q) c[j][q] = select_lanes(dup[j], c[j - 1][q], c[j][q]);
    // validity: with NaN-marked cells a NaN corner makes every step below NaN, so the value itself
    // says whether all 8 corners are in the band; otherwise each corner is tested
    constexpr bool kNanTest = !MASK && LAYOUT != PF_LAYOUT_LINEAR && Fmt<FMT>::nan_cells;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        bool ok = inb[j] & need[j];
        if constexpr (!kNanTest && !MASK) {
#pragma unroll
            for (int q = 0; q < 8; ++q) ok &= Fmt<FMT>::in_band(c[j][q]);
        }
        const float v = trilerp(f[j][0], f[j][1], f[j][2], c[j]);
        if constexpr (kNanTest) ok &= !__builtin_isnan(v);
        sum[j] += (FixSum)(ok ? fixed_point<FMT>(v) : 0u);
        if constexpr (WAVE_COUNT && kNanTest && !MASK)
            cnt[j] += __popcll(minb[j] & __builtin_amdgcn_ballot_w64(v == v));
        else if constexpr (WAVE_COUNT)
            cnt[j] += __popcll(__builtin_amdgcn_ballot_w64(ok));
        else
            cnt[j] += ok ? 1 : 0;
    }
}

// One pose against NQ points of the lane (act: the lane holds that point), each sample through
// eval_poses' own steps (the same transform, cell, fraction, in-grid test, gather, validity test,
// interpolation and fixed-point value, so the same bits), with the gathers of all NQ samples in
// flight together; sample q adds to (sum[q], cnt[q]).
template <int FMT, int LAYOUT, int NQ>
__attribute__((always_inline))
__device__ inline void eval_pose_points(const Gather<FMT, LAYOUT>& G, unsigned lx, unsigned ly, unsigned lz,
                                        const GridPose& g, const float (&x)[NQ], const float (&y)[NQ],
                                        const float (&z)[NQ], const bool (&act)[NQ], FixSum (&sum)[NQ],
                                        int (&cnt)[NQ]) {
    using ST = typename Fmt<FMT>::T;
    const ST* p[NQ];
    float f[NQ][3];
    bool inb[NQ];
    int cl[NQ][3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const float gx = fmaf(g.r[0], x[q], fmaf(g.r[1], y[q], fmaf(g.r[2], z[q], g.t[0])));
        const float gy = fmaf(g.r[3], x[q], fmaf(g.r[4], y[q], fmaf(g.r[5], z[q], g.t[1])));
        const float gz = fmaf(g.r[6], x[q], fmaf(g.r[7], y[q], fmaf(g.r[8], z[q], g.t[2])));
        const unsigned ux = (unsigned)floor_to_int(gx), uy = (unsigned)floor_to_int(gy), uz = (unsigned)floor_to_int(gz);
        inb[q] = act[q] & (ux < lx) & (uy < ly) & (uz < lz);
        f[q][0] = __builtin_amdgcn_fractf(gx);
        f[q][1] = __builtin_amdgcn_fractf(gy);
        f[q][2] = __builtin_amdgcn_fractf(gz);
        if constexpr (LAYOUT == PF_LAYOUT_CELLS) {
            p[q] = G.at(inb[q] ? G.index(ux, uy, uz) : 0u);
        } else {
            cl[q][0] = (int)min(ux, lx - 1u);
            cl[q][1] = (int)min(uy, ly - 1u);
            cl[q][2] = (int)min(uz, lz - 1u);
            if constexpr (LAYOUT == PF_LAYOUT_LINEAR) p[q] = G.addr(cl[q][0], cl[q][1], cl[q][2]);
        }
    }
    if constexpr (LAYOUT == PF_LAYOUT_BRICKS) {
        int slot[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) slot[q] = G.slot(G.key(cl[q][0], cl[q][1], cl[q][2]));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) p[q] = G.at(slot[q], cl[q][0], cl[q][1], cl[q][2]);
    }
    __builtin_amdgcn_sched_barrier(0);
    float c[NQ][8];
#pragma unroll
    for (int q = 0; q < NQ; ++q) G.load(p[q], c[q]);
    __builtin_amdgcn_sched_barrier(0);
    constexpr bool kNanTest = LAYOUT != PF_LAYOUT_LINEAR && Fmt<FMT>::nan_cells;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        bool ok = inb[q];
        if constexpr (!kNanTest) {
#pragma unroll
            for (int e = 0; e < 8; ++e) ok &= Fmt<FMT>::in_band(c[q][e]);
        }
        const float v = trilerp(f[q][0], f[q][1], f[q][2], c[q]);
        if constexpr (kNanTest) ok &= !__builtin_isnan(v);
        sum[q] += (FixSum)(ok ? fixed_point<FMT>(v) : 0u);
        cnt[q] += ok ? 1 : 0;
    }
}

// Workgroup reduction of TK exact (sum, count) pairs; thread j < TK returns pair j in s[0], c[0].
template <int TK, int BLOCK>
__device__ inline void block_reduce(FixSum (&s)[TK], int (&c)[TK]) {
    __shared__ FixSum ls[TK][BLOCK / kWave];
    __shared__ int lc[TK][BLOCK / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < TK; ++j) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            s[j] += __shfl_xor(s[j], off);
            c[j] += __shfl_xor(c[j], off);
        }
        if (lane == 0) {
            ls[j][wid] = s[j];
            lc[j][wid] = c[j];
        }
    }
    __syncthreads();
    if (threadIdx.x < TK) {
        const int j = threadIdx.x;
        FixSum a = 0;
        int b = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / kWave; ++w) {
            a += ls[j][w];
            b += lc[j][w];
        }
        s[0] = a;
        c[0] = b;
    }
}

// Volume accessor for a launch: the layout-specific gather and the cell limits.
template <int FMT, int LAYOUT>
__host__ __device__ inline Gather<FMT, LAYOUT> make_gather(const VolView& vv) {
    Gather<FMT, LAYOUT> G;
    if constexpr (LAYOUT == PF_LAYOUT_LINEAR) {
        G.T = static_cast<const typename Fmt<FMT>::T*>(vv.T);
        G.nx = vv.nx;
        G.nxy = vv.nx * vv.ny;
    } else if constexpr (LAYOUT == PF_LAYOUT_CELLS) {
        G.C = static_cast<const typename Fmt<FMT>::T*>(vv.cells);
        G.cnx = vv.nx - 1;
        G.cnxy = (vv.nx - 1) * (vv.ny - 1);
        G.rowb = (unsigned)G.cnx << Gather<FMT, LAYOUT>::kBlockShift;
        G.sliceb = (unsigned)G.cnxy << Gather<FMT, LAYOUT>::kBlockShift;
        G.M = vv.mask;
        G.mwx = vv.mwx;
        G.mwxy = vv.mwx * vv.mwy;
    } else {
        G.C = static_cast<const typename Fmt<FMT>::T*>(vv.cells);
        G.ones = static_cast<const typename Fmt<FMT>::T*>(vv.ones);
        G.idx = vv.bindex;
        G.M = vv.mask;
        G.nbx = vv.nbx;
        G.nbxy = vv.nbx * vv.nby;
    }
    return G;
}

}  // namespace pf
