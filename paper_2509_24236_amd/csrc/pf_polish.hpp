// Device bodies of the adjoint (Sec. III-B objective, differentiated with the valid set, the
// stencil cells and the signs frozen at the evaluated pose) and of the gradient polish, with the
// workgroup / problem index passed explicitly: the single-problem kernels and the batched kernels
// run the same code, so a batched problem's polish reproduces track_frame's bit for bit.
#pragma once

#include <math.h>

#include "pf_sample.hpp"

namespace pf {

struct GradPartial {
    FixSum sabs;     // sum |T|, exact (the scoring kernels' fixed point)
    float gt[3];     // sum s grad T          (translation part)
    float gr[3];     // sum (y - c) x s grad T (rotation part)
    float rmax;      // max |y - c| over all points of the chunk
    int cnt;
};

struct Partial2 {
    FixSum sum;
    int cnt;
    int pad;
};

// State of the on-device polish (lives in track_frame's workspace).
struct PolishState {
    double P[12];          // current pose, row-major [R | t]
    double cand[6][12];    // Armijo candidates alpha0 * 2^-h, h = 0..5
    double alpha[6];
    double E, gg;          // fitness and |grad|^2 at P
    int accepted, stop, best_k, pad;
};

constexpr int kGradThreads = 256;

__device__ inline void rows_to_pose(const double* P12, double R[9], double t[3]) {
    for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c) R[a * 3 + c] = P12[a * 4 + c];
        t[a] = P12[a * 4 + 3];
    }
}

__device__ inline void pose_to_rows(const double R[9], const double t[3], double* P12) {
    for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c) P12[a * 4 + c] = R[a * 3 + c];
        P12[a * 4 + 3] = t[a];
    }
}

// SO(3) left Jacobian J(phi) = I + (1 - cos th)/th^2 [phi]x + (th - sin th)/th^3 [phi]x^2, with the
// series 1/2 - th^2/24 and 1/6 - th^2/120 for small th.
__device__ inline void left_jacobian(const double w[3], double J[9]) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double a, b;
    if (th < 1e-4) {
        a = 0.5 - th2 / 24.0;
        b = 1.0 / 6.0 - th2 / 120.0;
    } else {
        double s, c;
        sincos(th, &s, &c);
        a = (1.0 - c) / th2;
        b = (th - s) / (th2 * th);
    }
    const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double k2 = 0.0;
            for (int m = 0; m < 3; ++m) k2 += K[r * 3 + m] * K[m * 3 + c];
            J[r * 3 + c] = (r == c ? 1.0 : 0.0) + a * K[r * 3 + c] + b * k2;
        }
}

// Accumulates E, the frozen-set gradient and the lever-arm maximum of one pose over points
// [q0, q1) into the thread's partial; pose_sh holds the FP32 pose, c the rotation centre. Each sample
// goes through the scoring kernels' own steps (eval_poses with one pose: cell, fraction, the in-grid
// test, the gather of the cell, the validity test, the trilinear value and its fixed-point |T|), so
// the exact |T| sum, the count and hence E are bitwise those of particles_score; the analytic
// gradient of the same interpolation is added alongside. No branch on validity: an invalid sample
// contributes zeros, and the next point is loaded while the current sample's gather is in flight.
template <int FMT, int LAYOUT>
__device__ inline void grad_accumulate(const VolView& vv, const float* __restrict__ px, const float* __restrict__ py,
                                       const float* __restrict__ pz, int q0, int q1, const float* pose_sh,
                                       const float c[3], GradPartial& acc) {
    using ST = typename Fmt<FMT>::T;
    const Gather<FMT, LAYOUT> G = make_gather<FMT, LAYOUT>(vv);
    const GridPose g = fold_pose(pose_sh, vv.inv_vs, vv.gx0, vv.gy0, vv.gz0);
    const unsigned lx = (unsigned)(vv.nx - 1), ly = (unsigned)(vv.ny - 1), lz = (unsigned)(vv.nz - 1);
    const float is = vv.inv_vs;
    constexpr bool kNanTest = LAYOUT != PF_LAYOUT_LINEAR && Fmt<FMT>::nan_cells;
    int q = q0 + (int)threadIdx.x;
    float X = 0.0f, Y = 0.0f, Z = 0.0f;
    if (q < q1) {
        X = px[q];
        Y = py[q];
        Z = pz[q];
    }
    for (; q < q1; q += kGradThreads) {
        const float x = X * is, y = Y * is, z = Z * is;
        const float Xc = X, Yc = Y, Zc = Z;
        if (q + kGradThreads < q1) {
            X = px[q + kGradThreads];
            Y = py[q + kGradThreads];
            Z = pz[q + kGradThreads];
        }
        const float gx = fmaf(g.r[0], x, fmaf(g.r[1], y, fmaf(g.r[2], z, g.t[0])));
        const float gy = fmaf(g.r[3], x, fmaf(g.r[4], y, fmaf(g.r[5], z, g.t[1])));
        const float gz = fmaf(g.r[6], x, fmaf(g.r[7], y, fmaf(g.r[8], z, g.t[2])));
        const unsigned ux = (unsigned)floor_to_int(gx), uy = (unsigned)floor_to_int(gy), uz = (unsigned)floor_to_int(gz);
        const bool inb = (ux < lx) & (uy < ly) & (uz < lz);
        const float fx = __builtin_amdgcn_fractf(gx), fy = __builtin_amdgcn_fractf(gy),
                    fz = __builtin_amdgcn_fractf(gz);
        const ST* p;
        if constexpr (LAYOUT == PF_LAYOUT_CELLS) {
            p = G.at(inb ? G.index(ux, uy, uz) : 0u);
        } else {
            p = G.addr((int)min(ux, lx - 1u), (int)min(uy, ly - 1u), (int)min(uz, lz - 1u));
        }
        float cv[8];
        G.load(p, cv);
        // lever arm u = y - c in metres: R x + t - c
        const float ux_m = fmaf(pose_sh[0], Xc, fmaf(pose_sh[1], Yc, fmaf(pose_sh[2], Zc, pose_sh[3] - c[0])));
        const float uy_m = fmaf(pose_sh[4], Xc, fmaf(pose_sh[5], Yc, fmaf(pose_sh[6], Zc, pose_sh[7] - c[1])));
        const float uz_m = fmaf(pose_sh[8], Xc, fmaf(pose_sh[9], Yc, fmaf(pose_sh[10], Zc, pose_sh[11] - c[2])));
        acc.rmax = fmaxf(acc.rmax, sqrtf(ux_m * ux_m + uy_m * uy_m + uz_m * uz_m));
        bool ok = inb;
        if constexpr (!kNanTest) {
#pragma unroll
            for (int e = 0; e < 8; ++e) ok &= Fmt<FMT>::in_band(cv[e]);
        }
        const float v = trilerp(fx, fy, fz, cv);
        if constexpr (kNanTest) ok &= !__builtin_isnan(v);
        acc.sabs += (FixSum)(ok ? fixed_point<FMT>(v) : 0u);
        acc.cnt += ok ? 1 : 0;
        // analytic gradient of the same interpolation, in grid units
        const float b0 = fmaf(fy, fmaf(fx, cv[3] - cv[2], cv[2]) - fmaf(fx, cv[1] - cv[0], cv[0]),
                              fmaf(fx, cv[1] - cv[0], cv[0]));
        const float b1 = fmaf(fy, fmaf(fx, cv[7] - cv[6], cv[6]) - fmaf(fx, cv[5] - cv[4], cv[4]),
                              fmaf(fx, cv[5] - cv[4], cv[4]));
        const float dx0 = fmaf(fy, (cv[3] - cv[2]) - (cv[1] - cv[0]), cv[1] - cv[0]);
        const float dx1 = fmaf(fy, (cv[7] - cv[6]) - (cv[5] - cv[4]), cv[5] - cv[4]);
        const float dTx = fmaf(fz, dx1 - dx0, dx0);
        const float dy0 = fmaf(fx, (cv[3] - cv[1]) - (cv[2] - cv[0]), cv[2] - cv[0]);
        const float dy1 = fmaf(fx, (cv[7] - cv[5]) - (cv[6] - cv[4]), cv[6] - cv[4]);
        const float dTy = fmaf(fz, dy1 - dy0, dy0);
        const float dTz = b1 - b0;
        // sign, times d(grid)/d(metre); zero for an invalid sample (its NaNs are selected away)
        const float s = !ok ? 0.0f : (v > 0.0f ? is : (v < 0.0f ? -is : 0.0f));
        const float wx = ok ? s * dTx : 0.0f, wy = ok ? s * dTy : 0.0f, wz = ok ? s * dTz : 0.0f;
        acc.gt[0] += wx;
        acc.gt[1] += wy;
        acc.gt[2] += wz;
        acc.gr[0] += uy_m * wz - uz_m * wy;
        acc.gr[1] += uz_m * wx - ux_m * wz;
        acc.gr[2] += ux_m * wy - uy_m * wx;
    }
}

// Fixed-order workgroup reduction of a GradPartial; thread 0 returns the total.
__device__ inline GradPartial grad_block_reduce(GradPartial a) {
    __shared__ float fs[7][kGradThreads / kWave];
    __shared__ FixSum ss[kGradThreads / kWave];
    __shared__ int cs[kGradThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    float v[6] = {a.gt[0], a.gt[1], a.gt[2], a.gr[0], a.gr[1], a.gr[2]};
    float m = a.rmax;
    FixSum sa = a.sabs;
    int c = a.cnt;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int e = 0; e < 6; ++e) v[e] += __shfl_xor(v[e], off);
        m = fmaxf(m, __shfl_xor(m, off));
        sa += __shfl_xor(sa, off);
        c += __shfl_xor(c, off);
    }
    if (lane == 0) {
        for (int e = 0; e < 6; ++e) fs[e][wid] = v[e];
        fs[6][wid] = m;
        ss[wid] = sa;
        cs[wid] = c;
    }
    __syncthreads();
    GradPartial r = {};
    if (threadIdx.x == 0) {
        for (int w = 0; w < kGradThreads / kWave; ++w) {
            r.sabs += ss[w];
            for (int e = 0; e < 3; ++e) {
                r.gt[e] += fs[e][w];
                r.gr[e] += fs[3 + e][w];
            }
            r.rmax = fmaxf(r.rmax, fs[6][w]);
            r.cnt += cs[w];
        }
    }
    return r;
}

// E (as the scoring kernels form it from the exact sum) and dE/dxi from the frozen-set sums:
// translation part g_t, rotation part g_r, then the chain through compose(xi, base) (left Jacobian
// of the rotation vector phi; LITERAL also couples rho).
template <int FMT>
__device__ inline void finish_gradient(const GradPartial& t, int mode, const double* xi, float* E_out,
                                       float* grad_out, int* nv_out) {
    if (t.cnt == 0) {
        *E_out = 1.0f;
        for (int e = 0; e < 6; ++e) grad_out[e] = 0.0f;
        if (nv_out) *nv_out = 0;
        return;
    }
    const float inv = Fmt<FMT>::scale / (float)t.cnt;
    *E_out = fitness_from<FMT>(t.sabs, t.cnt);
    double gt[3], gr[3];
    for (int e = 0; e < 3; ++e) {
        gt[e] = (double)(t.gt[e] * inv);
        gr[e] = (double)(t.gr[e] * inv);
    }
    if (xi) {
        const double rho[3] = {xi[0], xi[1], xi[2]};
        double J[9];
        left_jacobian(xi + 3, J);
        double w[3] = {gr[0], gr[1], gr[2]};
        if (mode == PF_COMPOSE_LITERAL) {
            w[0] -= rho[1] * gt[2] - rho[2] * gt[1];
            w[1] -= rho[2] * gt[0] - rho[0] * gt[2];
            w[2] -= rho[0] * gt[1] - rho[1] * gt[0];
        }
        for (int c = 0; c < 3; ++c) gr[c] = J[0 * 3 + c] * w[0] + J[1 * 3 + c] * w[1] + J[2 * 3 + c] * w[2];
    }
    for (int e = 0; e < 3; ++e) {
        grad_out[e] = (float)gt[e];
        grad_out[3 + e] = (float)gr[e];
    }
    if (nv_out) *nv_out = t.cnt;
}

// Pose b = compose(xi_b, base_b) in FP64; writes the FP32 pose and the rotation centre to LDS.
__device__ inline void setup_pose(const double* base12, const double* xi6, int mode, float* pose_sh, float* c_sh) {
    double R[9], t[3];
    rows_to_pose(base12, R, t);
    if (xi6) {
        double Ro[9], to[3];
        apply_delta(mode, xi6 + 3, xi6, R, t, Ro, to);
        for (int q = 0; q < 9; ++q) R[q] = Ro[q];
        for (int q = 0; q < 3; ++q) t[q] = to[q];
    }
    store_pose12(pose_sh, R, t);
    for (int a = 0; a < 3; ++a) c_sh[a] = mode == PF_COMPOSE_LITERAL ? 0.0f : (float)t[a];
}

// Pose b = compose(xi_b, base_b) on point chunk s of S: S == 1 finishes in place, otherwise the
// partial goes to partials[b * S + s].
template <int FMT, int LAYOUT>
__device__ inline void grad_step(const VolView& vv, const float* __restrict__ px, const float* __restrict__ py,
                                 const float* __restrict__ pz, int n, const double* __restrict__ base,
                                 const double* __restrict__ xi, int mode, float* E_out, float* grad_out, int* nv_out,
                                 GradPartial* partials, int b, int S, int s) {
    __shared__ float pose_sh[12];
    __shared__ float c_sh[3];
    if (threadIdx.x == 0) setup_pose(base + (size_t)b * 12, xi ? xi + (size_t)b * 6 : nullptr, mode, pose_sh, c_sh);
    __syncthreads();
    const float c[3] = {c_sh[0], c_sh[1], c_sh[2]};
    const int chunk = (n + S - 1) / S;
    const int q0 = s * chunk, q1 = min(n, q0 + chunk);
    GradPartial acc = {};
    grad_accumulate<FMT, LAYOUT>(vv, px, py, pz, q0, q1, pose_sh, c, acc);
    const GradPartial tot = grad_block_reduce(acc);
    if (threadIdx.x == 0) {
        if (partials)
            partials[(size_t)b * S + s] = tot;
        else
            finish_gradient<FMT>(tot, mode, xi ? xi + (size_t)b * 6 : nullptr, E_out + b, grad_out + (size_t)b * 6,
                                 nv_out ? nv_out + b : nullptr);
    }
    __syncthreads();
}

// Exact fitness partial of FP64 pose p (row-major [R | t]) on point chunk s of S. PRIO: the scoring
// loop's raised-priority window (left off by the batched kernels).
template <int FMT, int LAYOUT, bool PRIO = true>
__device__ inline void pose_partials_step(const VolView& vv, const float* __restrict__ px,
                                          const float* __restrict__ py, const float* __restrict__ pz, int n,
                                          const double* __restrict__ poses, Partial2* partials, int p, int S, int s) {
    __shared__ float pose_sh[12];
    if (threadIdx.x == 0) {
        double R[9], t[3];
        rows_to_pose(poses + (size_t)p * 12, R, t);
        store_pose12(pose_sh, R, t);
    }
    __syncthreads();
    const Gather<FMT, LAYOUT> G = make_gather<FMT, LAYOUT>(vv);
    GridPose g[1] = {fold_pose(pose_sh, vv.inv_vs, vv.gx0, vv.gy0, vv.gz0)};
    const unsigned lx = (unsigned)(vv.nx - 1), ly = (unsigned)(vv.ny - 1), lz = (unsigned)(vv.nz - 1);
    const int chunk = (n + S - 1) / S;
    const int q0 = s * chunk, q1 = min(n, q0 + chunk);
    FixSum sum[1] = {0};
    int cnt[1] = {0};
    const float sc = vv.inv_vs;
    for (int q = q0 + (int)threadIdx.x; q < q1; q += kGradThreads)
        eval_poses<FMT, LAYOUT, 1, false, false, false, PRIO>(G, lx, ly, lz, g, px[q] * sc, py[q] * sc, pz[q] * sc,
                                                             sum, cnt);
    block_reduce<1, kGradThreads>(sum, cnt);
    if (threadIdx.x == 0) {
        partials[(size_t)p * S + s].sum = sum[0];
        partials[(size_t)p * S + s].cnt = cnt[0];
    }
    __syncthreads();
}

template <int FMT>
__device__ inline float fitness_of(const Partial2* pt, int S, int* cnt_out) {
    FixSum sum = 0;
    int cnt = 0;
    for (int s = 0; s < S; ++s) {
        sum += pt[s].sum;
        cnt += pt[s].cnt;
    }
    if (cnt_out) *cnt_out = cnt;
    return fitness_from<FMT>(sum, cnt);
}

// Best candidate: the lowest fitness among P^(I) (E*) and the particles of iteration I (fit[1..K],
// deltas in the state around P^(I-1)); ties go to P^(I), then to the lowest k.
__device__ inline void best_step(pf_track_state* st, const float* __restrict__ fit, PolishState* ps) {
    const double* dl = reinterpret_cast<const double*>(reinterpret_cast<const char*>(st) + PF_STATE_DELTAS_OFFSET);
    const int K = st->K_cur;   // particles of the last iteration that ran
    float bv = INFINITY;
    int bk = K + 1;
    for (int k = 1 + threadIdx.x; k <= K; k += 256)
        if (fit[k] < bv) {
            bv = fit[k];
            bk = k;
        }
    __shared__ float sv[256];
    __shared__ int sk[256];
    sv[threadIdx.x] = bv;
    sk[threadIdx.x] = bk;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            const float ov = sv[threadIdx.x + off];
            const int ok = sk[threadIdx.x + off];
            if (ov < sv[threadIdx.x] || (ov == sv[threadIdx.x] && ok < sk[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                sk[threadIdx.x] = ok;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;   // one thread finishes; no barrier follows
    double R[9], t[3];
    if (sk[0] <= K && (double)sv[0] < st->Estar) {
        const int k = sk[0];
        double Rp[9], tp[3];
        for (int q = 0; q < 9; ++q) Rp[q] = st->R_prev[q];
        for (int q = 0; q < 3; ++q) tp[q] = st->t_prev[q];
        apply_delta(st->compose_mode, dl + 6 * k, dl + 6 * k + 3, Rp, tp, R, t);
        ps->best_k = k;
    } else {
        for (int q = 0; q < 9; ++q) R[q] = st->R[q];
        for (int q = 0; q < 3; ++q) t[q] = st->t[q];
        ps->best_k = 0;
    }
    pose_to_rows(R, t, ps->P);
    ps->accepted = 0;
    ps->stop = 0;
}

// From the gradient partials at P: E, grad, alpha0 = vs / (2 (|g_rho| + |g_phi| rmax)) and the
// six Armijo candidates compose(-alpha0 2^-h grad, P).
template <int FMT>
__device__ inline void polish_prep_step(PolishState* ps, const GradPartial* gp, int S, int mode, double vs) {
    if (ps->stop) return;
    GradPartial t = {};
    for (int s = 0; s < S; ++s) {
        t.sabs += gp[s].sabs;
        for (int e = 0; e < 3; ++e) {
            t.gt[e] += gp[s].gt[e];
            t.gr[e] += gp[s].gr[e];
        }
        t.rmax = fmaxf(t.rmax, gp[s].rmax);
        t.cnt += gp[s].cnt;
    }
    float E, g[6];
    int cnt;
    finish_gradient<FMT>(t, mode, nullptr, &E, g, &cnt);
    double nr = 0.0, nphi = 0.0;
    for (int e = 0; e < 3; ++e) {
        nr += (double)g[e] * g[e];
        nphi += (double)g[3 + e] * g[3 + e];
    }
    const double gg = nr + nphi;
    const double denom = sqrt(nr) + sqrt(nphi) * (double)t.rmax;
    if (cnt == 0 || !(denom > 0.0)) {
        ps->stop = 1;
        return;
    }
    ps->E = (double)E;
    ps->gg = gg;
    double R[9], tt[3];
    rows_to_pose(ps->P, R, tt);
    double alpha = 0.5 * vs / denom;
    for (int h = 0; h < 6; ++h) {
        double x[6];
        for (int e = 0; e < 6; ++e) x[e] = -alpha * (double)g[e];
        double Ro[9], to[3];
        apply_delta(mode, x + 3, x, R, tt, Ro, to);
        pose_to_rows(Ro, to, ps->cand[h]);
        ps->alpha[h] = alpha;
        alpha *= 0.5;
    }
}

// Accepts the first candidate with E_h <= E - 1e-4 alpha_h |grad|^2, else stops the polish.
template <int FMT>
__device__ inline void polish_pick_step(PolishState* ps, const Partial2* cp, int S) {
    if (ps->stop) return;
    for (int h = 0; h < 6; ++h) {
        const float Eh = fitness_of<FMT>(cp + (size_t)h * S, S, nullptr);
        if ((double)Eh <= ps->E - 1e-4 * ps->alpha[h] * ps->gg) {
            for (int q = 0; q < 12; ++q) ps->P[q] = ps->cand[h][q];
            ps->accepted += 1;
            return;
        }
    }
    ps->stop = 1;
}

// Writes the polished pose back as the state's current pose.
__device__ inline void polish_commit_step(PolishState* ps, pf_track_state* st) {
    double R[9], t[3];
    rows_to_pose(ps->P, R, t);
    for (int q = 0; q < 9; ++q) st->R[q] = R[q];
    for (int q = 0; q < 3; ++q) st->t[q] = t[q];
}

__device__ inline void state_pose_rows_step(const pf_track_state* st, double* P12) {
    // the state's current pose as FP64 rows
    double R[9], t[3];
    for (int q = 0; q < 9; ++q) R[q] = st->R[q];
    for (int q = 0; q < 3; ++q) t[q] = st->t[q];
    pose_to_rows(R, t, P12);
}

}  // namespace pf
