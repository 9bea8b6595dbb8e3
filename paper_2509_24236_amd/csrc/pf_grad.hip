// Adjoint of the fitness equation (Sec. III-B) and the gradient polish of the tracked pose.
//
// The paper optimizes with particles only; the adjoint differentiates its fitness with the valid
// set, the stencil cells and the signs frozen at the evaluated pose. One gather pass yields E and
// its gradient: per valid sample, the 8 corners give the trilinear value and its analytic gradient
// (three differences of lerps), accumulated with the sign of the value and crossed with the lever
// arm from the rotation centre. The bodies live in pf_polish.hpp, shared with the batched path.
#include <math.h>

#include "pf_polish.hpp"

namespace pf {
namespace {

// grid (B, S): workgroup (b, s) handles pose b on point chunk s.
template <int FMT, int LAYOUT>
__global__ __launch_bounds__(kGradThreads) void k_grad(VolView vv, const float* __restrict__ px,
                                                       const float* __restrict__ py, const float* __restrict__ pz,
                                                       int n_host, const int* __restrict__ n_dev,
                                                       const double* __restrict__ base,
                                                       const double* __restrict__ xi, int mode, float* E_out,
                                                       float* grad_out, int* nv_out, GradPartial* partials) {
    grad_step<FMT, LAYOUT>(vv, px, py, pz, n_dev ? *n_dev : n_host, base, xi, mode, E_out, grad_out, nv_out, partials,
                           blockIdx.x, gridDim.y, blockIdx.y);
}

// grid (P, S): exact fitness partials of FP64 poses (row-major [R | t]) on point chunks.
template <int FMT, int LAYOUT>
__global__ __launch_bounds__(kGradThreads) void k_pose_partials(VolView vv, const float* __restrict__ px,
                                                                const float* __restrict__ py,
                                                                const float* __restrict__ pz, int n_host,
                                                                const int* __restrict__ n_dev,
                                                                const double* __restrict__ poses, const int* stop,
                                                                Partial2* partials) {
    if (stop && *stop) return;
    pose_partials_step<FMT, LAYOUT>(vv, px, py, pz, n_dev ? *n_dev : n_host, poses, partials, blockIdx.x, gridDim.y,
                                    blockIdx.y);
}

__global__ __launch_bounds__(256) void k_best(pf_track_state* st, const float* __restrict__ fit, PolishState* ps) {
    best_step(st, fit, ps);
}

template <int FMT>
__global__ void k_polish_prep(PolishState* ps, const GradPartial* gp, int S, int mode, double vs) {
    polish_prep_step<FMT>(ps, gp, S, mode, vs);
}

template <int FMT>
__global__ void k_polish_pick(PolishState* ps, const Partial2* cp, int S) {
    polish_pick_step<FMT>(ps, cp, S);
}

__global__ void k_polish_commit(PolishState* ps, pf_track_state* st) { polish_commit_step(ps, st); }

__global__ void k_state_pose_rows(const pf_track_state* st, double* P12) { state_pose_rows_step(st, P12); }

template <int FMT, int LAYOUT>
int32_t grad_t(const VolView& vv, const Points& p, const double* base, const double* xi, int B, int S, int mode,
               float* E, float* g, int* nv, GradPartial* partials, hipStream_t s) {
    hipLaunchKernelGGL((k_grad<FMT, LAYOUT>), dim3(B, S), dim3(kGradThreads), 0, s, vv, p.x, p.y, p.z, p.n, p.n_dev,
                       base, xi, mode, E, g, nv, partials);
    return check_launch("particles_score_grad");
}

template <int FMT, int LAYOUT>
int32_t pose_partials_t(const VolView& vv, const Points& p, const double* poses, int P, int S, const int* stop,
                        Partial2* out, hipStream_t s) {
    hipLaunchKernelGGL((k_pose_partials<FMT, LAYOUT>), dim3(P, S), dim3(kGradThreads), 0, s, vv, p.x, p.y, p.z, p.n,
                       p.n_dev, poses, stop, out);
    return check_launch("pose fitness");
}

}  // namespace

#define PF_DISPATCH(vv, FN, ...)                                                                 \
    return with_volume((vv).format, (vv).layout, [&](auto fmt_, auto layout_) {                      \
        return FN<decltype(fmt_)::value, decltype(layout_)::value>(__VA_ARGS__);                     \
    })

int32_t launch_grad(const VolView& vv, const Points& p, const double* base, const double* xi, int B, int S, int mode,
                    float* E, float* g, int* nv, GradPartial* partials, hipStream_t s) {
    PF_DISPATCH(vv, grad_t, vv, p, base, xi, B, S, mode, E, g, nv, partials, s);
}

int32_t launch_pose_partials(const VolView& vv, const Points& p, const double* poses, int P, int S, const int* stop,
                             Partial2* out, hipStream_t s) {
    PF_DISPATCH(vv, pose_partials_t, vv, p, poses, P, S, stop, out, s);
}

size_t polish_scratch_bytes(int S) {
    return ((sizeof(PolishState) + 255) & ~(size_t)255) + ((S * sizeof(GradPartial) + 255) & ~(size_t)255) +
           6 * S * sizeof(Partial2);
}

// Best candidate of iteration I, then `steps` polish steps on view p, then commit to the state.
int32_t launch_polish(const VolView& vv, const Points& p, int S, pf_track_state* st, int K, const float* fit,
                      int mode, double vs, int steps, void* scratch, hipStream_t s) {
    char* base = static_cast<char*>(scratch);
    PolishState* ps = reinterpret_cast<PolishState*>(base);
    double* ps_P = reinterpret_cast<double*>(base + offsetof(PolishState, P));
    double* ps_cand = reinterpret_cast<double*>(base + offsetof(PolishState, cand));
    int* ps_stop = reinterpret_cast<int*>(base + offsetof(PolishState, stop));
    GradPartial* gp = reinterpret_cast<GradPartial*>(base + ((sizeof(PolishState) + 255) & ~(size_t)255));
    Partial2* cp = reinterpret_cast<Partial2*>(reinterpret_cast<char*>(gp) + ((S * sizeof(GradPartial) + 255) & ~(size_t)255));
    hipLaunchKernelGGL(k_best, dim3(1), dim3(256), 0, s, st, fit, ps);
    int32_t rc = check_launch("polish");
    if (rc) return rc;
    for (int it = 0; it < steps; ++it) {
        // the gradient pass skips nothing when stopped, but its result is then ignored
        if ((rc = launch_grad(vv, p, ps_P, nullptr, 1, S, mode, nullptr, nullptr, nullptr, gp, s))) return rc;
        switch (vv.format) {
            case PF_F32_W_F32: hipLaunchKernelGGL(k_polish_prep<PF_F32_W_F32>, dim3(1), dim3(1), 0, s, ps, gp, S, mode, vs); break;
            case PF_F16_W_U8: hipLaunchKernelGGL(k_polish_prep<PF_F16_W_U8>, dim3(1), dim3(1), 0, s, ps, gp, S, mode, vs); break;
            default: hipLaunchKernelGGL(k_polish_prep<PF_I16_W_U8>, dim3(1), dim3(1), 0, s, ps, gp, S, mode, vs); break;
        }
        if ((rc = check_launch("polish"))) return rc;
        if ((rc = launch_pose_partials(vv, p, ps_cand, 6, S, ps_stop, cp, s))) return rc;
        switch (vv.format) {
            case PF_F32_W_F32: hipLaunchKernelGGL(k_polish_pick<PF_F32_W_F32>, dim3(1), dim3(1), 0, s, ps, cp, S); break;
            case PF_F16_W_U8: hipLaunchKernelGGL(k_polish_pick<PF_F16_W_U8>, dim3(1), dim3(1), 0, s, ps, cp, S); break;
            default: hipLaunchKernelGGL(k_polish_pick<PF_I16_W_U8>, dim3(1), dim3(1), 0, s, ps, cp, S); break;
        }
        if ((rc = check_launch("polish"))) return rc;
    }
    hipLaunchKernelGGL(k_polish_commit, dim3(1), dim3(1), 0, s, ps, st);
    return check_launch("polish");
}

int polish_accepted_offset() { return (int)offsetof(PolishState, accepted); }

template <int FMT>
__global__ void k_final_pose(const Partial2* pt, int S, float* E_out, int* n_out) {
    int cnt;
    *E_out = fitness_of<FMT>(pt, S, &cnt);
    *n_out = cnt;
}

// Fitness of the state's current pose on view p: pose rows and partials in `scratch`.
int32_t launch_state_fitness(const VolView& vv, const Points& p, int S, const pf_track_state* st, void* scratch,
                             float* E_out, int* n_out, hipStream_t s) {
    double* P12 = static_cast<double*>(scratch);
    Partial2* pt = reinterpret_cast<Partial2*>(static_cast<char*>(scratch) + 256);
    hipLaunchKernelGGL(k_state_pose_rows, dim3(1), dim3(1), 0, s, st, P12);
    int32_t rc = check_launch("final pose");
    if (rc) return rc;
    if ((rc = launch_pose_partials(vv, p, P12, 1, S, nullptr, pt, s))) return rc;
    switch (vv.format) {
        case PF_F32_W_F32: hipLaunchKernelGGL(k_final_pose<PF_F32_W_F32>, dim3(1), dim3(1), 0, s, pt, S, E_out, n_out); break;
        case PF_F16_W_U8: hipLaunchKernelGGL(k_final_pose<PF_F16_W_U8>, dim3(1), dim3(1), 0, s, pt, S, E_out, n_out); break;
        default: hipLaunchKernelGGL(k_final_pose<PF_I16_W_U8>, dim3(1), dim3(1), 0, s, pt, S, E_out, n_out); break;
    }
    return check_launch("final pose");
}

}  // namespace pf
