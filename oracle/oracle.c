/*
 * FP64 CPU oracle for PROFusion's tracking-and-fusion hot path (arXiv 2509.24236).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the HIP library is
 * checked against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no code, header, table or helper with the HIP library, and the HIP
 * library never calls it.
 *
 * Everything is double precision, built with -O2 -ffp-contract=off and no fast-math. The only
 * parallelism is OpenMP over independent particles or independent z-slabs of the volume, which
 * does not change any arithmetic. Each function names the passage of the paper it follows.
 *
 * Readings of passages the paper leaves open are listed where they are used (pose direction,
 * the meaning of "Delta P * P", the sampling box, the valid-grid rule, empty sets, the SO(3)
 * average, and the order of the search-size update).
 *
 * Volume storage: T[(k*ny + j)*nx + i] and W[...] for voxel (i, j, k) whose centre is
 * origin + vs*(i, j, k). T is the normalised TSDF (sdf / tau, so the 1/tau of the fitness
 * equation is folded into storage); T = +1 means unobserved or free beyond the band.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double R[9]; double t[3]; } orc_pose;            /* camera -> world */
typedef struct { double fx, fy, cx, cy; int32_t width, height; } orc_intr;
typedef struct {
    int32_t nx, ny, nz, w_max;
    double vs, tau;
    double origin[3];
    double* T;
    double* W;
} orc_vol;

/* Threads the OpenMP loops of this oracle use (1 without OpenMP). */
int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the threads of later OpenMP loops (for timing on one core); no effect without OpenMP. */
void orc_set_num_threads(int32_t n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* ----------------------------------------------------------------------------------------
 * Counter-based random numbers (reading: the paper does not name a generator).
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the n-th output (n = 0, 1, ...) of the
 * generator whose state starts at `seed` is mix(seed + (n + 1) * gamma), with
 * gamma = 0x9E3779B97F4A7C15 and the mix of the published reference implementation.
 * ---------------------------------------------------------------------------------------- */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n) {
    uint64_t z = seed + (n + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* The draw for (frame t, iteration i, particle k, dimension d) uses counter
 * n = t<<40 | i<<32 | k<<3 | d, and maps the top 53 bits to a in [-1, 1): a = 2u - 1,
 * u = (x >> 11) * 2^-53. Both steps are exact in double precision. */
uint64_t orc_counter(int64_t t, int64_t i, int64_t k, int64_t d) {
    return ((uint64_t)t << 40) | ((uint64_t)i << 32) | ((uint64_t)k << 3) | (uint64_t)d;
}

double orc_uniform_pm1(uint64_t seed, int64_t t, int64_t i, int64_t k, int64_t d) {
    uint64_t x = orc_splitmix64(seed, orc_counter(t, i, k, d));
    double u = (double)(x >> 11) * 0x1.0p-53;
    return 2.0 * u - 1.0;
}

/* ----------------------------------------------------------------------------------------
 * SO(3) exponential (Rodrigues) and logarithm. The paper averages rotations "in SO(3)"
 * (Sec. III-B); the exponential maps rotation vectors (radians) to matrices.
 * R = I + A K + B K^2 with K = [r]x, A = sin(th)/th, B = (1 - cos(th))/th^2, and the Taylor
 * forms A = 1 - th^2/6, B = 1/2 - th^2/24 for th < 1e-6.
 * ---------------------------------------------------------------------------------------- */
void orc_so3_exp(const double r[3], double R[9]) {
    double th2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double th = sqrt(th2);
    double A, B;
    if (th < 1e-6) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
    }
    double K[9] = {0.0, -r[2], r[1], r[2], 0.0, -r[0], -r[1], r[0], 0.0};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double k2 = 0.0;
            for (int c = 0; c < 3; ++c) k2 += K[a * 3 + c] * K[c * 3 + b];
            R[a * 3 + b] = (a == b ? 1.0 : 0.0) + A * K[a * 3 + b] + B * k2;
        }
}

/* Logarithm: th = acos((tr R - 1)/2); r = th / (2 sin th) * vee(R - R^T); near th = 0 the
 * factor tends to 1/2; near th = pi the axis comes from the diagonal of (R + I)/2. */
void orc_so3_log(const double R[9], double r[3]) {
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double th = acos(c);
    double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    if (th < 1e-7) {
        for (int a = 0; a < 3; ++a) r[a] = 0.5 * v[a];
        return;
    }
    if (M_PI - th < 1e-6) {
        double d[3] = {sqrt(fmax(0.0, 0.5 * (R[0] + 1.0))), sqrt(fmax(0.0, 0.5 * (R[4] + 1.0))),
                       sqrt(fmax(0.0, 0.5 * (R[8] + 1.0)))};
        int m = (d[0] >= d[1] && d[0] >= d[2]) ? 0 : (d[1] >= d[2] ? 1 : 2);
        double ax[3];
        ax[m] = d[m];
        for (int a = 0; a < 3; ++a)
            if (a != m) ax[a] = 0.5 * R[m * 3 + a] / d[m];   /* (R + R^T)/2 off-diagonal = ax_m ax_a */
        double n = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
        for (int a = 0; a < 3; ++a) r[a] = th * ax[a] / n;
        return;
    }
    double f = th / (2.0 * sin(th));
    for (int a = 0; a < 3; ++a) r[a] = f * v[a];
}

static void mat3_mul(const double A[9], const double B[9], double C[9]) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += A[a * 3 + c] * B[c * 3 + b];
            C[a * 3 + b] = s;
        }
}

static void mat3_vec(const double A[9], const double x[3], double y[3]) {
    for (int a = 0; a < 3; ++a) y[a] = A[a * 3 + 0] * x[0] + A[a * 3 + 1] * x[1] + A[a * 3 + 2] * x[2];
}

/* ----------------------------------------------------------------------------------------
 * Delta-pose composition "Delta P_k P^(i-1)" (Sec. III-B).
 * Reading DECOUPLED (mode 0, default): the delta rotation acts about the camera centre on
 * world-aligned axes and the delta translation is added: (exp(r) R, t + tau). This keeps the
 * search size s = (omega degrees, v cm) meaning a rotation of omega and a shift of v.
 * Reading LITERAL (mode 1): the left product with Delta P = [exp(r) | tau]:
 * (exp(r) R, exp(r) t + tau).
 * ---------------------------------------------------------------------------------------- */
void orc_compose(int mode, const double r[3], const double tau[3], const orc_pose* P, orc_pose* out) {
    double E[9], Rn[9], tn[3];
    orc_so3_exp(r, E);
    mat3_mul(E, P->R, Rn);
    if (mode == 1) {
        mat3_vec(E, P->t, tn);
        for (int a = 0; a < 3; ++a) tn[a] += tau[a];
    } else {
        for (int a = 0; a < 3; ++a) tn[a] = P->t[a] + tau[a];
    }
    memcpy(out->R, Rn, sizeof Rn);
    memcpy(out->t, tn, sizeof tn);
}

/* ----------------------------------------------------------------------------------------
 * Back-projection of the depth image to the metric point cloud M_t (Sec. III, problem
 * setting). Pixel (u, v) with depth z is valid iff z is finite and > 0 (reading: no range
 * clip) and u, v are multiples of `pixel_stride`. x = (u - cx) z / fx, y = (v - cy) z / fy.
 * Points are written compacted in raster order (v-major), xyz interleaved.
 * ---------------------------------------------------------------------------------------- */
int64_t orc_backproject(const float* depth, const orc_intr* K, int32_t pixel_stride, double* xyz,
                        int32_t* pix) {
    int64_t n = 0;
    for (int v = 0; v < K->height; ++v)
        for (int u = 0; u < K->width; ++u) {
            if (u % pixel_stride != 0 || v % pixel_stride != 0) continue;
            double z = (double)depth[(int64_t)v * K->width + u];
            if (!(isfinite(z) && z > 0.0)) continue;
            xyz[3 * n + 0] = ((double)u - K->cx) * z / K->fx;
            xyz[3 * n + 1] = ((double)v - K->cy) * z / K->fy;
            xyz[3 * n + 2] = z;
            if (pix) pix[n] = v * K->width + u;
            ++n;
        }
    return n;
}

/* ----------------------------------------------------------------------------------------
 * Initial volume: T = +1 (unobserved), W = 0 (Sec. III overview: the TSDF is a dense tensor).
 * ---------------------------------------------------------------------------------------- */
void orc_vol_init(orc_vol* V) {
    int64_t n = (int64_t)V->nx * V->ny * V->nz;
    for (int64_t q = 0; q < n; ++q) {
        V->T[q] = 1.0;
        V->W[q] = 0.0;
    }
}

/* ----------------------------------------------------------------------------------------
 * Fusion of one aligned depth frame, "the same as KinectFusion" (Sec. III overview; Fig. 2:
 * modify known grids, fill new ones). Reading of the unspecified details:
 *   q = R^T (p - t); skip if q_z <= 0; project u = fx q_x/q_z + cx, v = fy q_y/q_z + cy; nearest
 *   pixel (floor(u + 1/2), floor(v + 1/2)); skip outside the image or on invalid depth;
 *   eta = D - q_z; skip if eta < -tau; phi = min(1, eta/tau);
 *   T <- (T W + phi)/(W + 1); W <- min(W + 1, W_max) (at the cap the update still uses W_max).
 * If `amb` is non-null, voxel flags are written: bit 0 when a decision (pixel choice within
 * `pix_margin` of a rounding boundary, q_z within `eta_margin` of 0, or eta within
 * `eta_margin` of -tau) is so close that a lower-precision implementation may take it the
 * other way. Returns the number of updated voxels.
 * ---------------------------------------------------------------------------------------- */
int64_t orc_integrate(orc_vol* V, const float* depth, const orc_intr* K, const orc_pose* P,
                      uint8_t* amb, double pix_margin, double eta_margin) {
    int64_t total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (int k = 0; k < V->nz; ++k) {
        for (int j = 0; j < V->ny; ++j)
            for (int i = 0; i < V->nx; ++i) {
                int64_t idx = ((int64_t)k * V->ny + j) * V->nx + i;
                uint8_t flag = 0;
                double p[3] = {V->origin[0] + V->vs * i, V->origin[1] + V->vs * j, V->origin[2] + V->vs * k};
                double d[3] = {p[0] - P->t[0], p[1] - P->t[1], p[2] - P->t[2]};
                double q[3];
                for (int a = 0; a < 3; ++a) q[a] = P->R[0 * 3 + a] * d[0] + P->R[1 * 3 + a] * d[1] + P->R[2 * 3 + a] * d[2];
                if (fabs(q[2]) < eta_margin) flag = 1;
                if (q[2] <= 0.0) {
                    if (amb) amb[idx] = flag;
                    continue;
                }
                double u = K->fx * q[0] / q[2] + K->cx;
                double v = K->fy * q[1] / q[2] + K->cy;
                double uh = u + 0.5, vh = v + 0.5;
                if (fabs(uh - nearbyint(uh)) < pix_margin || fabs(vh - nearbyint(vh)) < pix_margin) flag = 1;
                double uf = floor(uh), vf = floor(vh);
                if (uf < 0.0 || uf >= K->width || vf < 0.0 || vf >= K->height) {
                    if (amb) amb[idx] = flag;
                    continue;
                }
                int ui = (int)uf, vi = (int)vf;
                double D = (double)depth[(int64_t)vi * K->width + ui];
                if (!(isfinite(D) && D > 0.0)) {
                    if (amb) amb[idx] = flag;
                    continue;
                }
                double eta = D - q[2];
                if (fabs(eta + V->tau) < eta_margin) flag = 1;
                if (amb) amb[idx] = flag;
                if (eta < -V->tau) continue;
                double phi = eta / V->tau;
                if (phi > 1.0) phi = 1.0;
                double w = V->W[idx];
                V->T[idx] = (V->T[idx] * w + phi) / (w + 1.0);
                V->W[idx] = (w + 1.0 < (double)V->w_max) ? w + 1.0 : (double)V->w_max;
                total += 1;
            }
    }
    return total;
}

/* ----------------------------------------------------------------------------------------
 * Sparse reading of the same fusion, for scenes larger than a dense grid affords (the paper's
 * tensor is dense; this is the bricked extension). The grid is cut into bricks of E x E x E
 * voxels (dims multiples of E). A brick is recorded in the first frame that puts one of its
 * voxels inside the truncation band, i.e. gives it an observation phi < 1 under exactly the
 * decisions of orc_integrate above (-tau <= eta < tau). Only voxels of recorded bricks are
 * updated, by the same running average; every other voxel keeps T = +1, W = 0, so free space
 * far from any surface is not stored. `alloc` holds one flag per brick, brick (bx, by, bz) at
 * (bz * ny/E + by) * nx/E + bx. Returns the number of bricks recorded by this frame.
 * ---------------------------------------------------------------------------------------- */
static int observe(const orc_vol* V, const float* depth, const orc_intr* K, const orc_pose* P, int i, int j, int k,
                   double* phi_out) {
    double p[3] = {V->origin[0] + V->vs * i, V->origin[1] + V->vs * j, V->origin[2] + V->vs * k};
    double d[3] = {p[0] - P->t[0], p[1] - P->t[1], p[2] - P->t[2]};
    double q[3];
    for (int a = 0; a < 3; ++a) q[a] = P->R[0 * 3 + a] * d[0] + P->R[1 * 3 + a] * d[1] + P->R[2 * 3 + a] * d[2];
    if (q[2] <= 0.0) return 0;
    double uf = floor(K->fx * q[0] / q[2] + K->cx + 0.5), vf = floor(K->fy * q[1] / q[2] + K->cy + 0.5);
    if (uf < 0.0 || uf >= K->width || vf < 0.0 || vf >= K->height) return 0;
    double D = (double)depth[(int64_t)(int)vf * K->width + (int)uf];
    if (!(isfinite(D) && D > 0.0)) return 0;
    double eta = D - q[2];
    if (eta < -V->tau) return 0;
    double phi = eta / V->tau;
    *phi_out = phi > 1.0 ? 1.0 : phi;
    return 1;
}

int64_t orc_integrate_bricks(orc_vol* V, uint8_t* alloc, int32_t E, const float* depth, const orc_intr* K,
                             const orc_pose* P) {
    const int nbx = V->nx / E, nby = V->ny / E, nbz = V->nz / E;
    uint8_t* fresh = (uint8_t*)calloc((size_t)nbx * nby * nbz, 1);
    int64_t recorded = 0;
    /* bricks the frame puts a band voxel into */
#pragma omp parallel for reduction(+ : recorded) schedule(static)
    for (int bz = 0; bz < nbz; ++bz)
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) {
                int64_t b = ((int64_t)bz * nby + by) * nbx + bx;
                if (alloc[b]) continue;
                int hit = 0;
                for (int k = bz * E; k < (bz + 1) * E && !hit; ++k)
                    for (int j = by * E; j < (by + 1) * E && !hit; ++j)
                        for (int i = bx * E; i < (bx + 1) * E && !hit; ++i) {
                            double phi;
                            if (observe(V, depth, K, P, i, j, k, &phi) && phi < 1.0) hit = 1;
                        }
                fresh[b] = (uint8_t)hit;
                recorded += hit;
            }
    for (int64_t b = 0; b < (int64_t)nbx * nby * nbz; ++b) alloc[b] |= fresh[b];
    free(fresh);
    /* the running average over the voxels of recorded bricks */
#pragma omp parallel for schedule(static)
    for (int k = 0; k < V->nz; ++k)
        for (int j = 0; j < V->ny; ++j)
            for (int i = 0; i < V->nx; ++i) {
                if (!alloc[((int64_t)(k / E) * nby + j / E) * nbx + i / E]) continue;
                double phi;
                if (!observe(V, depth, K, P, i, j, k, &phi)) continue;
                int64_t idx = ((int64_t)k * V->ny + j) * V->nx + i;
                double w = V->W[idx];
                V->T[idx] = (V->T[idx] * w + phi) / (w + 1.0);
                V->W[idx] = (w + 1.0 < (double)V->w_max) ? w + 1.0 : (double)V->w_max;
            }
    return recorded;
}

/* ----------------------------------------------------------------------------------------
 * TSDF query at a world point (Sec. III-B, fitness equation; valid grids). Reading: the query
 * is trilinear over the 8 voxel centres around the point (lerp in x, then y, then z); the
 * point is in X_k iff the whole stencil is inside the grid and all 8 corners satisfy |T| < 1
 * (observed and within the truncation distance; the +1 sentinel marks unobserved voxels).
 * `cell` optionally forces the lower stencil corner (used for the near-face interval rule).
 * ---------------------------------------------------------------------------------------- */
static int sample_cell(const orc_vol* V, const double g[3], const int64_t c[3], double* val) {
    if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] > V->nx - 2 || c[1] > V->ny - 2 || c[2] > V->nz - 2) return 0;
    double f[3] = {g[0] - (double)c[0], g[1] - (double)c[1], g[2] - (double)c[2]};
    double t[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int64_t idx = ((c[2] + dz) * V->ny + (c[1] + dy)) * V->nx + (c[0] + dx);
                double x = V->T[idx];
                if (!(fabs(x) < 1.0)) return 0;
                t[dz][dy][dx] = x;
            }
    double a00 = t[0][0][0] + f[0] * (t[0][0][1] - t[0][0][0]);
    double a10 = t[0][1][0] + f[0] * (t[0][1][1] - t[0][1][0]);
    double a01 = t[1][0][0] + f[0] * (t[1][0][1] - t[1][0][0]);
    double a11 = t[1][1][0] + f[0] * (t[1][1][1] - t[1][1][0]);
    double b0 = a00 + f[1] * (a10 - a00);
    double b1 = a01 + f[1] * (a11 - a01);
    *val = b0 + f[2] * (b1 - b0);
    return 1;
}

static void grid_coord(const orc_vol* V, const double y[3], double g[3]) {
    for (int a = 0; a < 3; ++a) g[a] = (y[a] - V->origin[a]) / V->vs;
}

int orc_sample(const orc_vol* V, const double y[3], double* val) {
    double g[3];
    grid_coord(V, y, g);
    int64_t c[3] = {(int64_t)floor(g[0]), (int64_t)floor(g[1]), (int64_t)floor(g[2])};
    return sample_cell(V, g, c, val);
}

static void transform(const orc_pose* P, const double x[3], double y[3]) {
    mat3_vec(P->R, x, y);
    for (int a = 0; a < 3; ++a) y[a] += P->t[a];
}

/* ----------------------------------------------------------------------------------------
 * Fitness E(P) = (1/|X|) sum_{x in X} |TSDF(P x)| / tau (Sec. III-B equation); T is stored
 * already divided by tau. Reading: E = 1 (the worst value) when X is empty.
 * ---------------------------------------------------------------------------------------- */
void orc_fitness(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, double* E, int64_t* nvalid) {
    double s = 0.0;
    int64_t c = 0;
    for (int64_t j = 0; j < n; ++j) {
        double y[3], v;
        transform(P, xyz + 3 * j, y);
        if (orc_sample(V, y, &v)) {
            s += fabs(v);
            c += 1;
        }
    }
    *E = c > 0 ? s / (double)c : 1.0;
    if (nvalid) *nvalid = c;
}

void orc_fitness_many(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, int32_t K,
                      double* E, int64_t* nvalid) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < K; ++k) orc_fitness(V, xyz, n, P + k, E + k, nvalid ? nvalid + k : NULL);
}

/* Interval form for comparison with a float32 evaluation. Samples whose grid coordinate lies
 * within `eps` voxels of a cell face are evaluated with every admissible lower-corner choice;
 * the bounds take, per ambiguous sample, the smallest/largest |value| contribution and the
 * largest/smallest count, so [E_lo, E_hi] contains every outcome of such choices. */
void orc_fitness_interval(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, double eps,
                          double* E_lo, double* E_hi, int64_t* n_amb) {
    double s_lo = 0.0, s_hi = 0.0;
    int64_t c_lo = 0, c_hi = 0, amb = 0;
    for (int64_t j = 0; j < n; ++j) {
        double y[3], g[3];
        transform(P, xyz + 3 * j, y);
        grid_coord(V, y, g);
        int64_t opts[3][2];
        int nopt[3];
        int any = 0;
        for (int a = 0; a < 3; ++a) {
            double fl = floor(g[a]);
            opts[a][0] = (int64_t)fl;
            nopt[a] = 1;
            double fr = g[a] - fl;
            if (fr < eps) { opts[a][1] = (int64_t)fl - 1; nopt[a] = 2; any = 1; }
            else if (fr > 1.0 - eps) { opts[a][1] = (int64_t)fl + 1; nopt[a] = 2; any = 1; }
        }
        double amin = 2.0, amax = -1.0;
        int cmin = 1, cmax = 0;
        for (int ox = 0; ox < nopt[0]; ++ox)
            for (int oy = 0; oy < nopt[1]; ++oy)
                for (int oz = 0; oz < nopt[2]; ++oz) {
                    int64_t c[3] = {opts[0][ox], opts[1][oy], opts[2][oz]};
                    double v = 0.0;
                    int ok = sample_cell(V, g, c, &v);
                    double a = ok ? fabs(v) : 0.0;
                    if (a < amin) amin = a;
                    if (a > amax) amax = a;
                    if (ok < cmin) cmin = ok;
                    if (ok > cmax) cmax = ok;
                }
        amb += any;
        s_lo += amin;
        s_hi += amax;
        c_lo += cmin;
        c_hi += cmax;
    }
    /* E_lo: smallest numerator over largest count; E_hi: largest numerator over smallest count. */
    *E_lo = c_hi > 0 ? s_lo / (double)c_hi : 1.0;
    *E_hi = c_lo > 0 ? s_hi / (double)c_lo : 1.0;
    if (c_lo == 0) *E_hi = 1.0 > *E_hi ? 1.0 : *E_hi;
    if (n_amb) *n_amb = amb;
}

void orc_fitness_interval_many(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, int32_t K,
                               double eps, double* E_lo, double* E_hi, int64_t* n_amb) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < K; ++k) orc_fitness_interval(V, xyz, n, P + k, eps, E_lo + k, E_hi + k, n_amb + k);
}

/* Interval form for a volume held in a rounded storage format (form (1): scaled int16 or FP16
 * values). Each stored corner may differ from its FP64 value x by up to d(x) = qrel |x| + qabs
 * (int16: half a step of 1/32767; FP16: half an ulp, at most 2^-11 |x|), on top of which the
 * near-face rule of orc_fitness_interval applies. Per cell choice, a corner with |x| >= 1 is out of
 * the band in any storage (rounding keeps it at or beyond 1); one with 1 - d(x) <= |x| < 1 may land
 * on either side, so a sample with such a corner may or may not be valid; otherwise the sample is
 * valid and, the trilinear weights summing to 1, its value moves by at most the largest d of its 8
 * corners. The bounds combine samples as orc_fitness_interval does (smallest and largest |value|
 * contribution, largest and smallest count), so [E_lo, E_hi] holds the fitness of every volume
 * within those roundings. With qrel = qabs = 0 it is orc_fitness_interval. */
static int sample_cell_rounded(const orc_vol* V, const double g[3], const int64_t c[3], double qrel, double qabs,
                               double* amin, double* amax) {
    /* returns 0: invalid in every storage; 1: valid; 2: either */
    if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] > V->nx - 2 || c[1] > V->ny - 2 || c[2] > V->nz - 2) return 0;
    double f[3] = {g[0] - (double)c[0], g[1] - (double)c[1], g[2] - (double)c[2]};
    double t[2][2][2];
    double dmax = 0.0;
    int edge = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int64_t idx = ((c[2] + dz) * V->ny + (c[1] + dy)) * V->nx + (c[0] + dx);
                double x = V->T[idx];
                if (!(fabs(x) < 1.0)) return 0;
                double d = qrel * fabs(x) + qabs;
                if (fabs(x) >= 1.0 - d) edge = 1;
                if (d > dmax) dmax = d;
                t[dz][dy][dx] = x;
            }
    double a00 = t[0][0][0] + f[0] * (t[0][0][1] - t[0][0][0]);
    double a10 = t[0][1][0] + f[0] * (t[0][1][1] - t[0][1][0]);
    double a01 = t[1][0][0] + f[0] * (t[1][0][1] - t[1][0][0]);
    double a11 = t[1][1][0] + f[0] * (t[1][1][1] - t[1][1][0]);
    double b0 = a00 + f[1] * (a10 - a00);
    double b1 = a01 + f[1] * (a11 - a01);
    double v = fabs(b0 + f[2] * (b1 - b0));
    *amin = v > dmax ? v - dmax : 0.0;
    *amax = v + dmax;
    return edge ? 2 : 1;
}

void orc_fitness_interval_rounded(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, double eps,
                                  double qrel, double qabs, double* E_lo, double* E_hi) {
    double s_lo = 0.0, s_hi = 0.0;
    int64_t c_lo = 0, c_hi = 0;
    for (int64_t j = 0; j < n; ++j) {
        double y[3], g[3];
        transform(P, xyz + 3 * j, y);
        grid_coord(V, y, g);
        int64_t opts[3][2];
        int nopt[3];
        for (int a = 0; a < 3; ++a) {
            double fl = floor(g[a]);
            opts[a][0] = (int64_t)fl;
            nopt[a] = 1;
            double fr = g[a] - fl;
            if (fr < eps) { opts[a][1] = (int64_t)fl - 1; nopt[a] = 2; }
            else if (fr > 1.0 - eps) { opts[a][1] = (int64_t)fl + 1; nopt[a] = 2; }
        }
        double amin = 2.0, amax = -1.0;
        int cmin = 1, cmax = 0;
        for (int ox = 0; ox < nopt[0]; ++ox)
            for (int oy = 0; oy < nopt[1]; ++oy)
                for (int oz = 0; oz < nopt[2]; ++oz) {
                    int64_t c[3] = {opts[0][ox], opts[1][oy], opts[2][oz]};
                    double lo = 0.0, hi = 0.0;
                    int st = sample_cell_rounded(V, g, c, qrel, qabs, &lo, &hi);
                    /* an invalid outcome contributes 0 with count 0 */
                    double olo = st == 1 ? lo : 0.0, ohi = st == 0 ? 0.0 : hi;
                    int ocmin = st == 1 ? 1 : 0, ocmax = st == 0 ? 0 : 1;
                    if (olo < amin) amin = olo;
                    if (ohi > amax) amax = ohi;
                    if (ocmin < cmin) cmin = ocmin;
                    if (ocmax > cmax) cmax = ocmax;
                }
        s_lo += amin;
        s_hi += amax;
        c_lo += cmin;
        c_hi += cmax;
    }
    *E_lo = c_hi > 0 ? s_lo / (double)c_hi : 1.0;
    *E_hi = c_lo > 0 ? s_hi / (double)c_lo : 1.0;
    if (c_lo == 0) *E_hi = 1.0 > *E_hi ? 1.0 : *E_hi;
}

void orc_fitness_interval_rounded_many(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P,
                                       int32_t K, double eps, double qrel, double qabs, double* E_lo, double* E_hi) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < K; ++k) orc_fitness_interval_rounded(V, xyz, n, P + k, eps, qrel, qabs, E_lo + k, E_hi + k);
}

/* ----------------------------------------------------------------------------------------
 * Randomized optimization of one frame (Sec. III-B; schedule of Sec. IV-A).
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    uint64_t seed;
    int32_t frame_index, n_iters, K, n_rates;
    int32_t rates[3];
    int32_t pixel_stride;
    double s1_deg, s1_m, beta;
    int32_t compose_mode, polish_steps, min_valid;
    /* the paper's own schedule (Sec. IV-A): the particle count alternates with the sampling rate,
     * iteration i drawing Ks[(i - 1) mod n_rates] particles when alt_K is set; and the optimization
     * stops once the updated search size is below (stop_deg, stop_m) in both parts (0 = never) */
    int32_t alt_K;
    int32_t Ks[3];
    double stop_deg, stop_m;
} orc_params;

/* Particles drawn in iteration i. */
static int32_t iter_K(const orc_params* prm, int32_t i) {
    return prm->alt_K ? prm->Ks[(i - 1) % prm->n_rates] : prm->K;
}

typedef struct {      /* per-iteration record, filled for i = 1..n_iters */
    double E0, Estar, s_rad, s_m;
    int64_t n_adv, n_pts, nvalid0;
    orc_pose pose;
    int64_t n_particles;  /* K of the iteration */
    int64_t n_near;       /* particles with |E_k - E_0| <= 1e-4 E_0: their membership in the advantage
                             set is decided within FP32 rounding of the fitness (a count, not used) */
} orc_iter_rec;

/* Subsample view S_r of the compacted cloud: S_r[j] = M[j r], j = 0 .. ceil(n/r) - 1
 * (reading of the alternating sampling rates; phase 0). */
static int64_t view(const double* xyz, int64_t n, int32_t r, double* out) {
    int64_t m = 0;
    for (int64_t j = 0; j * r < n; ++j, ++m)
        for (int a = 0; a < 3; ++a) out[3 * m + a] = xyz[3 * j * r + a];
    return m;
}

/* Particle k of iteration i: a_k uniform in [-1, 1)^6 (counter RNG), rotation vector
 * omega * a[0:3] (radians) and translation v * a[3:6] (metres): the "uniform sampling
 * according to s" read as a 6-D box. */
void orc_draw_delta(uint64_t seed, int32_t t, int32_t i, int32_t k, double s_rad, double s_m, double r[3], double tau[3]) {
    for (int d = 0; d < 3; ++d) r[d] = s_rad * orc_uniform_pm1(seed, t, i, k, d);
    for (int d = 0; d < 3; ++d) tau[d] = s_m * orc_uniform_pm1(seed, t, i, k, 3 + d);
}

/* One iteration i (1-based) from pose P and search size (s_rad, s_m) on the point set S.
 * E_0 = E(P; S), E_k = E(compose(delta_k, P); S); advantage set A = {k >= 1 : E_k < E_0}
 * (strict); the mean rotation vector and mean translation over A (ascending k) form the
 * averaged delta (reading: arithmetic mean of rotation vectors, then exp); P <- compose(mean,
 * P) if A is non-empty; E* = E(P; S); s <- s (beta + (1 - beta) E*), the same factor on both
 * components. If `Ek_out` is non-null the K+1 fitness values are stored (slot 0 = E_0). */
void orc_ro_iteration(const orc_vol* V, const double* S, int64_t n, const orc_params* prm, int32_t i,
                      orc_pose* P, double* s_rad, double* s_m, double* Ek_out, int64_t* nv_out, orc_iter_rec* rec) {
    int32_t K = iter_K(prm, i);
    orc_pose* poses = (orc_pose*)malloc(sizeof(orc_pose) * (size_t)(K + 1));
    double* dr = (double*)malloc(sizeof(double) * 6 * (size_t)(K + 1));
    double* E = (double*)malloc(sizeof(double) * (size_t)(K + 1));
    int64_t* nv = (int64_t*)malloc(sizeof(int64_t) * (size_t)(K + 1));
    poses[0] = *P;
    for (int32_t k = 1; k <= K; ++k) {
        orc_draw_delta(prm->seed, prm->frame_index, i, k, *s_rad, *s_m, dr + 6 * k, dr + 6 * k + 3);
        orc_compose(prm->compose_mode, dr + 6 * k, dr + 6 * k + 3, P, poses + k);
    }
    orc_fitness_many(V, S, n, poses, K + 1, E, nv);
    double sr[3] = {0, 0, 0}, st[3] = {0, 0, 0};
    int64_t na = 0;
    for (int32_t k = 1; k <= K; ++k)
        if (E[k] < E[0]) {
            for (int a = 0; a < 3; ++a) {
                sr[a] += dr[6 * k + a];
                st[a] += dr[6 * k + 3 + a];
            }
            na += 1;
        }
    if (na > 0) {
        double mr[3], mt[3];
        for (int a = 0; a < 3; ++a) {
            mr[a] = sr[a] / (double)na;
            mt[a] = st[a] / (double)na;
        }
        orc_pose Pn;
        orc_compose(prm->compose_mode, mr, mt, P, &Pn);
        *P = Pn;
    }
    double Es;
    int64_t nvs;
    orc_fitness(V, S, n, P, &Es, &nvs);
    double f = prm->beta + (1.0 - prm->beta) * Es;
    if (rec) {
        rec->E0 = E[0];
        rec->Estar = Es;
        rec->n_adv = na;
        rec->n_pts = n;
        rec->nvalid0 = nv[0];
        rec->s_rad = *s_rad;
        rec->s_m = *s_m;
        rec->pose = *P;
        rec->n_particles = K;
        int64_t near = 0;
        for (int32_t k = 1; k <= K; ++k)
            if (fabs(E[k] - E[0]) <= 1e-4 * E[0]) near += 1;
        rec->n_near = near;
    }
    *s_rad *= f;
    *s_m *= f;
    if (Ek_out) memcpy(Ek_out, E, sizeof(double) * (size_t)(K + 1));
    if (nv_out) memcpy(nv_out, nv, sizeof(int64_t) * (size_t)(K + 1));
    free(poses);
    free(dr);
    free(E);
    free(nv);
}

/* Advantage set and averaged update on given fitness values (no scoring): returns |A| and
 * writes the updated pose. Lets the selection be checked on identical fitness inputs. */
int64_t orc_advantage_update(const double* E, const double* deltas /*[K+1][6], slot 0 unused*/, int32_t K,
                             int32_t mode, const orc_pose* P, orc_pose* out, double mean_out[6]) {
    double s[6] = {0, 0, 0, 0, 0, 0};
    int64_t na = 0;
    for (int32_t k = 1; k <= K; ++k)
        if (E[k] < E[0]) {
            for (int a = 0; a < 6; ++a) s[a] += deltas[6 * k + a];
            na += 1;
        }
    *out = *P;
    for (int a = 0; a < 6; ++a) mean_out[a] = 0.0;
    if (na > 0) {
        for (int a = 0; a < 6; ++a) mean_out[a] = s[a] / (double)na;
        orc_compose(mode, mean_out, mean_out + 3, P, out);
    }
    return na;
}

/* ----------------------------------------------------------------------------------------
 * Gradient of the fitness with respect to a left twist xi = (rho, phi) applied by the same
 * composition as the delta poses, at xi = 0, with the valid set, the stencil cells and the
 * signs frozen (not in the paper, which uses no gradients; it differentiates the fitness
 * equation of Sec. III-B):
 *   dE/drho = (1/|X|) sum_j s_j grad T(y_j),   dE/dphi = (1/|X|) sum_j (y_j - c) x s_j grad T(y_j)
 * with s_j = sign(T(y_j)) (sign(0) = 0), grad T the analytic trilinear gradient / vs, and c the
 * camera centre t (decoupled) or 0 (literal). grad6 = (rho[3], phi[3]).
 * ---------------------------------------------------------------------------------------- */
static void trilinear_grad(const orc_vol* V, const int64_t c[3], const double f[3], double gT[3]) {
    double t[2][2][2];
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                t[dz][dy][dx] = V->T[((c[2] + dz) * V->ny + (c[1] + dy)) * V->nx + (c[0] + dx)];
    double gx = 0, gy = 0, gz = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy) {
            double wy = dy ? f[1] : 1.0 - f[1], wz = dz ? f[2] : 1.0 - f[2];
            gx += (t[dz][dy][1] - t[dz][dy][0]) * wy * wz;
        }
    for (int dz = 0; dz < 2; ++dz)
        for (int dx = 0; dx < 2; ++dx) {
            double wx = dx ? f[0] : 1.0 - f[0], wz = dz ? f[2] : 1.0 - f[2];
            gy += (t[dz][1][dx] - t[dz][0][dx]) * wx * wz;
        }
    for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
            double wx = dx ? f[0] : 1.0 - f[0], wy = dy ? f[1] : 1.0 - f[1];
            gz += (t[1][dy][dx] - t[0][dy][dx]) * wx * wy;
        }
    gT[0] = gx / V->vs;
    gT[1] = gy / V->vs;
    gT[2] = gz / V->vs;
}

void orc_fitness_grad(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, int32_t mode,
                      double* E, double grad6[6], int64_t* nvalid) {
    double s = 0.0, g[6] = {0, 0, 0, 0, 0, 0};
    int64_t cnt = 0;
    double cc[3] = {0, 0, 0};
    if (mode == 0)
        for (int a = 0; a < 3; ++a) cc[a] = P->t[a];
    for (int64_t j = 0; j < n; ++j) {
        double y[3], gg[3], v;
        transform(P, xyz + 3 * j, y);
        grid_coord(V, y, gg);
        int64_t c[3] = {(int64_t)floor(gg[0]), (int64_t)floor(gg[1]), (int64_t)floor(gg[2])};
        if (!sample_cell(V, gg, c, &v)) continue;
        double f[3] = {gg[0] - c[0], gg[1] - c[1], gg[2] - c[2]};
        double gT[3];
        trilinear_grad(V, c, f, gT);
        double sg = v > 0 ? 1.0 : (v < 0 ? -1.0 : 0.0);
        double u[3] = {y[0] - cc[0], y[1] - cc[1], y[2] - cc[2]};
        s += fabs(v);
        cnt += 1;
        for (int a = 0; a < 3; ++a) g[a] += sg * gT[a];
        g[3] += sg * (u[1] * gT[2] - u[2] * gT[1]);
        g[4] += sg * (u[2] * gT[0] - u[0] * gT[2]);
        g[5] += sg * (u[0] * gT[1] - u[1] * gT[0]);
    }
    if (cnt > 0) {
        *E = s / (double)cnt;
        for (int a = 0; a < 6; ++a) grad6[a] = g[a] / (double)cnt;
    } else {
        *E = 1.0;
        for (int a = 0; a < 6; ++a) grad6[a] = 0.0;
    }
    if (nvalid) *nvalid = cnt;
}

/* Interval form of E and of the frozen-set gradient for comparison with a float32 evaluation:
 * samples whose grid coordinate lies within `eps` voxels of a cell face are evaluated with every
 * admissible cell choice, and samples whose value lies within `sign_eps` of 0 with both signs. With S_a the component sum and C the valid count, each bound is taken
 * over the box [S_lo, S_hi] x [C_lo, C_hi] (S/C is monotone in each for C > 0), so the intervals
 * contain every outcome of such choices. lo/hi: E then the 6 gradient components. */
void orc_fitness_grad_interval(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, int32_t mode,
                               double eps, double sign_eps, double lo[7], double hi[7]) {
    double Slo[7] = {0}, Shi[7] = {0};
    int64_t Clo = 0, Chi = 0;
    double cc[3] = {0, 0, 0};
    if (mode == 0)
        for (int a = 0; a < 3; ++a) cc[a] = P->t[a];
    for (int64_t j = 0; j < n; ++j) {
        double y[3], g[3];
        transform(P, xyz + 3 * j, y);
        grid_coord(V, y, g);
        int64_t opts[3][2];
        int nopt[3];
        for (int a = 0; a < 3; ++a) {
            double fl = floor(g[a]);
            opts[a][0] = (int64_t)fl;
            nopt[a] = 1;
            double fr = g[a] - fl;
            if (fr < eps) { opts[a][1] = (int64_t)fl - 1; nopt[a] = 2; }
            else if (fr > 1.0 - eps) { opts[a][1] = (int64_t)fl + 1; nopt[a] = 2; }
        }
        double u[3] = {y[0] - cc[0], y[1] - cc[1], y[2] - cc[2]};
        double mn[7], mx[7];
        int cmin = 1, cmax = 0;
        for (int e = 0; e < 7; ++e) { mn[e] = INFINITY; mx[e] = -INFINITY; }
        for (int ox = 0; ox < nopt[0]; ++ox)
            for (int oy = 0; oy < nopt[1]; ++oy)
                for (int oz = 0; oz < nopt[2]; ++oz) {
                    int64_t c[3] = {opts[0][ox], opts[1][oy], opts[2][oz]};
                    double v = 0.0, term[7] = {0, 0, 0, 0, 0, 0, 0};
                    int ok = sample_cell(V, g, c, &v);
                    /* the sign of a value within sign_eps of 0 is ambiguous at lower precision:
                     * both signs are admissible there */
                    int ns = 1;
                    double signs[2] = {v > 0 ? 1.0 : (v < 0 ? -1.0 : 0.0), 0.0};
                    if (ok && fabs(v) < sign_eps) { signs[0] = 1.0; signs[1] = -1.0; ns = 2; }
                    for (int si = 0; si < ns; ++si) {
                        if (ok) {
                            double f[3] = {g[0] - c[0], g[1] - c[1], g[2] - c[2]};
                            double gT[3];
                            trilinear_grad(V, c, f, gT);
                            double sg = signs[si];
                            term[0] = fabs(v);
                            for (int a = 0; a < 3; ++a) term[1 + a] = sg * gT[a];
                            term[4] = sg * (u[1] * gT[2] - u[2] * gT[1]);
                            term[5] = sg * (u[2] * gT[0] - u[0] * gT[2]);
                            term[6] = sg * (u[0] * gT[1] - u[1] * gT[0]);
                        }
                        for (int e = 0; e < 7; ++e) {
                            if (term[e] < mn[e]) mn[e] = term[e];
                            if (term[e] > mx[e]) mx[e] = term[e];
                        }
                    }
                    if (ok < cmin) cmin = ok;
                    if (ok > cmax) cmax = ok;
                }
        for (int e = 0; e < 7; ++e) {
            Slo[e] += mn[e];
            Shi[e] += mx[e];
        }
        Clo += cmin;
        Chi += cmax;
    }
    for (int e = 0; e < 7; ++e) {
        if (Chi == 0) { lo[e] = hi[e] = (e == 0 ? 1.0 : 0.0); continue; }
        double cl = Clo > 0 ? (double)Clo : 1.0, ch = (double)Chi;
        double a1 = Slo[e] / cl, a2 = Slo[e] / ch, b1 = Shi[e] / cl, b2 = Shi[e] / ch;
        lo[e] = a1 < a2 ? a1 : a2;
        hi[e] = b1 > b2 ? b1 : b2;
        if (Clo == 0) {               /* every sample may drop out: E may be 1, gradient 0 */
            if (e == 0) hi[e] = hi[e] > 1.0 ? hi[e] : 1.0;
            else { lo[e] = lo[e] < 0.0 ? lo[e] : 0.0; hi[e] = hi[e] > 0.0 ? hi[e] : 0.0; }
        }
    }
}

void orc_fitness_grad_interval_many(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, int32_t B,
                                    int32_t mode, double eps, double sign_eps, double* lo, double* hi) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < B; ++b)
        orc_fitness_grad_interval(V, xyz, n, P + b, mode, eps, sign_eps, lo + 7 * b, hi + 7 * b);
}

void orc_fitness_grad_many(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, int32_t B,
                           int32_t mode, double* E, double* grad, int64_t* nvalid) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < B; ++b) orc_fitness_grad(V, xyz, n, P + b, mode, E + b, grad + 6 * b, nvalid ? nvalid + b : NULL);
}

/* Frozen objective: the valid set X0, the stencil cells and the signs are those of the pose
 * P_freeze; E_f = (1/|X0|) sum_{j in X0} s_j T_cell_j(y_j), with y_j = P_eval x_j and T_cell_j the
 * trilinear polynomial of the frozen cell (extended beyond the cell if y_j leaves it). It equals
 * E(P_freeze) at P_eval = P_freeze and is a polynomial in y, so central differences of it converge
 * at O(h^2) to the analytic gradient. */
double orc_fitness_frozen_at(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P_freeze,
                             const orc_pose* P_eval) {
    double s = 0.0;
    int64_t cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        double y0[3], g0[3], v0;
        transform(P_freeze, xyz + 3 * j, y0);
        grid_coord(V, y0, g0);
        int64_t c[3] = {(int64_t)floor(g0[0]), (int64_t)floor(g0[1]), (int64_t)floor(g0[2])};
        if (!sample_cell(V, g0, c, &v0)) continue;
        double sg = v0 > 0 ? 1.0 : (v0 < 0 ? -1.0 : 0.0);
        double y[3], g[3];
        transform(P_eval, xyz + 3 * j, y);
        grid_coord(V, y, g);
        double f[3] = {g[0] - c[0], g[1] - c[1], g[2] - c[2]};
        double t[2][2][2];
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx)
                    t[dz][dy][dx] = V->T[((c[2] + dz) * V->ny + (c[1] + dy)) * V->nx + (c[0] + dx)];
        double a00 = t[0][0][0] + f[0] * (t[0][0][1] - t[0][0][0]);
        double a10 = t[0][1][0] + f[0] * (t[0][1][1] - t[0][1][0]);
        double a01 = t[1][0][0] + f[0] * (t[1][0][1] - t[1][0][0]);
        double a11 = t[1][1][0] + f[0] * (t[1][1][1] - t[1][1][0]);
        double b0 = a00 + f[1] * (a10 - a00);
        double b1 = a01 + f[1] * (a11 - a01);
        s += sg * (b0 + f[2] * (b1 - b0));
        cnt += 1;
    }
    return cnt > 0 ? s / (double)cnt : 1.0;
}

/* The frozen objective at P with a twist xi = (rho, phi) applied by the delta composition
 * (rotation vector phi, translation rho), frozen at xi = 0: its derivative at 0 is
 * orc_fitness_grad. */
double orc_fitness_frozen(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* P, int32_t mode,
                          const double xi[6]) {
    orc_pose Px;
    orc_compose(mode, xi + 3, xi, P, &Px);
    return orc_fitness_frozen_at(V, xyz, n, P, &Px);
}

/* Gradient with respect to the twist parameters xi0 + dxi of compose(xi, base), frozen at
 * compose(xi0, base), by central differences of the frozen objective with step h (the reference
 * for the adjoint at xi0 != 0, where the chain through the SO(3) exponential matters). */
void orc_grad_xi_fd(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* base, int32_t mode,
                    const double xi0[6], double h, double grad6[6]) {
    orc_pose P0;
    orc_compose(mode, xi0 + 3, xi0, base, &P0);
    for (int a = 0; a < 6; ++a) {
        double xp[6], xm[6];
        for (int b = 0; b < 6; ++b) xp[b] = xm[b] = xi0[b];
        xp[a] += h;
        xm[a] -= h;
        orc_pose Pp, Pm;
        orc_compose(mode, xp + 3, xp, base, &Pp);
        orc_compose(mode, xm + 3, xm, base, &Pm);
        grad6[a] = (orc_fitness_frozen_at(V, xyz, n, &P0, &Pp) - orc_fitness_frozen_at(V, xyz, n, &P0, &Pm)) / (2.0 * h);
    }
}

/* ----------------------------------------------------------------------------------------
 * Gradient polish of a pose (not in the paper; a deterministic rule stated here):
 * `steps` steps of xi = -alpha grad E (grad from orc_fitness_grad). The first alpha of each
 * step makes the largest point displacement bound alpha (|g_rho| + |g_phi| Rmax) equal to half
 * a voxel, Rmax = max_j |y_j - c|; Armijo: accept if E(new) <= E - 1e-4 alpha |g|^2, else halve,
 * at most 5 halvings; stop when no halving is accepted. Returns the number of accepted steps.
 * ---------------------------------------------------------------------------------------- */
int32_t orc_polish(const orc_vol* V, const double* xyz, int64_t n, orc_pose* P, int32_t mode, int32_t steps,
                   double* E_out) {
    int32_t acc = 0;
    double E, g[6];
    int64_t nv;
    orc_fitness_grad(V, xyz, n, P, mode, &E, g, &nv);
    for (int32_t it = 0; it < steps; ++it) {
        if (nv == 0) break;
        double cc[3] = {0, 0, 0};
        if (mode == 0)
            for (int a = 0; a < 3; ++a) cc[a] = P->t[a];
        double rmax = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double y[3];
            transform(P, xyz + 3 * j, y);
            double d = sqrt((y[0] - cc[0]) * (y[0] - cc[0]) + (y[1] - cc[1]) * (y[1] - cc[1]) + (y[2] - cc[2]) * (y[2] - cc[2]));
            if (d > rmax) rmax = d;
        }
        double nr = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        double nphi = sqrt(g[3] * g[3] + g[4] * g[4] + g[5] * g[5]);
        double gg = nr * nr + nphi * nphi;
        double denom = nr + nphi * rmax;
        if (!(denom > 0.0)) break;
        double alpha = 0.5 * V->vs / denom;
        int ok = 0;
        orc_pose Pn;
        double En = E;
        for (int h = 0; h <= 5; ++h) {
            double xi[6];
            for (int a = 0; a < 6; ++a) xi[a] = -alpha * g[a];
            orc_compose(mode, xi + 3, xi, P, &Pn);
            int64_t nvn;
            orc_fitness(V, xyz, n, &Pn, &En, &nvn);
            if (En <= E - 1e-4 * alpha * gg) {
                ok = 1;
                break;
            }
            alpha *= 0.5;
        }
        if (!ok) break;
        *P = Pn;
        acc += 1;
        orc_fitness_grad(V, xyz, n, P, mode, &E, g, &nv);
    }
    if (E_out) *E_out = E;
    return acc;
}

/* ----------------------------------------------------------------------------------------
 * Candidate that the polish starts from (not in the paper; a rule stated here): the lowest
 * fitness among the optimized pose P^(I) (fitness Estar) and the particles k = 1..K of the last
 * iteration (fitness E[k], all on the same view). Ties go to P^(I), then to the lowest particle
 * index. Returns 0 for P^(I), else the particle index k.
 * ---------------------------------------------------------------------------------------- */
int32_t orc_best_candidate(double Estar, const double* E, int32_t K) {
    double Eb = Estar;
    int32_t kb = 0;
    for (int32_t k = 1; k <= K; ++k)
        if (E[k] < Eb) {
            Eb = E[k];
            kb = k;
        }
    return kb;
}

/* ----------------------------------------------------------------------------------------
 * Tracking of one frame: back-project with the pixel stride, then n_iters iterations with the
 * rate cycle rates[(i-1) mod n_rates] and s^(1) = (s1_deg, s1_m) (Sec. IV-A), then optional
 * polish of the best of {P^(I)} and the last iteration's particles on the densest view.
 * Returns the number of points of the full cloud; -1 on allocation failure.
 * ---------------------------------------------------------------------------------------- */
int64_t orc_track_frame(const orc_vol* V, const float* depth, const orc_intr* Kin, const orc_pose* init,
                        const orc_params* prm, orc_pose* out, orc_iter_rec* recs, int32_t* iters_done) {
    int64_t npix = (int64_t)Kin->width * Kin->height;
    double* xyz = (double*)malloc(sizeof(double) * 3 * (size_t)npix);
    double* S = (double*)malloc(sizeof(double) * 3 * (size_t)npix);
    if (!xyz || !S) { free(xyz); free(S); return -1; }
    int64_t n = orc_backproject(depth, Kin, prm->pixel_stride, xyz, NULL);
    orc_pose P = *init;
    double s_rad = prm->s1_deg * M_PI / 180.0, s_m = prm->s1_m;
    const double stop_rad = prm->stop_deg * M_PI / 180.0;
    int32_t Kmax = prm->K;
    for (int q = 0; prm->alt_K && q < prm->n_rates; ++q) Kmax = prm->Ks[q] > Kmax ? prm->Ks[q] : Kmax;
    double* Ek = (double*)malloc(sizeof(double) * (size_t)(Kmax + 1));
    orc_pose best = P;
    int32_t done = 0;
    for (int32_t i = 1; i <= prm->n_iters; ++i) {
        int32_t r = prm->rates[(i - 1) % prm->n_rates];
        int64_t m = view(xyz, n, r, S);
        orc_pose Pprev = P;
        double sr_prev = s_rad, sm_prev = s_m;
        orc_iter_rec rec;
        orc_ro_iteration(V, S, m, prm, i, &P, &s_rad, &s_m, Ek, NULL, &rec);
        if (recs) recs[i - 1] = rec;
        done = i;
        /* early exit: the updated search size s^(i+1) is below the stop size in both parts */
        const int last = i == prm->n_iters ||
                         (prm->stop_deg > 0.0 && prm->stop_m > 0.0 && s_rad < stop_rad && s_m < prm->stop_m);
        if (last) {
            const int32_t kb = orc_best_candidate(rec.Estar, Ek, iter_K(prm, i));
            best = P;
            if (kb > 0) {
                double dr[3], dt[3];
                orc_draw_delta(prm->seed, prm->frame_index, i, kb, sr_prev, sm_prev, dr, dt);
                orc_compose(prm->compose_mode, dr, dt, &Pprev, &best);
            }
            break;
        }
    }
    if (iters_done) *iters_done = done;
    free(Ek);
    if (prm->polish_steps > 0 && n > 0 && prm->n_iters > 0) {
        /* polish the best candidate on the densest view */
        int32_t rmin = prm->rates[0];
        for (int q = 1; q < prm->n_rates; ++q) rmin = prm->rates[q] < rmin ? prm->rates[q] : rmin;
        int64_t m = view(xyz, n, rmin, S);
        double E;
        P = best;
        orc_polish(V, S, m, &P, prm->compose_mode, prm->polish_steps, &E);
    }
    *out = P;
    free(xyz);
    free(S);
    return n;
}

/* ----------------------------------------------------------------------------------------
 * Exhaustive search over a 6-D grid of deltas around `centre`: m points per axis on
 * {-(m-1)/2 .. (m-1)/2} times (rot_step rad, trans_step m) in the order
 * index = ((((r0*m + r1)*m + r2)*m + t0)*m + t1)*m + t2. Returns the argmin (ties to the lowest
 * index) and writes every fitness to E (m^6 values).
 * ---------------------------------------------------------------------------------------- */
int64_t orc_grid_search(const orc_vol* V, const double* xyz, int64_t n, const orc_pose* centre, int32_t m,
                        double rot_step, double trans_step, int32_t mode, double* E) {
    int64_t total = 1;
    for (int a = 0; a < 6; ++a) total *= m;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < total; ++q) {
        int64_t rem = q;
        int idx[6];
        for (int a = 5; a >= 0; --a) {
            idx[a] = (int)(rem % m);
            rem /= m;
        }
        double r[3], tau[3];
        for (int a = 0; a < 3; ++a) {
            r[a] = (idx[a] - 0.5 * (m - 1)) * rot_step;
            tau[a] = (idx[3 + a] - 0.5 * (m - 1)) * trans_step;
        }
        orc_pose P;
        orc_compose(mode, r, tau, centre, &P);
        orc_fitness(V, xyz, n, &P, E + q, NULL);
    }
    int64_t best = 0;
    for (int64_t q = 1; q < total; ++q)
        if (E[q] < E[best]) best = q;
    return best;
}
