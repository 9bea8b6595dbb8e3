/*
 * profusion.h - C ABI of the MI355X (gfx950) library for the data-parallel hot path of
 * PROFusion (arXiv 2509.24236): the randomized, particle-based 6-DoF pose optimization that
 * aligns a depth frame to the scene TSDF (Sec. III-B), and the per-frame TSDF fusion
 * (Sec. III, "Method overview"; Fig. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status:   every int32_t-returning call returns PF_OK (0) or a negative PF_E* code and never
 *           throws. pf_last_error() returns a thread-local message for the last failure.
 *           Arguments are validated before any launch; on PF_EINVAL nothing was enqueued.
 * Memory:   every pointer documented as "device" is caller-owned device memory of the current
 *           HIP device (for example torch tensors). The library never allocates or frees
 *           device memory in these calls; scratch space is passed in as `workspace` (except in
 *           track_frame_noalloc, whose workspace is a fixed array the library holds per GPU).
 *           "host" pointers are read during the call only.
 * Streams:  `stream` is a hipStream_t (NULL = the default stream). All work is enqueued on it
 *           and the calls return without waiting, except where a call says it synchronises.
 * Poses:    camera -> world, x_world = R x_cam + t, R row-major (Sec. III: the camera pose "in
 *           the world coordinate system"); the world frame is the first frame's camera frame.
 * Units:    metres and radians inside; the search size parameters are given in degrees and
 *           metres (the paper states s = (omega degrees, v cm), Sec. III-B).
 * Volume:   voxel (i, j, k) has its centre at origin + voxel_size * (i, j, k); storage is
 *           x-fastest, T[(k*ny + j)*nx + i]. T is the TSDF divided by the truncation distance
 *           tau (so the fitness equation's 1/tau is folded into storage) and +1 marks a voxel
 *           that is unobserved or free beyond the band.
 */
#ifndef PROFUSION_H
#define PROFUSION_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------------ status */
#define PF_OK 0
#define PF_EINVAL (-1)       /* bad argument: null pointer, bad size, non-orthonormal R ... */
#define PF_ENOMEM (-2)       /* workspace smaller than the size query returned */
#define PF_EHIP (-3)         /* a HIP runtime call or kernel launch failed */
#define PF_EUNSUPPORTED (-4) /* a valid request this build does not implement */

/* ------------------------------------------------------------------------------ formats */
#define PF_F32_W_F32 0   /* T float32, W float32 (integer-valued) */
#define PF_F16_W_U8 1    /* T float16 (+1 sentinel), W uint8 */
#define PF_I16_W_U8 2    /* T int16 = RNE(T * 32767), 32767 sentinel, W uint8 */

/* Storage layouts of the T buffer.
 * LINEAR: T x-fastest only (nx*ny*nz elements).
 * CELLS:  T x-fastest, then (at byte offset tsdf_cells_offset()) a cell-major replica used by
 *         particle scoring: cell (i, j, k), i < nx-1, j < ny-1, k < nz-1, stored at index
 *         (k*(ny-1) + j)*(nx-1) + i as its 8 corner values in the order (dx, dy, dz) =
 *         (0,0,0) (1,0,0) (0,1,0) (1,1,0) (0,0,1) (1,0,1) (0,1,1) (1,1,1). A sample then reads
 *         one contiguous 32-byte (FP32) or 16-byte block instead of four rows; the replica is 8x
 *         the size of T and is kept equal to T by tsdf_init, tsdf_import_linear and
 *         tsdf_integrate (which rewrites only the cells of voxels whose stored value changed),
 *         except that in the FP32 and FP16 formats a corner outside the band (|T| >= 1, the +1
 *         sentinel included) is stored as NaN: the interpolated value of a sample is then NaN
 *         exactly when the sample is not valid, which replaces eight corner tests by one.
 *         After the replica (at tsdf_mask_offset()) a cell-validity mask: one uint64 word per
 *         block of 4x4x4 cells, word ((k/4)*mwy + j/4)*mwx + i/4 with mwx = ceil((nx-1)/4),
 *         mwy = ceil((ny-1)/4), mwz = ceil((nz-1)/4), whose bit (i%4) + 4(j%4) + 16(k%4) is set
 *         iff all 8 corners of cell (i, j, k) are in the band; then one byte per word (at
 *         tsdf_mask_offset() + 8*mwx*mwy*mwz rounded up to 256) that is 0 between calls.
 *         Scoring reads the mask before the replica while the particles are widely spread, where
 *         most samples miss the band. The same three calls keep it equal to the replica: fusion
 *         flags the words of voxels that enter or leave the band and rebuilds exactly those. */
/* BRICKS: a sparse volume for scenes larger than a dense grid affords (nx, ny, nz multiples of 8).
 *         Bricks of 8x8x8 voxels live in a pool of max_bricks slots behind a dense brick-index
 *         grid (one int32 per brick: its slot, or -1); there is no hash table. The T buffer holds,
 *         at the offsets tsdf_brick_offsets() returns: a 256-byte header (int32 bricks in use,
 *         int32 overflow flag, int32 bricks in use before the last fusion; at byte 64 a cell of
 *         +1 corners), the index grid (entry (bz * ny/8 + by) * nx/8 + bx for the brick of voxels
 *         8bx..8bx+7, ...), a candidate list of the same size (scratch of tsdf_integrate), the
 *         brick coordinates of every slot (int32 x4), the slots' T (512 values each, x-fastest
 *         inside the brick) and their cells (512 per brick, cell (x, y, z) local to the brick at
 *         x + 8y + 64z, its 8 corners in the CELLS order and with the CELLS marking of corners
 *         outside the band; corners in the next brick along +x/+y/+z read that brick, or +1
 *         where it has no slot), then (at tsdf_mask_offset()) 8 uint64 cell-validity words per
 *         slot: bit (l % 64) of word l / 64 is set iff all 8 corners of the slot's cell at local
 *         index l are in the band (rebuilt for every slot by tsdf_integrate and
 *         tsdf_import_linear; read by scoring as the dense mask is).
 *         The W buffer holds the slots' W. A voxel outside every allocated brick reads T = +1,
 *         W = 0. tsdf_integrate first gives a slot to every brick that holds a voxel the frame
 *         puts in the band (-tau <= eta < tau, the same FP64 test as the update), then updates
 *         the voxels of all allocated bricks exactly as the dense layouts do; voxels of bricks
 *         without a slot are not updated (free space far from any surface is not recorded).
 *         When the pool is full further bricks are not allocated and the overflow flag is set. */
#define PF_LAYOUT_LINEAR 0
#define PF_LAYOUT_CELLS 1
#define PF_LAYOUT_BRICKS 2

/* Delta-pose composition, the reading of "Delta P_k P^(i-1)" (Sec. III-B):
 * DECOUPLED: (exp(r) R, t + tau) - rotate about the camera centre, then shift;
 * LITERAL:   (exp(r) R, exp(r) t + tau) - the left matrix product [exp(r) | tau] P. */
#define PF_COMPOSE_DECOUPLED 0
#define PF_COMPOSE_LITERAL 1

#define PF_MAX_ITERS 64
#define PF_MAX_K 65536

typedef struct pf_pose {
    double R[9]; /* row-major rotation, camera -> world */
    double t[3]; /* camera centre in world coordinates, metres */
} pf_pose;

typedef struct pf_intrinsics {
    double fx, fy, cx, cy; /* pinhole: u = fx x/z + cx, v = fy y/z + cy (pixels) */
    int32_t width, height;
} pf_intrinsics;

typedef struct pf_tsdf {
    int32_t nx, ny, nz;  /* voxels per axis, each >= 2; dense layouts: nx*ny*nz < 2^31 and
                          * nx*ny < 2^24 (index arithmetic in 24-bit multiplies); BRICKS:
                          * (nx/8)(ny/8)(nz/8) < 2^31 and (nx/8)(ny/8) < 2^24 */
    int32_t format;      /* PF_F32_W_F32, PF_F16_W_U8 or PF_I16_W_U8 */
    double voxel_size;   /* metres, > 0 */
    double trunc;        /* truncation distance tau, metres, > 0 */
    double origin[3];    /* centre of voxel (0,0,0), world metres */
    int32_t w_max;       /* weight cap, 1..255 */
    int32_t layout;      /* PF_LAYOUT_LINEAR, PF_LAYOUT_CELLS or PF_LAYOUT_BRICKS */
    int32_t max_bricks;  /* BRICKS: pool slots (1 .. 2^23); 0 for the dense layouts */
    int32_t reserved;    /* must be 0 */
    void* tsdf;          /* device, tsdf_bytes() bytes */
    void* weight;        /* device, *weight_bytes bytes */
} pf_tsdf;

/* Parameters of one frame's randomized optimization (Sec. III-B; schedule of Sec. IV-A). */
typedef struct pf_track_params {
    uint64_t seed;          /* key of the counter-based random stream */
    int32_t frame_index;    /* t, part of the random-stream counter, 0 .. 2^24-1 */
    int32_t n_iters;        /* I, 1 .. PF_MAX_ITERS (the paper caps it at 20) */
    int32_t K;              /* particles per iteration, 1 .. PF_MAX_K */
    int32_t n_rates;        /* 1 .. 3 */
    int32_t rates[3];       /* point sub-sampling strides; iteration i uses rates[(i-1) mod n_rates] */
    int32_t pixel_stride;   /* keep pixels with u, v multiples of it (1 = every pixel) */
    double s1_deg, s1_m;    /* initial search size s^(1) (the paper uses 10 deg, 10 cm) */
    double beta;            /* search-size momentum (the paper uses 0.1) */
    int32_t compose_mode;   /* PF_COMPOSE_* */
    int32_t polish_steps;   /* gradient polish steps after the last iteration (0 = none) */
    int32_t min_valid;      /* stats.lost is set when the final pose has fewer valid samples */
    /* The paper's own schedule (Sec. IV-A): the particle count alternates with the sampling rate
     * (1024, 3072, 10240 there), and the optimization typically stops early. alt_K = 1: iteration
     * i draws Ks[(i-1) mod n_rates] particles, each in 1 .. K (K is the capacity). stop_deg,
     * stop_m > 0: the optimization ends after the first iteration whose updated search size
     * s^(i+1) is below both (the stop rule is a reading; 0 = always run n_iters). */
    int32_t alt_K;
    int32_t Ks[3];
    int32_t reserved;       /* must be 0 */
    double stop_deg, stop_m;
} pf_track_params;

/* Per-frame record written by track_frame (host). */
typedef struct pf_track_stats {
    int32_t n_points;               /* valid back-projected points at the pixel stride */
    int32_t n_iters;                /* iterations that ran */
    int32_t lost;                   /* 1 if the final valid count < min_valid */
    int32_t polish_accepted;        /* accepted polish steps */
    float E0[PF_MAX_ITERS];         /* E(P^(i-1)) on S_i */
    float Estar[PF_MAX_ITERS];      /* E(P^(i)) on S_i */
    int32_t n_adv[PF_MAX_ITERS];    /* |advantage set| */
    int32_t n_sub[PF_MAX_ITERS];    /* |S_i| */
    int32_t n_valid[PF_MAX_ITERS];  /* |X| of P^(i) on S_i */
    double s_rad[PF_MAX_ITERS];     /* s^(i), rotation part */
    double s_m[PF_MAX_ITERS];       /* s^(i), translation part */
    float E_final;                  /* fitness of the returned pose on the densest view */
    int32_t n_valid_final;
    int32_t n_particles[PF_MAX_ITERS]; /* K of iteration i */
} pf_track_stats;

/* Device-resident optimizer state used by particles_update. The layout is public so callers
 * can read it back. The same buffer holds, at byte offset PF_STATE_DELTAS_OFFSET, the deltas of
 * the pending particles as FP64 [K+1][6] (rotation vector, translation; slot 0 is zero), and
 * after them scratch for per-workgroup partial sums. */
typedef struct pf_track_state {
    /* the pending iteration: particles drawn around P^(i-1) with search size s^(i) */
    double R[9], t[3];     /* P^(i-1) */
    double s_rad, s_m;     /* s^(i) */
    /* the last completed iteration */
    double R_new[9], t_new[3]; /* P^(i) */
    double s_rad_done, s_m_done; /* s^(i) of that iteration */
    double E0, Estar;      /* E(P^(i-1)) and E(P^(i)) on S_i */
    double mean[6];        /* averaged delta (r, tau) */
    double R_prev[9], t_prev[3]; /* P^(i-1) of the last completed iteration */
    double beta;
    uint64_t seed;
    int32_t frame_index;
    int32_t iter;          /* i of the pending particles (1-based) */
    int32_t iter_done;     /* i of the last completed iteration (0 = none) */
    int32_t K;
    int32_t compose_mode;
    int32_t n_adv;         /* |A| of the last completed iteration */
    int32_t n_sub;         /* |S_i| of the last completed iteration */
    int32_t n_valid_star;  /* |X| of P^(i) */
    int32_t flags;         /* bit 0: particles_update called with a K other than the state's */
    int32_t K_cur;         /* particles drawn for the pending iteration (K unless alt_K) */
    int32_t done;          /* 1 once the stop rule ended the optimization */
    int32_t alt_K, n_rates;
    int32_t Ks[3];
    int32_t reserved;
    double stop_rad, stop_m;
} pf_track_state;

#define PF_STATE_DELTAS_OFFSET 512

/* ------------------------------------------------------------------------------ errors */

/* Message of the last failed call on this thread ("" if none). Owned by the library. */
const char* pf_last_error(void);

/* ------------------------------------------------------------------------------ volume */

/* Bytes the caller must allocate for v->tsdf (returned) and v->weight (*weight_bytes, may be
 * NULL). Reads only nx, ny, nz, format and layout; returns 0 for an invalid description. */
size_t tsdf_bytes(const pf_tsdf* v, size_t* weight_bytes);

/* Byte offset of the cell-major replica inside v->tsdf (PF_LAYOUT_CELLS), 0 otherwise. */
size_t tsdf_cells_offset(const pf_tsdf* v);

/* Byte offset of the cell-validity mask inside v->tsdf (PF_LAYOUT_CELLS: the dense mask;
 * PF_LAYOUT_BRICKS: the slots' words), 0 otherwise. */
size_t tsdf_mask_offset(const pf_tsdf* v);

/* BRICKS: byte offsets inside v->tsdf of the index grid, the slot coordinates, the slots' T and
 * their cells (each may be NULL); returns PF_EINVAL for another layout or a bad description. */
int32_t tsdf_brick_offsets(const pf_tsdf* v, size_t* index, size_t* coords, size_t* pool_t, size_t* pool_cells);

/* BRICKS: bricks in use and the overflow flag (host ints). Synchronises the stream. */
int32_t tsdf_bricks_used(const pf_tsdf* v, int32_t* n_bricks, int32_t* overflow, void* stream);

/* Sets every voxel to the initial state T = +1 (unobserved), W = 0 (Sec. III overview: the
 * scene is a dense tensor of distance values; the first frame fills it). */
int32_t tsdf_init(const pf_tsdf* v, void* stream);

/* Fuses one aligned depth frame, "the same as KinectFusion" (Sec. III overview; Fig. 2:
 * known grids are modified and new ones filled). For each voxel centre p:
 *   q = R^T (p - t); skip if q_z <= 0; (u, v) = (fx q_x/q_z + cx, fy q_y/q_z + cy);
 *   nearest pixel (floor(u + 1/2), floor(v + 1/2)), skip if outside the image or if its depth
 *   is not finite and > 0; eta = D - q_z; skip if eta < -tau; phi = min(1, eta/tau);
 *   T <- (T W + phi)/(W + 1); W <- min(W + 1, w_max).
 * The projection runs in FP64 (so the update decisions match an FP64 reference exactly) and
 * the running average in the storage format's arithmetic (FP32).
 * depth: device, float32 [height][width], metres; 0, negative or non-finite = invalid.
 * K, cam_to_world: host. R must be orthonormal to 1e-9, else PF_EINVAL. */
int32_t tsdf_integrate(const pf_tsdf* v, const float* depth, const pf_intrinsics* K,
                       const pf_pose* cam_to_world, void* stream);

/* Copies the volume out as FP32 x-fastest arrays (T_out, W_out: device, nx*ny*nz floats;
 * W_out may be NULL). For the int16 format T = q/32767; for fp16, T = (float)half. BRICKS:
 * voxels outside allocated bricks come out as T = +1, W = 0. */
int32_t tsdf_export_linear(const pf_tsdf* v, float* T_out, float* W_out, void* stream);

/* Loads the volume from FP32 x-fastest arrays (device; W_in may be NULL = all 0), converting
 * to the storage format (int16: RNE(T*32767) clamped to +-32767; uint8: RNE, clamped).
 * BRICKS: the volume is cleared and a slot is given to every brick holding a voxel other than
 * (T, W) = (+1, 0); bricks that do not fit in the pool are dropped and set the overflow flag. */
int32_t tsdf_import_linear(const pf_tsdf* v, const float* T_in, const float* W_in, void* stream);

/* ------------------------------------------------------------------------------ points */

/* Back-projects a depth image to the metric point cloud M_t (Sec. III, problem setting):
 * pixel (u, v) with finite depth z > 0 and u, v multiples of pixel_stride gives
 * (x, y, z) = ((u - cx) z/fx, (v - cy) z/fy, z). Points are compacted in raster order
 * (v-major) into px, py, pz (device, width*height floats each). n_out: device int32 buffer of
 * at least 1 + ceil(width*height / 1024) values; n_out[0] receives the count, the rest is
 * scratch for the per-workgroup counts of the compaction. */
int32_t backproject(const float* depth, const pf_intrinsics* K, int32_t pixel_stride, float* px,
                    float* py, float* pz, int32_t* n_out, void* stream);

/* ------------------------------------------------------------------------------ particles */

/* Fitness of K poses against the TSDF (Sec. III-B, fitness equation):
 *   E_k = (1/|X_k|) sum_{x in X_k} |T(R_k x + t_k)|,
 * where T(.) is the trilinear interpolation of the 8 voxel centres around the point and x is
 * in X_k iff that stencil lies inside the grid and all 8 stored values satisfy |T| < 1
 * (observed and within the truncation distance: the "valid grids"). E_k = 1 if X_k is empty.
 * px, py, pz: device, n_pts floats (camera coordinates, metres), 1 <= n_pts < 2^30 (the kernels
 * address a point by a 32-bit byte offset); PF_EINVAL otherwise.
 * poses: device, [K][12] float32, row-major 3x4 [R | t] camera -> world.
 * fitness: device, K floats; n_valid: device, K int32 (|X_k|).
 * Each valid |T| is converted to 32-bit fixed point (units of 2^-32; 2^-17 stored units for
 * int16) and summed exactly in 64-bit integers, so E_k does not depend on the launch shape or on
 * how points are split: results are bitwise reproducible. E_k = sum / |X_k| rounded to FP32. */
int32_t particles_score(const pf_tsdf* v, const float* px, const float* py, const float* pz,
                        int32_t n_pts, const float* poses, int32_t K, float* fitness,
                        int32_t* n_valid, void* stream);

/* Adjoint of the fitness (not in the paper, which uses no gradients; it differentiates the
 * fitness equation of Sec. III-B): for each of B poses P_b = compose(xi_b, base_b) it returns
 * E_b and dE_b/dxi_b, xi = (rho, phi) = (translation, rotation vector) applied by the delta
 * composition (PF_COMPOSE_*). The valid set, stencil cells and signs are frozen at P_b:
 *   dE/d(delta_tau) = (1/|X|) sum_j s_j grad T(y_j),
 *   dE/d(delta_r)   = (1/|X|) sum_j (y_j - c) x s_j grad T(y_j),
 * s_j = sign(T(y_j)), grad T the analytic trilinear gradient, c = the camera centre (DECOUPLED) or
 * the origin (LITERAL); the chain through compose uses the SO(3) left Jacobian J(phi):
 * dE/dphi = J^T dE/d(delta_r) (DECOUPLED) or J^T (dE/d(delta_r) - rho x dE/d(delta_tau)) (LITERAL).
 * E and the gradient come from one gather pass; sums are FP32 in a fixed order.
 * base: device FP64 [B][12] row-major [R | t]; xi: device FP64 [B][6] or NULL (xi = 0);
 * fitness: device float [B]; grad: device float [B][6] (rho, phi); n_valid: device int32 [B] or NULL. */
int32_t particles_score_grad(const pf_tsdf* v, const float* px, const float* py, const float* pz,
                             int32_t n_pts, const double* base, const double* xi, int32_t B,
                             int32_t compose_mode, float* fitness, float* grad, int32_t* n_valid,
                             void* stream);

/* Launch shape of the scoring launches with more than 64 poses (particles_score and
 * track_frame): poses per workgroup (1, 2, 4, 8) and workgroup size (64, 128, 256, 512; 1 pose
 * needs >= 256), or 0 and 0 (the default) for the automatic shape, 4 poses x 256 threads (fewer
 * poses per workgroup when K is too small to fill the GPU); track_frame then also picks, per
 * iteration, the launch of the spread regime of the search size that drew its particles (see
 * pf_score_mask); with the automatic 4 x 256 shape and that regime known from the previous call
 * with the same parameters, the particle launch also draws its particles (otherwise a separate
 * launch draws them first). Process-wide: a launch in flight on another thread takes the old or the new
 * shape. Fitness sums are exact (64-bit fixed point), so every shape, and
 * the batched path, gives bitwise identical results; the shape changes speed only. Returns
 * PF_EINVAL for an unsupported shape. */
int32_t pf_score_config(int32_t poses_per_group, int32_t group_size);

/* When the scoring launches of particles_score and track_frame read a CELLS or BRICKS volume's
 * cells through its cell-validity mask: PF_MASK_BY_SPREAD (the default: the automatic launches of
 * track_frame while the particles are spread over more than a quarter voxel, where many samples
 * miss the band; never in particles_score, which has no spread, nor with a configured shape),
 * PF_MASK_ALWAYS (every launch, configured shapes included) or PF_MASK_NEVER. A launch that reads
 * the mask gathers and interpolates only the valid samples, compacted into full waves (a BRICKS
 * launch whose queues would not fit in LDS does not read it). LINEAR volumes have no mask; the
 * batched path reads it by spread whatever the mode. Process-wide. The mask bit of a cell equals
 * the cell's validity, so results are bitwise identical in every mode; the mode changes speed
 * only. Returns PF_EINVAL for another value. */
#define PF_MASK_BY_SPREAD 0
#define PF_MASK_ALWAYS 1
#define PF_MASK_NEVER 2
int32_t pf_score_mask(int32_t mode);

/* Bytes of the device state buffer for K particles (pf_track_state + (K+1)*6 doubles). */
size_t particles_state_bytes(int32_t K);

/* Initialises the device state for one frame: P^(0) = init (host), s^(1) from p (degrees are
 * converted to radians), iteration 1, the particle schedule and stop size of p, and draws the
 * particles of iteration 1 (K, or Ks[0] with alt_K) into next_poses (device, [K+1][12]
 * float32; slot 0 = P^(0)). */
int32_t particles_state_init(void* state, const pf_pose* init, const pf_track_params* p,
                             float* next_poses, void* stream);

/* One step of the randomized optimization (Sec. III-B) after the pending particles of
 * iteration i (state->K_cur of them) were scored on the point set S_i (px, py, pz, n_pts) into
 * fitness / n_valid ([K_cur+1], slot 0 = the current pose P^(i-1)):
 *   A = {k >= 1 : E_k < E_0} (strict); if A is non-empty, P^(i) = compose(mean over A of the
 *   rotation vectors and of the translations, P^(i-1)), else P^(i) = P^(i-1);
 *   E* = E(P^(i); S_i); s^(i+1) = s^(i) (beta + (1 - beta) E*);
 * then, unless s^(i+1) is below the stop size (state->done is then set and every later call
 * returns without work), draws the particles of iteration i+1 (K, or Ks[i mod n_rates] with
 * alt_K; state->K_cur): a in [-1,1)^6 from SplitMix64 at counter t<<40 | (i+1)<<32 | k<<3 | d,
 * rotation vector omega a[0:3], translation v a[3:6], composed with P^(i) in FP64 and rounded to
 * float32 into next_poses (slot 0 = P^(i)).
 * state: device buffer of particles_state_bytes(K) bytes; K is the capacity the state was
 * initialised with (a mismatch sets bit 0 of state->flags and leaves the state unchanged). */
int32_t particles_update(const pf_tsdf* v, const float* px, const float* py, const float* pz,
                         int32_t n_pts, const float* fitness, const int32_t* n_valid,
                         void* state, int32_t K, float* next_poses, void* stream);

/* ------------------------------------------------------------------------------ frame */

/* Workspace bytes for track_frame with these intrinsics and parameters. */
size_t track_workspace_bytes(const pf_intrinsics* K, const pf_track_params* p);

/* Randomized optimization of one frame (Sec. III-B, schedule of Sec. IV-A): back-projects
 * the depth at the pixel stride, builds the sub-sampled views S_r[j] = M[j r], runs n_iters
 * iterations of particles_score + particles_update on the device (fewer when the stop size ends
 * the optimization; the launches of the remaining iterations return at once, with no host
 * synchronisation), optionally polishes the best
 * candidate (polish_steps > 0: the lowest fitness among P^(I) and the particles of iteration I,
 * ties to P^(I) then the lowest index, refined by polish_steps gradient steps xi = -alpha grad E on
 * the densest view; the first alpha of a step moves no point more than half a voxel, Armijo
 * acceptance E_new <= E - 1e-4 alpha |grad|^2 with up to 5 halvings, stop when none is accepted),
 * then synchronises the stream and
 * writes the final pose to *out (host) and the per-iteration record to *stats (host,
 * nullable). It does not fuse the frame: call tsdf_integrate with *out afterwards.
 * depth: device float32 [height][width]; init: host; workspace: device, >= ws_bytes. */
int32_t track_frame(const pf_tsdf* v, const float* depth, const pf_intrinsics* K,
                    const pf_pose* init, const pf_track_params* p, pf_pose* out,
                    pf_track_stats* stats, void* workspace, size_t ws_bytes, void* stream);

/* One frame of the method's per-frame cycle (Sec. III "Method overview", Fig. 2: the pose is
 * tracked, then the frame is fused into the TSDF at that pose): track_frame, then the fusion of
 * tsdf_integrate at the pose written to *out, with the same results as those two calls in turn.
 * For the dense layouts the fusion reads the tracked pose from the device and is enqueued before
 * the call waits for its read-back, so the GPU fuses while the host reads the result; the fusion
 * may still be running when the call returns (it is ordered on `stream`). For BRICKS the fusion is
 * enqueued after the read-back, from the host. The volume is fused only when the call returns
 * PF_OK. The first call on a host thread allocates a small pinned host buffer and an event for the
 * read-back (kept until the process ends). Needs v->weight. */
int32_t track_frame_fuse(const pf_tsdf* v, const float* depth, const pf_intrinsics* K, const pf_pose* init,
                         const pf_track_params* p, pf_pose* out, pf_track_stats* stats, void* workspace,
                         size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): track_frame with its workspace in an array the library holds on each GPU instead
 * of a caller buffer. Same arguments, results and synchronisation as track_frame, bit for bit,
 * without workspace and ws_bytes. The array is PF_NOALLOC_WORKSPACE_BYTES per GPU (enough for
 * 1280x960 depth at PF_MAX_K particles); it is set up on the first call on a device and held until
 * the process ends. The call allocates and frees nothing. A call whose track_workspace_bytes()
 * exceeds the array returns PF_ENOMEM with a message, before any launch. Every call on a GPU
 * uses that GPU's one array: calls that overlap on one GPU (other host threads, or other streams
 * before this call has returned) race and must be serialised by the caller. Nothing in the
 * array needs clearing between calls; each call rewrites what it reads. */
#define PF_NOALLOC_WORKSPACE_BYTES (32u << 20)
int32_t track_frame_noalloc(const pf_tsdf* v, const float* depth, const pf_intrinsics* K,
                            const pf_pose* init, const pf_track_params* p, pf_pose* out,
                            pf_track_stats* stats, void* stream);

/* ------------------------------------------------------------------------------ batches */

/* Many independent tracking problems run together: every step of the frame optimization is one
 * launch over all problems (the scoring launch is persistent: a fixed grid walks the list of
 * (problem, pose group) items), so the whole batch is a short fixed sequence of kernels that a
 * HIP graph can capture once and replay. Each problem computes bit for bit what track_frame
 * computes for it alone (the per-pose reduction order does not depend on the batching); this
 * needs K >= 64 (track_frame scores up to 64 poses with wider workgroups), which is enforced. */
typedef struct pf_batch_problem {
    pf_tsdf vol;             /* the problem's volume (all problems share format and layout) */
    const float* depth;      /* device, float32 [height][width] */
    pf_intrinsics K;
    pf_pose init;            /* P^(0) */
    pf_track_params params;  /* n_iters, rates and polish_steps equal across the batch; the fixed
                                schedule only (alt_K = 0, no stop rule) */
} pf_batch_problem;

/* Launch plan of a batch (the project autotuner chooses it per shape class). */
typedef struct pf_batch_plan {
    int32_t score_tk;        /* poses per scoring workgroup of 256 threads: 1, 2, 4 or 8; or 0,
                                track_frame's automatic shape (4) */
    int32_t score_grid;      /* workgroups of the persistent scoring launch, >= 1 */
    int32_t order;           /* 0: items in problem order; 1: problems with most points first */
    int32_t reserved;        /* must be 0 */
} pf_batch_plan;

typedef struct pf_batch pf_batch; /* opaque host-side record of a prepared batch */

/* Workspace bytes for a batch of n problems (host array). */
size_t track_batch_workspace_bytes(const pf_batch_problem* problems, int32_t n);

/* Validates the problems (host array), lays them out in `workspace` (device) and uploads the
 * problem table and item lists; synchronises `stream`. Returns NULL on error (pf_last_error).
 * The returned record is host memory owned by the caller via track_batch_destroy. */
pf_batch* track_batch_create(const pf_batch_problem* problems, int32_t n, const pf_batch_plan* plan,
                             void* workspace, size_t ws_bytes, void* stream);

/* Enqueues the whole batch (back-projection, views, every iteration, final fitness) on
 * `stream`. Kernel launches only: no host synchronisation, copy or allocation, so it can be
 * captured into a HIP graph and replayed; the depth and volume contents are read at run time. */
int32_t track_batch_run(pf_batch* b, void* stream);

/* Synchronises `stream` and copies each problem's pose (out[n], host) and record (stats[n], host,
 * nullable) back. */
int32_t track_batch_results(pf_batch* b, pf_pose* out, pf_track_stats* stats, void* stream);

void track_batch_destroy(pf_batch* b);

/* ------------------------------------------------------------------------------ timing */

/* Kernel timing of the particle-scoring launches made by track_frame (the draw included when the
 * launch draws its own particles): when enabled, each such launch is bracketed by HIP events on
 * the call's stream (the interval includes the launch's dispatch) and, once track_frame has synchronised,
 * the elapsed times, the number of launches and the number of evaluated (pose, point) samples
 * (sum of poses x points per launch) are accumulated. Switch, events and counters belong to the
 * calling host thread: enable and read on the thread that calls track_frame. */
int32_t pf_timing_enable(int32_t on);

/* Reads the counters (any pointer may be NULL) and optionally resets them. */
int32_t pf_timing_read(double* score_ms, int64_t* score_launches, int64_t* score_evals, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* PROFUSION_H */
