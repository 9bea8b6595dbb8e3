"""FP64 CPU oracle for PROFusion's tracking-and-fusion hot path (arXiv 2509.24236).

TEST INFRASTRUCTURE ONLY: the plain reference that the HIP library is checked against. Only
the tests, the smoke check and the benchmark's CPU-baseline leg use it; the product path
never imports it. It shares no code with the HIP library: the arithmetic lives in
`oracle.c` (built with gcc, -O2 -ffp-contract=off, OpenMP over independent particles or
slabs) and this module only marshals numpy arrays through ctypes.

Each wrapper names the passage of the paper it follows (see `oracle.c` for the readings of
passages the paper leaves open). Pose convention: camera -> world, (R 3x3, t 3) float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

COMPOSE_DECOUPLED = 0
COMPOSE_LITERAL = 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]

    @staticmethod
    def of(R, t) -> "Pose":
        p = Pose()
        p.R[:] = [float(x) for x in np.asarray(R, np.float64).reshape(9)]
        p.t[:] = [float(x) for x in np.asarray(t, np.float64).reshape(3)]
        return p

    def rt(self) -> Tuple[np.ndarray, np.ndarray]:
        return np.array(self.R[:], np.float64).reshape(3, 3), np.array(self.t[:], np.float64)


class Intr(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]

    @staticmethod
    def of(k) -> "Intr":
        return Intr(float(k.fx), float(k.fy), float(k.cx), float(k.cy), int(k.width), int(k.height))


class Vol(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("w_max", C.c_int32),
                ("vs", C.c_double), ("tau", C.c_double), ("origin", C.c_double * 3),
                ("T", C.POINTER(C.c_double)), ("W", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("frame_index", C.c_int32), ("n_iters", C.c_int32),
                ("K", C.c_int32), ("n_rates", C.c_int32), ("rates", C.c_int32 * 3),
                ("pixel_stride", C.c_int32), ("s1_deg", C.c_double), ("s1_m", C.c_double),
                ("beta", C.c_double), ("compose_mode", C.c_int32), ("polish_steps", C.c_int32),
                ("min_valid", C.c_int32), ("alt_K", C.c_int32), ("Ks", C.c_int32 * 3), ("stop_deg", C.c_double),
                ("stop_m", C.c_double)]


class IterRec(C.Structure):
    _fields_ = [("E0", C.c_double), ("Estar", C.c_double), ("s_rad", C.c_double), ("s_m", C.c_double),
                ("n_adv", C.c_int64), ("n_pts", C.c_int64), ("nvalid0", C.c_int64), ("pose", Pose),
                ("n_particles", C.c_int64), ("n_near", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp, i64p = P(C.c_double), P(C.c_int64)
        L.orc_num_threads.restype = C.c_int32
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_counter.restype = C.c_uint64
        L.orc_counter.argtypes = [C.c_int64] * 4
        L.orc_uniform_pm1.restype = C.c_double
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [C.c_int32]
        L.orc_uniform_pm1.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int64, C.c_int64]
        L.orc_so3_exp.argtypes = [dp, dp]
        L.orc_so3_log.argtypes = [dp, dp]
        L.orc_compose.argtypes = [C.c_int, dp, dp, P(Pose), P(Pose)]
        L.orc_backproject.restype = C.c_int64
        L.orc_backproject.argtypes = [P(C.c_float), P(Intr), C.c_int32, dp, P(C.c_int32)]
        L.orc_vol_init.argtypes = [P(Vol)]
        L.orc_integrate.restype = C.c_int64
        L.orc_integrate.argtypes = [P(Vol), P(C.c_float), P(Intr), P(Pose), P(C.c_uint8), C.c_double, C.c_double]
        L.orc_integrate_bricks.restype = C.c_int64
        L.orc_integrate_bricks.argtypes = [P(Vol), P(C.c_uint8), C.c_int32, P(C.c_float), P(Intr), P(Pose)]
        L.orc_sample.restype = C.c_int
        L.orc_sample.argtypes = [P(Vol), dp, dp]
        L.orc_fitness.argtypes = [P(Vol), dp, C.c_int64, P(Pose), dp, i64p]
        L.orc_fitness_many.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, dp, i64p]
        L.orc_fitness_interval_many.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, C.c_double, dp, dp, i64p]
        L.orc_fitness_interval_rounded_many.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, C.c_double,
                                                        C.c_double, C.c_double, dp, dp]
        L.orc_draw_delta.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_double, dp, dp]
        L.orc_ro_iteration.argtypes = [P(Vol), dp, C.c_int64, P(Params), C.c_int32, P(Pose), dp, dp, dp, i64p, P(IterRec)]
        L.orc_advantage_update.restype = C.c_int64
        L.orc_advantage_update.argtypes = [dp, dp, C.c_int32, C.c_int32, P(Pose), P(Pose), dp]
        L.orc_fitness_grad.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, dp, dp, i64p]
        L.orc_fitness_grad_many.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, C.c_int32, dp, dp, i64p]
        L.orc_fitness_grad_interval_many.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, C.c_int32,
                                                     C.c_double, C.c_double, dp, dp]
        L.orc_fitness_frozen_at.restype = C.c_double
        L.orc_fitness_frozen_at.argtypes = [P(Vol), dp, C.c_int64, P(Pose), P(Pose)]
        L.orc_grad_xi_fd.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, dp, C.c_double, dp]
        L.orc_fitness_frozen.restype = C.c_double
        L.orc_fitness_frozen.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, dp]
        L.orc_polish.restype = C.c_int32
        L.orc_polish.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, C.c_int32, dp]
        L.orc_best_candidate.restype = C.c_int32
        L.orc_best_candidate.argtypes = [C.c_double, dp, C.c_int32]
        L.orc_track_frame.restype = C.c_int64
        L.orc_track_frame.argtypes = [P(Vol), P(C.c_float), P(Intr), P(Pose), P(Params), P(Pose), P(IterRec),
                                      P(C.c_int32)]
        L.orc_grid_search.restype = C.c_int64
        L.orc_grid_search.argtypes = [P(Vol), dp, C.c_int64, P(Pose), C.c_int32, C.c_double, C.c_double, C.c_int32, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops (used to time it on one core)."""
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(lib().orc_num_threads())


# ----------------------------------------------------------------------------- RNG and SO(3)
def splitmix64(seed: int, n: int) -> int:
    """n-th output of SplitMix64 started at `seed` (Steele, Lea, Flood 2014)."""
    return int(lib().orc_splitmix64(C.c_uint64(seed & (2**64 - 1)), C.c_uint64(n)))


def counter(t, i, k, d) -> int:
    return int(lib().orc_counter(t, i, k, d))


def uniform_pm1(seed, t, i, k, d) -> float:
    return float(lib().orc_uniform_pm1(C.c_uint64(seed), t, i, k, d))


def so3_exp(r) -> np.ndarray:
    r = _f64(r).reshape(3)
    R = np.zeros(9)
    lib().orc_so3_exp(_dp(r), _dp(R))
    return R.reshape(3, 3)


def so3_log(R) -> np.ndarray:
    R = _f64(R).reshape(9)
    r = np.zeros(3)
    lib().orc_so3_log(_dp(R), _dp(r))
    return r


def compose(r, tau, R, t, mode=COMPOSE_DECOUPLED):
    """Delta pose applied to (R, t) (Sec. III-B, 'Delta P_k P^(i-1)')."""
    r, tau = _f64(r).reshape(3), _f64(tau).reshape(3)
    P, out = Pose.of(R, t), Pose()
    lib().orc_compose(mode, _dp(r), _dp(tau), C.byref(P), C.byref(out))
    return out.rt()


def draw_delta(seed, t, i, k, s_rad, s_m):
    r, tau = np.zeros(3), np.zeros(3)
    lib().orc_draw_delta(C.c_uint64(seed), t, i, k, s_rad, s_m, _dp(r), _dp(tau))
    return r, tau


def rot_err(Ra, Rb) -> float:
    """Rotation angle between two rotations: arccos((tr(Ra^T Rb) - 1)/2) (the rotation term of
    the paper's regression loss, Sec. III-A), with the chordal form 2 asin(|Ra - Rb|_F / (2 sqrt 2))
    used below 1e-3 rad for precision."""
    Ra, Rb = np.asarray(Ra, np.float64), np.asarray(Rb, np.float64)
    ch = 2.0 * np.arcsin(min(1.0, np.linalg.norm(Ra - Rb) / (2.0 * np.sqrt(2.0))))
    if ch < 1e-3:
        return float(ch)
    c = (np.trace(Ra.T @ Rb) - 1.0) / 2.0
    return float(np.arccos(np.clip(c, -1.0, 1.0)))


# ----------------------------------------------------------------------------- geometry
def backproject(depth: np.ndarray, intr, pixel_stride: int = 1):
    """Depth -> compacted metric point cloud M_t (Sec. III): (N, 3) float64 and pixel indices."""
    d = np.ascontiguousarray(depth, dtype=np.float32)
    n_pix = d.size
    xyz = np.zeros((n_pix, 3))
    pix = np.zeros(n_pix, np.int32)
    K = Intr.of(intr)
    n = lib().orc_backproject(d.ctypes.data_as(C.POINTER(C.c_float)), C.byref(K), pixel_stride, _dp(xyz),
                              pix.ctypes.data_as(C.POINTER(C.c_int32)))
    return xyz[:n].copy(), pix[:n].copy()


def subsample(xyz: np.ndarray, r: int) -> np.ndarray:
    """S_r[j] = M[j r] (phase 0)."""
    return np.ascontiguousarray(xyz[::r])


class Volume:
    """Dense FP64 TSDF volume: T (normalised, +1 = unobserved) and W, x-fastest (nz, ny, nx)."""

    def __init__(self, spec, w_max: int = 255, T: Optional[np.ndarray] = None, W: Optional[np.ndarray] = None):
        self.spec = spec
        shape = (spec.nz, spec.ny, spec.nx)
        self.T = _f64(T).reshape(shape).copy() if T is not None else np.ones(shape)
        self.W = _f64(W).reshape(shape).copy() if W is not None else np.zeros(shape)
        self.w_max = w_max

    def c(self) -> Vol:
        v = Vol()
        s = self.spec
        v.nx, v.ny, v.nz, v.w_max = s.nx, s.ny, s.nz, self.w_max
        v.vs, v.tau = s.voxel_size, s.trunc
        v.origin[:] = list(s.origin)
        v.T, v.W = _dp(self.T), _dp(self.W)
        self._keep = v
        return v

    def integrate(self, depth, intr, R, t, pix_margin=0.0, eta_margin=0.0, want_flags=False):
        """KinectFusion running-average fusion of one frame (Sec. III overview; Fig. 2)."""
        d = np.ascontiguousarray(depth, dtype=np.float32)
        flags = np.zeros(self.T.shape, np.uint8) if want_flags else None
        n = lib().orc_integrate(C.byref(self.c()), d.ctypes.data_as(C.POINTER(C.c_float)), C.byref(Intr.of(intr)),
                                C.byref(Pose.of(R, t)),
                                flags.ctypes.data_as(C.POINTER(C.c_uint8)) if want_flags else None,
                                pix_margin, eta_margin)
        return (int(n), flags) if want_flags else int(n)

    def integrate_bricks(self, depth, intr, R, t, edge=8):
        """Sparse reading of the fusion: bricks of edge^3 voxels recorded at the first frame that puts
        one of their voxels in the band; only their voxels are updated. Returns the bricks recorded;
        the flags are kept in self.bricks, shape (nz/edge, ny/edge, nx/edge)."""
        s = self.spec
        if getattr(self, "bricks", None) is None:
            self.bricks = np.zeros((s.nz // edge, s.ny // edge, s.nx // edge), np.uint8)
        d = np.ascontiguousarray(depth, dtype=np.float32)
        n = lib().orc_integrate_bricks(C.byref(self.c()), self.bricks.ctypes.data_as(C.POINTER(C.c_uint8)), edge,
                                       d.ctypes.data_as(C.POINTER(C.c_float)), C.byref(Intr.of(intr)),
                                       C.byref(Pose.of(R, t)))
        return int(n)

    def sample(self, y):
        y = _f64(y).reshape(3)
        v = C.c_double(0.0)
        ok = lib().orc_sample(C.byref(self.c()), _dp(y), C.byref(v))
        return bool(ok), float(v.value)

    def fitness(self, xyz, R, t):
        """E(P) of the fitness equation (Sec. III-B) and |X|."""
        x = _f64(xyz)
        E, nv = C.c_double(), C.c_int64()
        lib().orc_fitness(C.byref(self.c()), _dp(x), x.shape[0], C.byref(Pose.of(R, t)), C.byref(E), C.byref(nv))
        return float(E.value), int(nv.value)

    def fitness_many(self, xyz, poses: Sequence):
        x = _f64(xyz)
        K = len(poses)
        arr = (Pose * K)(*[Pose.of(R, t) for R, t in poses])
        E = np.zeros(K)
        nv = np.zeros(K, np.int64)
        lib().orc_fitness_many(C.byref(self.c()), _dp(x), x.shape[0], arr, K, _dp(E),
                               nv.ctypes.data_as(C.POINTER(C.c_int64)))
        return E, nv

    def fitness_interval_many(self, xyz, poses: Sequence, eps=1e-3):
        x = _f64(xyz)
        K = len(poses)
        arr = (Pose * K)(*[Pose.of(R, t) for R, t in poses])
        lo, hi = np.zeros(K), np.zeros(K)
        na = np.zeros(K, np.int64)
        lib().orc_fitness_interval_many(C.byref(self.c()), _dp(x), x.shape[0], arr, K, eps, _dp(lo), _dp(hi),
                                        na.ctypes.data_as(C.POINTER(C.c_int64)))
        return lo, hi, na

    def fitness_interval_rounded_many(self, xyz, poses: Sequence, eps=1e-3, qrel=0.0, qabs=0.0):
        """[E_lo, E_hi] over every storage rounding of this volume's values by at most
        qrel |T| + qabs per voxel (and the near-face cell choices within eps)."""
        x = _f64(xyz)
        K = len(poses)
        arr = (Pose * K)(*[Pose.of(R, t) for R, t in poses])
        lo, hi = np.zeros(K), np.zeros(K)
        lib().orc_fitness_interval_rounded_many(C.byref(self.c()), _dp(x), x.shape[0], arr, K, eps, qrel, qabs,
                                                _dp(lo), _dp(hi))
        return lo, hi

    def fitness_grad(self, xyz, R, t, mode=COMPOSE_DECOUPLED):
        x = _f64(xyz)
        E, nv = C.c_double(), C.c_int64()
        g = np.zeros(6)
        lib().orc_fitness_grad(C.byref(self.c()), _dp(x), x.shape[0], C.byref(Pose.of(R, t)), mode, C.byref(E),
                               _dp(g), C.byref(nv))
        return float(E.value), g, int(nv.value)

    def fitness_grad_many(self, xyz, poses, mode=COMPOSE_DECOUPLED):
        x = _f64(xyz)
        B = len(poses)
        arr = (Pose * B)(*[Pose.of(R, t) for R, t in poses])
        E, g, nv = np.zeros(B), np.zeros((B, 6)), np.zeros(B, np.int64)
        lib().orc_fitness_grad_many(C.byref(self.c()), _dp(x), x.shape[0], arr, B, mode, _dp(E), _dp(g),
                                    nv.ctypes.data_as(C.POINTER(C.c_int64)))
        return E, g, nv

    def fitness_grad_interval_many(self, xyz, poses, mode=COMPOSE_DECOUPLED, eps=1e-3, sign_eps=0.0):
        """Per pose, [lo, hi] of (E, grad6) over every cell choice of samples within eps of a face
        and both signs of samples whose value is within sign_eps of 0."""
        x = _f64(xyz)
        B = len(poses)
        arr = (Pose * B)(*[Pose.of(R, t) for R, t in poses])
        lo, hi = np.zeros((B, 7)), np.zeros((B, 7))
        lib().orc_fitness_grad_interval_many(C.byref(self.c()), _dp(x), x.shape[0], arr, B, mode, eps, sign_eps,
                                             _dp(lo), _dp(hi))
        return lo, hi

    def fitness_frozen(self, xyz, R, t, xi, mode=COMPOSE_DECOUPLED):
        x = _f64(xyz)
        xi = _f64(xi).reshape(6)
        return float(lib().orc_fitness_frozen(C.byref(self.c()), _dp(x), x.shape[0], C.byref(Pose.of(R, t)), mode,
                                              _dp(xi)))

    def grad_xi_fd(self, xyz, R, t, xi0, mode=COMPOSE_DECOUPLED, h=1e-6):
        """d/dxi of E(compose(xi, (R, t))) at xi0 (frozen at xi0), by central differences."""
        x = _f64(xyz)
        xi0 = _f64(xi0).reshape(6)
        g = np.zeros(6)
        lib().orc_grad_xi_fd(C.byref(self.c()), _dp(x), x.shape[0], C.byref(Pose.of(R, t)), mode, _dp(xi0), h, _dp(g))
        return g

    def polish(self, xyz, R, t, steps=5, mode=COMPOSE_DECOUPLED):
        x = _f64(xyz)
        P = Pose.of(R, t)
        E = C.c_double()
        acc = lib().orc_polish(C.byref(self.c()), _dp(x), x.shape[0], C.byref(P), mode, steps, C.byref(E))
        R2, t2 = P.rt()
        return R2, t2, int(acc), float(E.value)

    def ro_iteration(self, S, params: "Params", i, R, t, s_rad, s_m):
        x = _f64(S)
        P = Pose.of(R, t)
        sr, sm = C.c_double(s_rad), C.c_double(s_m)
        E = np.zeros(params.K + 1)
        nv = np.zeros(params.K + 1, np.int64)
        rec = IterRec()
        lib().orc_ro_iteration(C.byref(self.c()), _dp(x), x.shape[0], C.byref(params), i, C.byref(P), C.byref(sr),
                               C.byref(sm), _dp(E), nv.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(rec))
        R2, t2 = P.rt()
        return R2, t2, sr.value, sm.value, E, nv, rec

    def track_frame(self, depth, intr, R0, t0, params: "Params"):
        """Randomized optimization of one frame (Sec. III-B with the Sec. IV-A schedule). Returns the
        pose and the records of the iterations that ran (fewer than n_iters after an early exit)."""
        d = np.ascontiguousarray(depth, dtype=np.float32)
        out = Pose()
        recs = (IterRec * max(1, params.n_iters))()
        done = C.c_int32(0)
        n = lib().orc_track_frame(C.byref(self.c()), d.ctypes.data_as(C.POINTER(C.c_float)), C.byref(Intr.of(intr)),
                                  C.byref(Pose.of(R0, t0)), C.byref(params), C.byref(out), recs, C.byref(done))
        if n < 0:
            raise MemoryError("oracle track_frame: allocation failed")
        R, t = out.rt()
        return R, t, [recs[i] for i in range(done.value)]

    def grid_search(self, xyz, R, t, m, rot_step, trans_step, mode=COMPOSE_DECOUPLED):
        x = _f64(xyz)
        E = np.zeros(m ** 6)
        best = lib().orc_grid_search(C.byref(self.c()), _dp(x), x.shape[0], C.byref(Pose.of(R, t)), m, rot_step,
                                     trans_step, mode, _dp(E))
        return int(best), E


def advantage_update(E, deltas, R, t, mode=COMPOSE_DECOUPLED):
    """Advantage set {k : E_k < E_0} and averaged delta applied to (R, t) (Sec. III-B)."""
    E = _f64(E)
    d = _f64(deltas).reshape(-1, 6)
    K = E.shape[0] - 1
    out = Pose()
    mean = np.zeros(6)
    na = lib().orc_advantage_update(_dp(E), _dp(d), K, mode, C.byref(Pose.of(R, t)), C.byref(out), _dp(mean))
    R2, t2 = out.rt()
    return int(na), R2, t2, mean


def best_candidate(Estar, E) -> int:
    """Start of the polish: 0 for the optimized pose (fitness Estar), else the index k >= 1 of the
    last iteration's particle with the lowest fitness E[k]; ties to the pose, then the lowest k."""
    E = _f64(E)
    return int(lib().orc_best_candidate(float(Estar), _dp(E), E.shape[0] - 1))


def make_params(seed=3, frame_index=1, n_iters=10, K=256, rates=(1,), pixel_stride=2, s1_deg=5.0, s1_m=0.03,
                beta=0.1, compose_mode=COMPOSE_DECOUPLED, polish_steps=0, min_valid=0, Ks=None, stop_deg=0.0,
                stop_m=0.0) -> Params:
    """Ks: particle counts paired with the rates (iteration i draws Ks[(i-1) mod n_rates]); stop_deg /
    stop_m: early exit once the updated search size is below both (0 = run all n_iters)."""
    p = Params()
    p.seed, p.frame_index, p.n_iters, p.K = seed, frame_index, n_iters, K
    if Ks is not None:
        assert len(Ks) == len(rates)
        p.alt_K = 1
        p.Ks[:] = (list(Ks) + [0, 0, 0])[:3]
        p.K = max(Ks)
    p.stop_deg, p.stop_m = stop_deg, stop_m
    p.n_rates = len(rates)
    rr = list(rates) + [1] * (3 - len(rates))
    p.rates[:] = rr[:3]
    p.pixel_stride = pixel_stride
    p.s1_deg, p.s1_m, p.beta = s1_deg, s1_m, beta
    p.compose_mode, p.polish_steps, p.min_valid = compose_mode, polish_steps, min_valid
    return p
