"""Python binding of libprofusion.so, the gfx950 HIP library for PROFusion's tracking-and-fusion
hot path (arXiv 2509.24236): particle-based pose optimization against a TSDF (Sec. III-B) and
KinectFusion-style TSDF fusion (Sec. III overview).

Argument marshalling only: every step runs in the library's HIP kernels. torch supplies device
memory and the current stream. The binding fails loudly when the library is missing; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprofusion.so")

PF_OK, PF_EINVAL, PF_ENOMEM, PF_EHIP, PF_EUNSUPPORTED = 0, -1, -2, -3, -4
F32_W_F32, F16_W_U8, I16_W_U8 = 0, 1, 2
COMPOSE_DECOUPLED, COMPOSE_LITERAL = 0, 1
MAX_ITERS = 64
LAYOUT_LINEAR, LAYOUT_CELLS, LAYOUT_BRICKS = 0, 1, 2
STATE_DELTAS_OFFSET = 512


class PFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


# ----------------------------------------------------------------------------- ABI structs
class pf_pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class pf_intrinsics(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32)]


class pf_tsdf(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("format", C.c_int32),
                ("voxel_size", C.c_double), ("trunc", C.c_double), ("origin", C.c_double * 3),
                ("w_max", C.c_int32), ("layout", C.c_int32), ("max_bricks", C.c_int32), ("reserved", C.c_int32),
                ("tsdf", C.c_void_p), ("weight", C.c_void_p)]


class pf_track_params(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("frame_index", C.c_int32), ("n_iters", C.c_int32), ("K", C.c_int32),
                ("n_rates", C.c_int32), ("rates", C.c_int32 * 3), ("pixel_stride", C.c_int32),
                ("s1_deg", C.c_double), ("s1_m", C.c_double), ("beta", C.c_double), ("compose_mode", C.c_int32),
                ("polish_steps", C.c_int32), ("min_valid", C.c_int32), ("alt_K", C.c_int32), ("Ks", C.c_int32 * 3),
                ("reserved", C.c_int32), ("stop_deg", C.c_double), ("stop_m", C.c_double)]


class pf_track_stats(C.Structure):
    _fields_ = [("n_points", C.c_int32), ("n_iters", C.c_int32), ("lost", C.c_int32),
                ("polish_accepted", C.c_int32), ("E0", C.c_float * MAX_ITERS), ("Estar", C.c_float * MAX_ITERS),
                ("n_adv", C.c_int32 * MAX_ITERS), ("n_sub", C.c_int32 * MAX_ITERS),
                ("n_valid", C.c_int32 * MAX_ITERS), ("s_rad", C.c_double * MAX_ITERS),
                ("s_m", C.c_double * MAX_ITERS), ("E_final", C.c_float), ("n_valid_final", C.c_int32),
                ("n_particles", C.c_int32 * MAX_ITERS)]


class pf_track_state(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("s_rad", C.c_double), ("s_m", C.c_double),
                ("R_new", C.c_double * 9), ("t_new", C.c_double * 3), ("s_rad_done", C.c_double),
                ("s_m_done", C.c_double), ("E0", C.c_double), ("Estar", C.c_double), ("mean", C.c_double * 6),
                ("R_prev", C.c_double * 9), ("t_prev", C.c_double * 3), ("beta", C.c_double), ("seed", C.c_uint64), ("frame_index", C.c_int32), ("iter", C.c_int32),
                ("iter_done", C.c_int32), ("K", C.c_int32), ("compose_mode", C.c_int32), ("n_adv", C.c_int32),
                ("n_sub", C.c_int32), ("n_valid_star", C.c_int32), ("flags", C.c_int32), ("K_cur", C.c_int32),
                ("done", C.c_int32), ("alt_K", C.c_int32), ("n_rates", C.c_int32), ("Ks", C.c_int32 * 3),
                ("reserved", C.c_int32), ("stop_rad", C.c_double), ("stop_m", C.c_double)]


class pf_batch_problem(C.Structure):
    _fields_ = [("vol", pf_tsdf), ("depth", C.c_void_p), ("K", pf_intrinsics), ("init", pf_pose),
                ("params", pf_track_params)]


class pf_batch_plan(C.Structure):
    _fields_ = [("score_tk", C.c_int32), ("score_grid", C.c_int32), ("order", C.c_int32), ("reserved", C.c_int32)]


# every symbol include/profusion.h declares
EXPORTS = ("pf_last_error", "tsdf_bytes", "tsdf_cells_offset", "tsdf_mask_offset", "tsdf_brick_offsets", "tsdf_bricks_used", "tsdf_init", "tsdf_integrate", "tsdf_export_linear", "tsdf_import_linear",
           "backproject", "particles_score", "particles_score_grad", "pf_score_config", "pf_score_mask", "particles_state_bytes", "particles_state_init", "particles_update",
           "track_workspace_bytes", "track_frame", "track_frame_fuse", "track_frame_noalloc", "track_batch_workspace_bytes", "track_batch_create",
           "track_batch_run", "track_batch_results", "track_batch_destroy", "pf_timing_enable", "pf_timing_read")

_lib = None


def lib() -> C.CDLL:
    """Loads libprofusion.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(paper_2509_24236_amd/build.py); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp, i32, P = C.c_void_p, C.c_int32, C.POINTER
    L.pf_last_error.restype = C.c_char_p
    L.tsdf_bytes.restype = C.c_size_t
    L.tsdf_bytes.argtypes = [P(pf_tsdf), P(C.c_size_t)]
    L.tsdf_cells_offset.restype = C.c_size_t
    L.tsdf_cells_offset.argtypes = [P(pf_tsdf)]
    L.tsdf_mask_offset.restype = C.c_size_t
    L.tsdf_mask_offset.argtypes = [P(pf_tsdf)]
    L.tsdf_brick_offsets.argtypes = [P(pf_tsdf), P(C.c_size_t), P(C.c_size_t), P(C.c_size_t), P(C.c_size_t)]
    L.tsdf_bricks_used.argtypes = [P(pf_tsdf), P(C.c_int32), P(C.c_int32), vp]
    for name in ("tsdf_init",):
        getattr(L, name).argtypes = [P(pf_tsdf), vp]
    L.tsdf_integrate.argtypes = [P(pf_tsdf), vp, P(pf_intrinsics), P(pf_pose), vp]
    L.tsdf_export_linear.argtypes = [P(pf_tsdf), vp, vp, vp]
    L.tsdf_import_linear.argtypes = [P(pf_tsdf), vp, vp, vp]
    L.backproject.argtypes = [vp, P(pf_intrinsics), i32, vp, vp, vp, vp, vp]
    L.particles_score.argtypes = [P(pf_tsdf), vp, vp, vp, i32, vp, i32, vp, vp, vp]
    L.particles_score_grad.argtypes = [P(pf_tsdf), vp, vp, vp, i32, vp, vp, i32, i32, vp, vp, vp, vp]
    L.pf_score_config.argtypes = [i32, i32]
    L.pf_score_mask.argtypes = [i32]
    L.particles_state_bytes.restype = C.c_size_t
    L.particles_state_bytes.argtypes = [i32]
    L.particles_state_init.argtypes = [vp, P(pf_pose), P(pf_track_params), vp, vp]
    L.particles_update.argtypes = [P(pf_tsdf), vp, vp, vp, i32, vp, vp, vp, i32, vp, vp]
    L.track_workspace_bytes.restype = C.c_size_t
    L.track_workspace_bytes.argtypes = [P(pf_intrinsics), P(pf_track_params)]
    L.track_frame.argtypes = [P(pf_tsdf), vp, P(pf_intrinsics), P(pf_pose), P(pf_track_params), P(pf_pose),
                              P(pf_track_stats), vp, C.c_size_t, vp]
    L.track_frame_fuse.argtypes = L.track_frame.argtypes
    L.track_frame_noalloc.argtypes = [P(pf_tsdf), vp, P(pf_intrinsics), P(pf_pose), P(pf_track_params), P(pf_pose),
                                      P(pf_track_stats), vp]
    L.track_batch_workspace_bytes.restype = C.c_size_t
    L.track_batch_workspace_bytes.argtypes = [P(pf_batch_problem), i32]
    L.track_batch_create.restype = vp
    L.track_batch_create.argtypes = [P(pf_batch_problem), i32, P(pf_batch_plan), vp, C.c_size_t, vp]
    L.track_batch_run.argtypes = [vp, vp]
    L.track_batch_results.argtypes = [vp, P(pf_pose), P(pf_track_stats), vp]
    L.track_batch_destroy.restype = None
    L.track_batch_destroy.argtypes = [vp]
    L.pf_timing_enable.argtypes = [i32]
    L.pf_timing_read.argtypes = [P(C.c_double), P(C.c_int64), P(C.c_int64), i32]
    for name in EXPORTS:
        if name not in ("pf_last_error", "track_batch_destroy") and getattr(L, name).restype is None:
            getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def _check(rc: int):
    if rc != PF_OK:
        raise PFError(rc, lib().pf_last_error().decode())


def last_error() -> str:
    return lib().pf_last_error().decode()


# ----------------------------------------------------------------------------- helpers
def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def make_pose(R, t) -> pf_pose:
    p = pf_pose()
    p.R[:] = [float(x) for x in np.asarray(R, np.float64).reshape(9)]
    p.t[:] = [float(x) for x in np.asarray(t, np.float64).reshape(3)]
    return p


def pose_rt(p: pf_pose) -> Tuple[np.ndarray, np.ndarray]:
    return np.array(p.R[:], np.float64).reshape(3, 3), np.array(p.t[:], np.float64)


def make_intrinsics(k) -> pf_intrinsics:
    return pf_intrinsics(float(k.fx), float(k.fy), float(k.cx), float(k.cy), int(k.width), int(k.height))


@dataclasses.dataclass
class TrackParams:
    seed: int = 3
    frame_index: int = 1
    n_iters: int = 20
    K: int = 3072
    rates: Sequence[int] = (8, 16, 32)
    pixel_stride: int = 1
    s1_deg: float = 10.0
    s1_m: float = 0.10
    beta: float = 0.1
    compose_mode: int = COMPOSE_DECOUPLED
    polish_steps: int = 0
    min_valid: int = 0
    Ks: Optional[Sequence[int]] = None   # particle counts paired with the rates (Sec. IV-A alternation)
    stop_deg: float = 0.0                # early exit once s^(i+1) is below (stop_deg, stop_m); 0 = never
    stop_m: float = 0.0

    def c(self) -> pf_track_params:
        p = pf_track_params()
        p.seed, p.frame_index, p.n_iters, p.K = self.seed, self.frame_index, self.n_iters, self.K
        if self.Ks is not None:
            if len(self.Ks) != len(self.rates):
                raise ValueError("Ks pairs with the rates: give one particle count per rate")
            p.alt_K = 1
            p.Ks[:] = (list(self.Ks) + [0, 0, 0])[:3]
            p.K = max(self.Ks)
        p.stop_deg, p.stop_m = self.stop_deg, self.stop_m
        p.n_rates = len(self.rates)
        rr = list(self.rates) + [1] * (3 - len(self.rates))
        p.rates[:] = rr[:3]
        p.pixel_stride = self.pixel_stride
        p.s1_deg, p.s1_m, p.beta = self.s1_deg, self.s1_m, self.beta
        p.compose_mode, p.polish_steps, p.min_valid, p.reserved = self.compose_mode, self.polish_steps, self.min_valid, 0
        return p


# ----------------------------------------------------------------------------- volume
_T_DTYPE = {F32_W_F32: "float32", F16_W_U8: "float16", I16_W_U8: "int16"}
_W_DTYPE = {F32_W_F32: "float32", F16_W_U8: "uint8", I16_W_U8: "uint8"}


class Tsdf:
    """A device TSDF volume: torch tensors for T and W plus the pf_tsdf descriptor."""

    def __init__(self, spec, fmt: int = F32_W_F32, w_max: int = 255, device="cuda", init=True, stream=None,
                 layout: int = LAYOUT_CELLS, max_bricks: int = 0):
        torch = _torch()
        self.spec, self.format, self.layout = spec, fmt, layout
        d = pf_tsdf()
        d.nx, d.ny, d.nz, d.format = spec.nx, spec.ny, spec.nz, fmt
        d.voxel_size, d.trunc = float(spec.voxel_size), float(spec.trunc)
        d.origin[:] = [float(x) for x in spec.origin]
        d.w_max, d.layout, d.max_bricks = w_max, layout, max_bricks
        wb = C.c_size_t(0)
        tb = lib().tsdf_bytes(C.byref(d), C.byref(wb))
        if tb == 0:
            raise PFError(PF_EINVAL, "invalid volume description")
        n = spec.nx * spec.ny * spec.nz
        tdt, wdt = getattr(torch, _T_DTYPE[fmt]), getattr(torch, _W_DTYPE[fmt])
        self.T = torch.empty(tb // torch.tensor([], dtype=tdt).element_size(), dtype=tdt, device=device)
        self.W = torch.empty(wb.value // torch.tensor([], dtype=wdt).element_size(), dtype=wdt, device=device)
        assert layout == LAYOUT_BRICKS or (self.T.numel() >= n and self.W.numel() >= n)
        d.tsdf, d.weight = self.T.data_ptr(), self.W.data_ptr()
        self.desc = d
        if init:
            self.init(stream)

    def init(self, stream=None):
        _check(lib().tsdf_init(C.byref(self.desc), _stream(stream)))

    def integrate(self, depth, intr, R, t, stream=None):
        """KinectFusion-style fusion of one aligned frame (Sec. III overview)."""
        _check(lib().tsdf_integrate(C.byref(self.desc), _ptr(depth), C.byref(make_intrinsics(intr)),
                                    C.byref(make_pose(R, t)), _stream(stream)))

    def bricks_used(self, stream=None):
        """BRICKS: (bricks in use, overflow flag); synchronises the stream."""
        n, ov = C.c_int32(0), C.c_int32(0)
        _check(lib().tsdf_bricks_used(C.byref(self.desc), C.byref(n), C.byref(ov), _stream(stream)))
        return int(n.value), int(ov.value)

    def brick_offsets(self):
        """BRICKS: byte offsets in the T buffer of (index grid, slot coordinates, slots' T, slots' cells)."""
        o = [C.c_size_t(0) for _ in range(4)]
        _check(lib().tsdf_brick_offsets(C.byref(self.desc), *[C.byref(x) for x in o]))
        return tuple(int(x.value) for x in o)

    def cell_mask(self):
        """CELLS: the cell-validity mask words, (mwz, mwy, mwx) int64 (a view of the T buffer), and the
        per-word flag bytes (all 0 between calls)."""
        torch = _torch()
        off = lib().tsdf_mask_offset(C.byref(self.desc))
        if self.layout != LAYOUT_CELLS or off == 0:
            raise PFError(PF_EINVAL, "cell_mask: not a CELLS volume")
        m = [(n - 1 + 3) // 4 for n in (self.spec.nz, self.spec.ny, self.spec.nx)]
        words = m[0] * m[1] * m[2]
        raw = self.T.view(torch.uint8)
        foff = (off + 8 * words + 255) // 256 * 256
        return raw[off:off + 8 * words].view(torch.int64).view(*m), raw[foff:foff + words].view(*m)

    def export_linear(self, with_weight=True, stream=None):
        torch = _torch()
        n = self.spec.nx * self.spec.ny * self.spec.nz
        To = torch.empty(n, dtype=torch.float32, device=self.T.device)
        Wo = torch.empty(n, dtype=torch.float32, device=self.T.device) if with_weight else None
        _check(lib().tsdf_export_linear(C.byref(self.desc), _ptr(To), _ptr(Wo), _stream(stream)))
        shape = (self.spec.nz, self.spec.ny, self.spec.nx)
        return To.view(shape), (Wo.view(shape) if Wo is not None else None)

    def import_linear(self, T, W=None, stream=None):
        torch = _torch()
        Ti = torch.as_tensor(np.ascontiguousarray(T, np.float32).reshape(-1)).to(self.T.device) \
            if not hasattr(T, "is_cuda") else T.reshape(-1).contiguous().float()
        Wi = None
        if W is not None:
            Wi = torch.as_tensor(np.ascontiguousarray(W, np.float32).reshape(-1)).to(self.T.device) \
                if not hasattr(W, "is_cuda") else W.reshape(-1).contiguous().float()
        _check(lib().tsdf_import_linear(C.byref(self.desc), _ptr(Ti), _ptr(Wi), _stream(stream)))


# ----------------------------------------------------------------------------- points and particles
def backproject(depth, intr, pixel_stride=1, stream=None):
    """Compacted raster-order point cloud of a depth image: (px, py, pz, n_dev) device tensors."""
    torch = _torch()
    npix = intr.width * intr.height
    dev = depth.device
    px = torch.empty(npix, dtype=torch.float32, device=dev)
    py = torch.empty_like(px)
    pz = torch.empty_like(px)
    n = torch.zeros(1 + (npix + 1023) // 1024, dtype=torch.int32, device=dev)
    _check(lib().backproject(_ptr(depth), C.byref(make_intrinsics(intr)), pixel_stride, _ptr(px), _ptr(py), _ptr(pz),
                             _ptr(n), _stream(stream)))
    return px, py, pz, n


def particles_score(vol: Tsdf, px, py, pz, poses, fitness=None, n_valid=None, n_pts=None, stream=None):
    """Fitness of each pose [K][12] float32 (Sec. III-B fitness equation): (fitness, n_valid)."""
    torch = _torch()
    K = poses.shape[0]
    n = int(px.numel() if n_pts is None else n_pts)
    if fitness is None:
        fitness = torch.empty(K, dtype=torch.float32, device=poses.device)
    if n_valid is None:
        n_valid = torch.empty(K, dtype=torch.int32, device=poses.device)
    _check(lib().particles_score(C.byref(vol.desc), _ptr(px), _ptr(py), _ptr(pz), n, _ptr(poses), K, _ptr(fitness),
                                 _ptr(n_valid), _stream(stream)))
    return fitness, n_valid


def particles_score_grad(vol: Tsdf, px, py, pz, base, xi=None, mode=COMPOSE_DECOUPLED, n_pts=None, stream=None):
    """E and dE/dxi for poses compose(xi_b, base_b) (base: [B][12] float64 [R | t]; xi: [B][6] float64
    (rho, phi) or None): returns (fitness [B], grad [B][6], n_valid [B])."""
    torch = _torch()
    B = base.shape[0]
    n = int(px.numel() if n_pts is None else n_pts)
    if base.dtype != torch.float64 or (xi is not None and xi.dtype != torch.float64):
        raise ValueError("base and xi must be float64")
    E = torch.empty(B, dtype=torch.float32, device=base.device)
    g = torch.empty((B, 6), dtype=torch.float32, device=base.device)
    nv = torch.empty(B, dtype=torch.int32, device=base.device)
    _check(lib().particles_score_grad(C.byref(vol.desc), _ptr(px), _ptr(py), _ptr(pz), n, _ptr(base), _ptr(xi), B,
                                      mode, _ptr(E), _ptr(g), _ptr(nv), _stream(stream)))
    return E, g, nv


def _fitness_fn():
    torch = _torch()

    class FitnessFn(torch.autograd.Function):
        """E(compose(xi, base)) with the hand-written adjoint as its backward.

        forward(xi [B][6] float64, base [B][12] float64, vol, px, py, pz, mode) -> E [B] float64.
        The backward multiplies the upstream gradient into the adjoint's dE/dxi (frozen valid set)."""

        @staticmethod
        def forward(ctx, xi, base, vol, px, py, pz, mode=COMPOSE_DECOUPLED):
            E, g, _ = particles_score_grad(vol, px, py, pz, base.contiguous(), xi.detach().contiguous(), mode)
            ctx.save_for_backward(g)
            return E.to(xi.dtype)

        @staticmethod
        def backward(ctx, gE):
            (g,) = ctx.saved_tensors
            return gE[:, None] * g.to(gE.dtype), None, None, None, None, None, None

    return FitnessFn


_FitnessFn = None


def fitness(xi, base, vol, px, py, pz, mode=COMPOSE_DECOUPLED):
    """Differentiable fitness (torch.autograd.Function backed by particles_score_grad)."""
    global _FitnessFn
    if _FitnessFn is None:
        _FitnessFn = _fitness_fn()
    return _FitnessFn.apply(xi, base, vol, px, py, pz, mode)


def score_config(poses_per_group: int = 0, group_size: int = 0):
    """Launch shape of the many-pose scoring launches (process-wide); 0, 0 = automatic."""
    _check(lib().pf_score_config(poses_per_group, group_size))


MASK_BY_SPREAD, MASK_ALWAYS, MASK_NEVER = 0, 1, 2


def score_mask(mode: int = MASK_BY_SPREAD):
    """When automatic scoring launches read the cell-validity mask (process-wide); speed only."""
    _check(lib().pf_score_mask(mode))


def state_bytes(K: int) -> int:
    return int(lib().particles_state_bytes(K))


def particles_state_init(state, R, t, params: TrackParams, next_poses, stream=None):
    _check(lib().particles_state_init(_ptr(state), C.byref(make_pose(R, t)), C.byref(params.c()), _ptr(next_poses),
                                      _stream(stream)))


def particles_update(vol: Tsdf, px, py, pz, fitness, n_valid, state, K, next_poses, n_pts=None, stream=None):
    n = int(px.numel() if n_pts is None else n_pts)
    _check(lib().particles_update(C.byref(vol.desc), _ptr(px), _ptr(py), _ptr(pz), n, _ptr(fitness), _ptr(n_valid),
                                  _ptr(state), K, _ptr(next_poses), _stream(stream)))


def read_state(state) -> pf_track_state:
    """Copies the header of a device state buffer to the host (synchronising)."""
    raw = state[:C.sizeof(pf_track_state)].cpu().numpy().tobytes()
    return pf_track_state.from_buffer_copy(raw)


def read_deltas(state, K):
    torch = _torch()
    b = state[STATE_DELTAS_OFFSET:STATE_DELTAS_OFFSET + (K + 1) * 48].cpu().numpy()
    return np.frombuffer(b.tobytes(), dtype=np.float64).reshape(K + 1, 6)


def track_workspace_bytes(intr, params: TrackParams) -> int:
    return int(lib().track_workspace_bytes(C.byref(make_intrinsics(intr)), C.byref(params.c())))


class Tracker:
    """Holds the workspace of track_frame for one image size and parameter set."""

    def __init__(self, intr, params: TrackParams, device="cuda"):
        torch = _torch()
        self.intr, self.params = intr, params
        self.ws_bytes = track_workspace_bytes(intr, params)
        if self.ws_bytes == 0:
            raise PFError(PF_EINVAL, last_error())
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self._intr_c = make_intrinsics(intr)
        self._params_c = params.c()

    def set_frame(self, frame_index: int):
        self.params.frame_index = frame_index
        self._params_c.frame_index = frame_index

    def track(self, vol: Tsdf, depth, R0, t0, stream=None):
        """Randomized optimization of one frame (Sec. III-B): returns (R, t, stats)."""
        out = pf_pose()
        st = pf_track_stats()
        _check(lib().track_frame(C.byref(vol.desc), _ptr(depth), C.byref(self._intr_c), C.byref(make_pose(R0, t0)),
                                 C.byref(self._params_c), C.byref(out), C.byref(st), _ptr(self.ws),
                                 C.c_size_t(self.ws_bytes), _stream(stream)))
        R, t = pose_rt(out)
        return R, t, st

    def track_fuse(self, vol: Tsdf, depth, R0, t0, stream=None):
        """Tracks the frame, then fuses it into `vol` at the tracked pose (track_frame_fuse: the
        fusion of a dense volume is enqueued on the device before the call waits for its
        result): returns (R, t, stats)."""
        out = pf_pose()
        st = pf_track_stats()
        _check(lib().track_frame_fuse(C.byref(vol.desc), _ptr(depth), C.byref(self._intr_c),
                                      C.byref(make_pose(R0, t0)), C.byref(self._params_c), C.byref(out), C.byref(st),
                                      _ptr(self.ws), C.c_size_t(self.ws_bytes), _stream(stream)))
        R, t = pose_rt(out)
        return R, t, st


NOALLOC_WORKSPACE_BYTES = 32 << 20   # PF_NOALLOC_WORKSPACE_BYTES


def track_frame_noalloc(vol: Tsdf, depth, intr, R0, t0, params: TrackParams, stream=None):
    """track_frame with the library's own per-GPU workspace array (no caller workspace, no
    allocation): returns (R, t, stats)."""
    out = pf_pose()
    st = pf_track_stats()
    _check(lib().track_frame_noalloc(C.byref(vol.desc), _ptr(depth), C.byref(make_intrinsics(intr)),
                                     C.byref(make_pose(R0, t0)), C.byref(params.c()), C.byref(out), C.byref(st),
                                     _stream(stream)))
    R, t = pose_rt(out)
    return R, t, st


def poses_to_f32(poses: Sequence[Tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    """Host helper: list of (R, t) -> [K][12] float32 row-major [R | t]."""
    out = np.zeros((len(poses), 12), np.float32)
    for k, (R, t) in enumerate(poses):
        M = np.concatenate([np.asarray(R, np.float64), np.asarray(t, np.float64).reshape(3, 1)], 1)
        out[k] = M.reshape(12).astype(np.float32)
    return out


def timing_enable(on: bool = True):
    """Brackets track_frame's scoring launches with HIP events on the call's stream."""
    _check(lib().pf_timing_enable(1 if on else 0))


def timing_read(reset: bool = False):
    """(summed scoring-kernel ms, launches, evaluated samples) since the last reset."""
    ms, nl, ne = C.c_double(), C.c_int64(), C.c_int64()
    _check(lib().pf_timing_read(C.byref(ms), C.byref(nl), C.byref(ne), 1 if reset else 0))
    return ms.value, nl.value, ne.value


# ----------------------------------------------------------------------------- batches
@dataclasses.dataclass
class BatchPlan:
    score_tk: int = 4        # poses per 256-thread workgroup (1, 2, 4, 8), or 0: track_frame's automatic shape (4)
    score_grid: int = 4096
    order: int = 1

    def c(self) -> pf_batch_plan:
        return pf_batch_plan(self.score_tk, self.score_grid, self.order, 0)


class Batch:
    """Many tracking problems run as one fixed kernel sequence (track_batch_*).

    problems: list of (Tsdf, depth tensor, intrinsics, R0, t0, TrackParams)."""

    def __init__(self, problems, plan: Optional[BatchPlan] = None, device="cuda", stream=None):
        torch = _torch()
        self.plan = plan or BatchPlan()
        n = len(problems)
        arr = (pf_batch_problem * n)()
        self._keep = []
        for i, (vol, depth, intr, R0, t0, prm) in enumerate(problems):
            arr[i].vol = vol.desc
            arr[i].depth = _ptr(depth).value
            arr[i].K = make_intrinsics(intr)
            arr[i].init = make_pose(R0, t0)
            arr[i].params = prm.c()
            self._keep.append((vol, depth))
        self._arr, self.n = arr, n
        self.ws_bytes = int(lib().track_batch_workspace_bytes(arr, n))
        if self.ws_bytes == 0:
            raise PFError(PF_EINVAL, last_error())
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        h = lib().track_batch_create(arr, n, C.byref(self.plan.c()), _ptr(self.ws), C.c_size_t(self.ws_bytes),
                                     _stream(stream))
        if not h:
            raise PFError(PF_EINVAL, last_error())
        self._h = C.c_void_p(h)

    def run(self, stream=None):
        """Enqueues the whole batch (kernels only; capturable into a HIP graph)."""
        _check(lib().track_batch_run(self._h, _stream(stream)))

    def results(self, stream=None):
        out = (pf_pose * self.n)()
        st = (pf_track_stats * self.n)()
        _check(lib().track_batch_results(self._h, out, st, _stream(stream)))
        return [(*pose_rt(out[i]), st[i]) for i in range(self.n)]

    def close(self):
        if getattr(self, "_h", None):
            lib().track_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
