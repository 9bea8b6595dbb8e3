"""C-ABI contract checks that need no GPU: the library loads and exports every function the
header declares, the ctypes mirrors match the C struct layouts, and invalid arguments are
rejected with PF_EINVAL (and a message) before anything touches a device."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "profusion.h")


@pytest.fixture(scope="module")
def pf():
    import paper_2509_24236_amd as pf
    if not os.path.exists(pf.LIB_PATH):
        from paper_2509_24236_amd import build
        build.build()
    pf.lib()
    return pf


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\*?\s*([A-Za-z_]\w*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_exports_every_declared_function(pf):
    names = declared_functions()
    assert len(names) >= 13
    L = C.CDLL(pf.LIB_PATH)
    for n in names:
        assert hasattr(L, n), f"{n} declared in profusion.h but not exported"
    assert set(names) == set(pf.EXPORTS)


def test_struct_layouts_match_header(pf):
    structs = {
        "pf_pose": pf.pf_pose, "pf_intrinsics": pf.pf_intrinsics, "pf_tsdf": pf.pf_tsdf,
        "pf_track_params": pf.pf_track_params, "pf_track_stats": pf.pf_track_stats,
        "pf_track_state": pf.pf_track_state, "pf_batch_problem": pf.pf_batch_problem,
        "pf_batch_plan": pf.pf_batch_plan,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append('printf("PF_STATE_DELTAS_OFFSET %d\\n", PF_STATE_DELTAS_OFFSET);')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        open(c, "w").write("\n".join(lines))
        exe = os.path.join(d, "layout")
        subprocess.check_call(["gcc", "-std=c11", "-o", exe, c])
        out = subprocess.check_output([exe], text=True)
    got = dict(l.rsplit(" ", 1) for l in out.strip().splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, f"{name}.{fname}"
    assert int(got["PF_STATE_DELTAS_OFFSET"]) == pf.STATE_DELTAS_OFFSET
    assert C.sizeof(pf.pf_track_state) <= pf.STATE_DELTAS_OFFSET


def _desc(pf, nx=8, ny=8, nz=8, fmt=0, layout=0):
    d = pf.pf_tsdf()
    d.nx, d.ny, d.nz, d.format, d.layout = nx, ny, nz, fmt, layout
    d.voxel_size, d.trunc = 0.01, 0.04
    d.origin[:] = [0.0, 0.0, 0.0]
    d.w_max = 255
    d.tsdf = 0x1000      # never dereferenced: every call below fails validation first
    d.weight = 0x2000
    return d


def test_tsdf_bytes(pf):
    L = pf.lib()
    wb = C.c_size_t()
    for fmt, (tb, wbb) in {0: (4, 4), 1: (2, 1), 2: (2, 1)}.items():
        d = _desc(pf, 16, 8, 4, fmt)
        assert L.tsdf_bytes(C.byref(d), C.byref(wb)) == 16 * 8 * 4 * tb
        assert wb.value == 16 * 8 * 4 * wbb
    for fmt, tb in {0: 4, 1: 2, 2: 2}.items():
        # CELLS: T, the replica, the cell-validity mask (one word per 4x4x4 cells: 4 x 2 x 1 words for
        # 15 x 7 x 3 cells) and one flag byte per word, each part starting on a 256-byte boundary
        d = _desc(pf, 16, 8, 4, fmt, layout=1)
        off = L.tsdf_cells_offset(C.byref(d))
        assert off >= 16 * 8 * 4 * tb and off % 256 == 0
        moff = L.tsdf_mask_offset(C.byref(d))
        assert moff >= off + 15 * 7 * 3 * 8 * tb and moff % 256 == 0 and moff - (off + 15 * 7 * 3 * 8 * tb) < 256
        words = 4 * 2 * 1
        foff = (moff + 8 * words + 255) // 256 * 256
        assert L.tsdf_bytes(C.byref(d), C.byref(wb)) == (foff + words + 255) // 256 * 256
    assert L.tsdf_cells_offset(C.byref(_desc(pf, 16, 8, 4, 0, layout=0))) == 0
    assert L.tsdf_mask_offset(C.byref(_desc(pf, 16, 8, 4, 0, layout=0))) == 0
    assert L.tsdf_mask_offset(None) == 0
    assert L.tsdf_bytes(C.byref(_desc(pf, layout=5)), C.byref(wb)) == 0
    assert L.tsdf_bytes(C.byref(_desc(pf, layout=2)), C.byref(wb)) == 0    # BRICKS without a pool
    d = _desc(pf)
    d.max_bricks = 4
    assert L.tsdf_bytes(C.byref(d), C.byref(wb)) == 0                      # a pool on a dense layout
    d = _desc(pf)
    d.reserved = 1
    assert L.tsdf_bytes(C.byref(d), C.byref(wb)) == 0
    assert L.tsdf_bytes(C.byref(_desc(pf, 1, 8, 8)), C.byref(wb)) == 0
    assert L.tsdf_bytes(C.byref(_desc(pf, fmt=7)), C.byref(wb)) == 0
    assert L.tsdf_bytes(None, None) == 0
    assert L.tsdf_bytes(C.byref(_desc(pf, 2048, 2048, 1024)), None) == 0   # > 2^31 voxels
    assert L.tsdf_bytes(C.byref(_desc(pf, 4096, 4096, 2)), None) == 0      # a slice of 2^24 voxels
    assert L.tsdf_bytes(C.byref(_desc(pf, 4096, 4095, 2)), None) > 0


def _rc(pf, rc, needle):
    assert rc == pf.PF_EINVAL
    assert needle in pf.last_error(), pf.last_error()


def test_validation_rejects_before_launch(pf):
    L = pf.lib()
    _rc(pf, L.tsdf_init(None, None), "null volume")
    _rc(pf, L.tsdf_init(C.byref(_desc(pf, 1, 4, 4)), None), "dims")
    d = _desc(pf)
    d.voxel_size = 0.0
    _rc(pf, L.tsdf_init(C.byref(d), None), "voxel_size")
    d = _desc(pf)
    d.trunc = float("nan")
    _rc(pf, L.tsdf_init(C.byref(d), None), "trunc")
    d = _desc(pf)
    d.w_max = 0
    _rc(pf, L.tsdf_init(C.byref(d), None), "w_max")
    d = _desc(pf)
    d.layout = 5
    _rc(pf, L.tsdf_init(C.byref(d), None), "layout")
    d = _desc(pf)
    d.tsdf = None
    _rc(pf, L.tsdf_init(C.byref(d), None), "null tsdf")
    K = pf.pf_intrinsics(525.0, 525.0, 319.5, 239.5, 640, 480)
    bad_R = pf.make_pose(np.diag([1.0, 1.0, 1.001]), np.zeros(3))
    _rc(pf, L.tsdf_integrate(C.byref(_desc(pf)), C.c_void_p(0x3000), C.byref(K), C.byref(bad_R), None), "rotation")
    refl = pf.make_pose(np.diag([1.0, 1.0, -1.0]), np.zeros(3))
    _rc(pf, L.tsdf_integrate(C.byref(_desc(pf)), C.c_void_p(0x3000), C.byref(K), C.byref(refl), None), "rotation")
    K0 = pf.pf_intrinsics(0.0, 525.0, 319.5, 239.5, 640, 480)
    good = pf.make_pose(np.eye(3), np.zeros(3))
    _rc(pf, L.tsdf_integrate(C.byref(_desc(pf)), C.c_void_p(0x3000), C.byref(K0), C.byref(good), None), "focal")
    _rc(pf, L.tsdf_integrate(C.byref(_desc(pf)), None, C.byref(K), C.byref(good), None), "null depth")
    p = C.c_void_p(0x4000)
    _rc(pf, L.particles_score(C.byref(_desc(pf)), p, p, p, 0, p, 4, p, p, None), "n_pts")
    _rc(pf, L.particles_score(C.byref(_desc(pf)), p, p, p, 1 << 30, p, 4, p, p, None), "n_pts")
    _rc(pf, L.particles_score(C.byref(_desc(pf)), p, p, p, 10, p, 0, p, p, None), "K")
    _rc(pf, L.particles_score(C.byref(_desc(pf)), p, None, p, 10, p, 4, p, p, None), "null pointer")
    _rc(pf, L.particles_update(C.byref(_desc(pf)), p, p, p, 10, p, p, p, 0, p, None), "K")


def test_params_validation(pf):
    L = pf.lib()
    intr = pf.pf_intrinsics(120.0, 120.0, 80.0, 60.0, 160, 120)
    good = pf.TrackParams(K=256, n_iters=10, rates=(1,), pixel_stride=2)
    assert L.track_workspace_bytes(C.byref(intr), C.byref(good.c())) > 0
    for field, val in [("K", 0), ("n_iters", 0), ("n_iters", 65), ("beta", 1.5), ("compose_mode", 2),
                       ("pixel_stride", 0), ("s1_deg", -1.0), ("frame_index", -1), ("polish_steps", 99)]:
        c = good.c()
        setattr(c, field, val)
        assert L.track_workspace_bytes(C.byref(intr), C.byref(c)) == 0, field
    c = good.c()
    c.n_rates = 0
    assert L.track_workspace_bytes(C.byref(intr), C.byref(c)) == 0
    c = good.c()
    c.rates[0] = 0
    assert L.track_workspace_bytes(C.byref(intr), C.byref(c)) == 0
    init = pf.make_pose(np.eye(3), np.zeros(3))
    out = pf.pf_pose()
    p = C.c_void_p(0x4000)
    c = good.c()
    c.K = -3
    rc = L.track_frame(C.byref(_desc(pf)), p, C.byref(intr), C.byref(init), C.byref(c), C.byref(out), None, p,
                       C.c_size_t(1 << 20), None)
    _rc(pf, rc, "K")
    assert L.particles_state_bytes(0) == 0
    # header, then the FP64 deltas at 512, then 256-byte aligned per-workgroup partials
    assert L.particles_state_bytes(10) == 512 + 768 + 2 * 256 * 16
    # the paper's schedule: Ks paired with the rates, each in 1..K; a finite, non-negative stop size
    sched = pf.TrackParams(K=256, n_iters=10, rates=(1, 2, 3), pixel_stride=2, Ks=(64, 128, 256), stop_deg=0.05,
                           stop_m=0.0005)
    assert L.track_workspace_bytes(C.byref(intr), C.byref(sched.c())) > 0
    for field, val in [("alt_K", 2), ("stop_deg", -1.0), ("stop_m", float("nan")), ("stop_deg", float("inf"))]:
        c = sched.c()
        setattr(c, field, val)
        assert L.track_workspace_bytes(C.byref(intr), C.byref(c)) == 0, field
    for r, val in [(0, 0), (1, 257), (2, -1)]:
        c = sched.c()
        c.Ks[r] = val
        assert L.track_workspace_bytes(C.byref(intr), C.byref(c)) == 0, (r, val)
    c = sched.c()
    c.reserved = 1
    assert L.track_workspace_bytes(C.byref(intr), C.byref(c)) == 0


def test_noalloc_rejects_before_launch(pf):
    """track_frame_noalloc validates like track_frame, and refuses a frame whose workspace would not
    fit the library's array with PF_ENOMEM, before touching a device."""
    L = pf.lib()
    init = pf.make_pose(np.eye(3), np.zeros(3))
    out = pf.pf_pose()
    p = C.c_void_p(0x4000)
    intr = pf.pf_intrinsics(120.0, 120.0, 80.0, 60.0, 160, 120)
    c = pf.TrackParams(K=256, n_iters=10, rates=(1,), pixel_stride=2).c()
    c.K = -3
    _rc(pf, L.track_frame_noalloc(C.byref(_desc(pf)), p, C.byref(intr), C.byref(init), C.byref(c), C.byref(out),
                                  None, None), "K")
    c.K = 256
    _rc(pf, L.track_frame_noalloc(C.byref(_desc(pf)), None, C.byref(intr), C.byref(init), C.byref(c), C.byref(out),
                                  None, None), "null")
    big = pf.pf_intrinsics(1000.0, 1000.0, 960.0, 540.0, 1920, 1080)
    c = pf.TrackParams(K=65536, n_iters=20, rates=(8, 16, 32), pixel_stride=1).c()
    need = L.track_workspace_bytes(C.byref(big), C.byref(c))
    assert need > pf.NOALLOC_WORKSPACE_BYTES
    rc = L.track_frame_noalloc(C.byref(_desc(pf)), p, C.byref(big), C.byref(init), C.byref(c), C.byref(out), None,
                               None)
    assert rc == pf.PF_ENOMEM
    assert str(need) in pf.last_error() and "array holds" in pf.last_error()
    # the largest frame the header promises fits: 1280x960 at the maximum particle count
    c960 = pf.pf_intrinsics(700.0, 700.0, 640.0, 480.0, 1280, 960)
    assert 0 < L.track_workspace_bytes(C.byref(c960), C.byref(c)) <= pf.NOALLOC_WORKSPACE_BYTES


def test_batch_validation(pf):
    L = pf.lib()
    q = (pf.pf_batch_problem * 2)()
    for i in range(2):
        q[i].vol = _desc(pf, 16, 16, 16, 0, 1)
        q[i].depth = 0x5000
        q[i].K = pf.pf_intrinsics(100.0, 100.0, 40.0, 30.0, 80, 60)
        q[i].init = pf.make_pose(np.eye(3), np.zeros(3))
        q[i].params = pf.TrackParams(K=256, n_iters=4, rates=(1,), pixel_stride=2).c()
    assert L.track_batch_workspace_bytes(q, 2) > 0
    q[1].params.K = 32                         # batching needs K >= 64
    assert L.track_batch_workspace_bytes(q, 2) == 0
    assert "K 32 < 64" in pf.last_error()
    q[1].params.K = 256
    q[1].params.stop_deg, q[1].params.stop_m = 0.05, 0.0005     # the stop rule is not batched
    assert L.track_batch_workspace_bytes(q, 2) == 0
    assert "not batched" in pf.last_error()
    q[1].params.stop_deg, q[1].params.stop_m = 0.0, 0.0
    q[1].params.polish_steps = 2               # polish is batched, with the same step count everywhere
    assert L.track_batch_workspace_bytes(q, 2) > 0
    h = L.track_batch_create(q, 2, C.byref(pf.pf_batch_plan(4, 1024, 1, 0)), C.c_void_p(0x6000),
                             C.c_size_t(1 << 30), None)
    assert not h and "differs" in pf.last_error()
    q[1].params.polish_steps = 0
    for tk in (3, -1, 16):                     # 0 (automatic) and 1, 2, 4, 8 are the plans
        bad = pf.pf_batch_plan(tk, 1024, 0, 0)
        h = L.track_batch_create(q, 2, C.byref(bad), C.c_void_p(0x6000), C.c_size_t(1 << 30), None)
        assert not h and "score_tk" in pf.last_error()
    q[1].params.n_iters = 5                    # all problems must share n_iters
    ok = pf.pf_batch_plan(0, 1024, 1, 0)
    h = L.track_batch_create(q, 2, C.byref(ok), C.c_void_p(0x6000), C.c_size_t(1 << 30), None)
    assert not h and "differs" in pf.last_error()
    assert L.track_batch_run(None, None) == pf.PF_EINVAL


def test_score_config_validation(pf):
    """Launch shapes: 0/0 (automatic) and the listed shapes are accepted; anything else is
    rejected with PF_EINVAL. The call is host-only."""
    L = pf.lib()
    try:
        for tk, blk in [(0, 0), (1, 256), (1, 512), (2, 64), (4, 128), (8, 512)]:
            assert L.pf_score_config(tk, blk) == pf.PF_OK, (tk, blk)
        for tk, blk in [(3, 256), (4, 96), (1, 128), (1, 64), (0, 256), (16, 256), (-1, 256)]:
            assert L.pf_score_config(tk, blk) == pf.PF_EINVAL, (tk, blk)
            assert b"pf_score_config" in L.pf_last_error()
    finally:
        L.pf_score_config(0, 0)


def _al(x):
    return (x + 255) // 256 * 256


def test_brick_pool_bytes_and_offsets(pf):
    """BRICKS: 256-byte header, index grid, slot coordinates, the slots' T and cells in the T
    buffer, the slots' W in the W buffer; dims must be multiples of 8 and the pool non-empty."""
    L = pf.lib()
    wb = C.c_size_t()
    for fmt, (tb, wbb) in {0: (4, 4), 1: (2, 1), 2: (2, 1)}.items():
        d = _desc(pf, 64, 40, 24, fmt, layout=2)
        d.max_bricks = 37
        nb = 8 * 5 * 3
        o = [C.c_size_t() for _ in range(4)]
        assert L.tsdf_brick_offsets(C.byref(d), *[C.byref(x) for x in o]) == pf.PF_OK
        index, coords, pool_t, pool_cells = (x.value for x in o)
        assert index == 256
        assert coords == index + 2 * _al(nb * 4)          # the index grid, then the candidate list
        assert pool_t == coords + _al(37 * 16)
        assert pool_cells == pool_t + _al(37 * 512 * tb)
        pool_mask = L.tsdf_mask_offset(C.byref(d))        # 8 cell-validity words per slot
        assert pool_mask == pool_cells + _al(37 * 512 * 8 * tb)
        assert L.tsdf_bytes(C.byref(d), C.byref(wb)) == pool_mask + 37 * 8 * 8
        assert wb.value == 37 * 512 * wbb
        assert all(x % 256 == 0 for x in (index, coords, pool_t, pool_cells))
    for nx, ny, nz, mb in ((60, 40, 24, 4), (64, 40, 20, 4), (64, 40, 24, 0), (64, 40, 24, -1),
                           (64, 40, 24, (1 << 23) + 1)):
        d = _desc(pf, nx, ny, nz, 0, layout=2)
        d.max_bricks = mb
        assert L.tsdf_bytes(C.byref(d), C.byref(wb)) == 0
        _rc(pf, L.tsdf_init(C.byref(d), None), "BRICKS")
        _rc(pf, L.tsdf_brick_offsets(C.byref(d), None, None, None, None), "BRICKS")
    # larger than a dense grid may be: 4096^3 voxels, 2^27 index entries
    d = _desc(pf, 4096, 4096, 4096, 1, layout=2)
    d.max_bricks = 1 << 20
    assert L.tsdf_bytes(C.byref(d), C.byref(wb)) > 0
    d = _desc(pf, 8, 8, 8, 0, layout=1)
    _rc(pf, L.tsdf_brick_offsets(C.byref(d), None, None, None, None), "BRICKS")
    _rc(pf, L.tsdf_bricks_used(C.byref(d), None, None, None), "BRICKS")
    d = _desc(pf, 8, 8, 8, 0, layout=1)
    d.reserved = 3
    _rc(pf, L.tsdf_init(C.byref(d), None), "reserved")
