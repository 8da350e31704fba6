"""Host-side contract of the C ABI (no GPU needed): the library loads, exports
every entry point include/omnigs.h declares, and rejects bad arguments and
allocator failures before any device work."""
import ctypes
import os
import re

import pytest

from paper_2404_03202_amd import omnigs as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "omnigs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(omnigs_\w+)\s*\(", hdr)) - {"omnigs_alloc_fn"})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libomnigs.so is not built: run `python -m paper_2404_03202_amd.build`")
    return B.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), f"{name} declared in omnigs.h but not exported"
    assert set(names) == set(B.EXPORTS)


def test_default_settings(lib):
    s = B.omnigs_default_settings()
    assert s["alpha_min"] == pytest.approx(1 / 255)
    assert s["alpha_max"] == 0.99 and s["T_min"] == 1e-4 and s["dilation"] == 0.3 and s["near_plane"] == 0.2
    assert tuple(s["bg"]) == (0.0, 0.0, 0.0)


def _fake_args(n=10, width=64, height=32, degree=3, coeffs=16):
    # non-null, 16-byte aligned fake device addresses: validation and
    # allocation failures are reported before any pointer is dereferenced
    g = B.c_gaussians(0x10000, 0x20000, 0x30000, 0x40000, 0x50000, n, degree, coeffs)
    c = B.c_camera()
    for k in range(9):
        c.R_cw[k] = 1.0 if k in (0, 4, 8) else 0.0
    c.width, c.height = width, height
    s = B.make_settings(None)
    out = B.c_image_out(0x60000, 0x70000, 0x80000, None)
    return g, c, s, out


def _pinhole(c, fx=50.0, fy=50.0, cx=32.0, cy=16.0):
    c.model = B.CAMERA_PINHOLE
    c.fx, c.fy, c.cx, c.cy = fx, fy, cx, cy


def _alloc(fail):
    calls = []

    def cb(user, nbytes, kind):
        calls.append((nbytes, kind))
        return None if fail else None

    f = B.ALLOC_FN(cb)
    return B.c_allocator(f, None), calls, f


def _forward(lib, g, c, s, out, alloc, cap=None):
    st = B.c_state()
    return lib.omnigs_forward(ctypes.byref(g), ctypes.byref(c), ctypes.byref(s), alloc, ctypes.byref(out),
                              ctypes.byref(st), ctypes.byref(cap) if cap is not None else None, None)


@pytest.mark.parametrize("mutate,needle", [
    (lambda g, c, s, o: setattr(c, "width", 100), "multiple of 16"),
    (lambda g, c, s, o: setattr(c, "height", 0), "height"),
    (lambda g, c, s, o: setattr(g, "sh_degree", 4), "sh_degree"),
    (lambda g, c, s, o: setattr(g, "sh_coeffs", 4), "sh_coeffs"),
    (lambda g, c, s, o: setattr(g, "n", -1), "out of range"),
    (lambda g, c, s, o: setattr(g, "means", None), "NULL"),
    (lambda g, c, s, o: setattr(g, "quats", 0x30004), "aligned"),
    (lambda g, c, s, o: c.R_cw.__setitem__(3, float("nan")), "non-finite"),
    (lambda g, c, s, o: setattr(s, "alpha_min", 0.0), "alpha_min"),
    (lambda g, c, s, o: setattr(s, "T_min", 1.5), "T_min"),
    (lambda g, c, s, o: setattr(s, "T_min", 1e-50), "T_min"),  # zero as a float
    (lambda g, c, s, o: setattr(o, "image", None), "NULL"),
    (lambda g, c, s, o: setattr(c, "model", 7), "unknown camera model"),
    (lambda g, c, s, o: setattr(c, "rows", 33), "rows"),
    (lambda g, c, s, o: setattr(c, "rows", -1), "rows"),
    (lambda g, c, s, o: _pinhole(c, fx=0.0), "intrinsics"),
    (lambda g, c, s, o: _pinhole(c, fy=float("nan")), "intrinsics"),
    (lambda g, c, s, o: _pinhole(c, cx=float("inf")), "intrinsics"),
    (lambda g, c, s, o: (_pinhole(c), setattr(c, "width", 0)), "width"),
])
def test_invalid_arguments(lib, mutate, needle):
    g, c, s, out = _fake_args()
    mutate(g, c, s, out)
    alloc, calls, keep = _alloc(fail=True)
    rc = _forward(lib, g, c, s, out, alloc)
    assert rc == B.OMNIGS_ERR_INVALID
    assert needle in B.omnigs_last_error()
    assert calls == []  # rejected before allocating


@pytest.mark.parametrize("instances,entries", [(-1, 0), (0, -5), (1 << 31, 0), (100, (1 << 31) - 1)])
def test_invalid_capacities(lib, instances, entries):
    g, c, s, out = _fake_args()
    alloc, calls, keep = _alloc(fail=True)
    rc = _forward(lib, g, c, s, out, alloc, B.c_capacity(instances, entries, None))
    assert rc == B.OMNIGS_ERR_INVALID
    assert "capacities" in B.omnigs_last_error()
    assert calls == []


def test_capacity_mode_allocates_up_front(lib):
    """With capacities the instance and block-entry buffers come with the
    per-Gaussian ones: one state and one scratch request, before any work
    (the failing allocator stops the call at the first)."""
    g, c, s, out = _fake_args(n=1000)
    alloc, calls, keep = _alloc(fail=True)
    rc = _forward(lib, g, c, s, out, alloc, B.c_capacity(5_000_000, 0, None))
    assert rc == B.OMNIGS_ERR_ALLOC
    assert len(calls) == 1 and calls[0][1] == B.OMNIGS_MEM_STATE and calls[0][0] >= 5_000_000 * 4


def test_pinhole_accepts_any_width(lib):
    """A pinhole image need not be a multiple of 16 wide: validation passes
    and the call proceeds to allocation."""
    g, c, s, out = _fake_args(n=1000, width=100)
    _pinhole(c)
    alloc, calls, keep = _alloc(fail=True)
    assert _forward(lib, g, c, s, out, alloc) == B.OMNIGS_ERR_ALLOC
    assert calls


def test_allocator_failure_reports_err_alloc(lib):
    g, c, s, out = _fake_args(n=1000)
    alloc, calls, keep = _alloc(fail=True)
    rc = _forward(lib, g, c, s, out, alloc)
    assert rc == B.OMNIGS_ERR_ALLOC
    assert "allocator returned NULL" in B.omnigs_last_error()
    assert len(calls) == 1 and calls[0][1] == B.OMNIGS_MEM_STATE and calls[0][0] >= 1000 * 48


def test_l1_and_backward_argument_checks(lib):
    alloc, calls, keep = _alloc(fail=True)
    assert lib.omnigs_l1_loss(None, None, 10, None, None, alloc, None) == B.OMNIGS_ERR_INVALID
    assert lib.omnigs_l1_loss(0x1000, 0x2000, 0, None, 0x3000, alloc, None) == B.OMNIGS_ERR_INVALID
    assert lib.omnigs_l1_loss(0x1000, 0x2000, 10, None, 0x3000, alloc, None) == B.OMNIGS_ERR_ALLOC
    g, c, s, out = _fake_args()
    st = B.c_state()
    st.n, st.width, st.height = 5, 64, 32  # does not match n = 10
    gr = B.c_grads(0x1000, 0x2000, 0x3000, 0x4000, 0x5000, 0x6000)
    rc = lib.omnigs_backward(ctypes.byref(g), ctypes.byref(c), ctypes.byref(s), ctypes.byref(st), ctypes.byref(out),
                             0x9000, None, None, ctypes.byref(gr), alloc, None)
    assert rc == B.OMNIGS_ERR_INVALID and "state does not match" in B.omnigs_last_error()
    # depth / alpha cotangents need the state's depth values
    st.n = 10
    st.records = st.n_tiles = st.inst_gauss = st.tile_range = st.tile_work = 0xa000
    rc = lib.omnigs_backward(ctypes.byref(g), ctypes.byref(c), ctypes.byref(s), ctypes.byref(st), ctypes.byref(out),
                             0x9000, 0xb000, None, ctypes.byref(gr), alloc, None)
    assert rc == B.OMNIGS_ERR_INVALID and "depth" in B.omnigs_last_error()
    # a crop's state has the rendered rows
    c.rows = 20
    rc = lib.omnigs_backward(ctypes.byref(g), ctypes.byref(c), ctypes.byref(s), ctypes.byref(st), ctypes.byref(out),
                             0x9000, None, None, ctypes.byref(gr), alloc, None)
    assert rc == B.OMNIGS_ERR_INVALID and "state does not match" in B.omnigs_last_error()


def test_ceilings_argument_checks(lib):
    alloc, calls, keep = _alloc(fail=True)
    out = B.c_ceilings()
    assert lib.omnigs_measure_ceilings(0, 0, 0, alloc, ctypes.byref(out), None) == B.OMNIGS_ERR_INVALID
    assert lib.omnigs_measure_ceilings(1 << 32, 0, 1, alloc, ctypes.byref(out), None) == B.OMNIGS_ERR_INVALID
    assert lib.omnigs_measure_ceilings(0, 17, 1, alloc, ctypes.byref(out), None) == B.OMNIGS_ERR_INVALID
    assert lib.omnigs_measure_ceilings(1024, 1 << 20, 1, alloc, None, None) == B.OMNIGS_ERR_INVALID
    assert lib.omnigs_measure_ceilings(1024, 1 << 20, 1, alloc, ctypes.byref(out), None) == B.OMNIGS_ERR_ALLOC


def test_profile_stage_names(lib):
    n = lib.omnigs_profile_num_stages()
    names = [lib.omnigs_profile_stage_name(k).decode() for k in range(n)]
    assert names[:8] == ["project", "depth_sort", "emit_count", "super_emit", "super_sort", "tile_bin", "tile_order",
                         "blend_fwd"]
    assert names[8:] == ["l1_loss", "bwd_clear", "blend_bwd", "project_bwd", "stats", "adam", "densify"]
    assert lib.omnigs_profile_stage_name(n).decode() == ""


def _forward_batch(lib, g, cams, s, outs, alloc, batch=None, capacity=0):
    B_ = len(cams) if batch is None else batch
    ca = (B.c_camera * max(len(cams), 1))(*cams)
    oa = (B.c_image_out * max(len(outs), 1))(*outs)
    m = ctypes.c_int64(7)
    rc = lib.omnigs_forward_batch(ctypes.byref(g), ca, B_, ctypes.byref(s), alloc, oa, capacity, None,
                                  ctypes.byref(m), None)
    return rc, m.value


@pytest.mark.parametrize("case,needle", [
    ("batch0", "batch 0"),
    ("batch17", "batch 17"),
    ("bad_width", "multiple of 16"),
    ("null_out", "camera 1 is NULL"),
    ("capacity", "instance_capacity"),
    ("too_many_records", "below 2^32"),
])
def test_forward_batch_invalid_arguments(lib, case, needle):
    g, c, s, out = _fake_args()
    cams = [B.c_camera.from_buffer_copy(c) for _ in range(3)]
    outs = [B.c_image_out(0x60000, 0x70000, 0x80000, None) for _ in range(3)]
    batch, cap = None, 0
    if case == "batch0":
        batch = 0
    elif case == "batch17":
        batch = 17
        cams = cams * 6
        outs = outs * 6
    elif case == "bad_width":
        cams[2].width = 72 + 4
    elif case == "null_out":
        outs[1].final_T = None
    elif case == "capacity":
        cap = -5
    elif case == "too_many_records":
        g.n = (1 << 31) - 1
    alloc, calls, keep = _alloc(fail=True)
    rc, m = _forward_batch(lib, g, cams, s, outs, alloc, batch=batch, capacity=cap)
    assert rc == B.OMNIGS_ERR_INVALID
    assert needle in B.omnigs_last_error()
    assert m == -1 and calls == []


def test_forward_batch_allocator_failure(lib):
    g, c, s, out = _fake_args(n=1000)
    cams = [B.c_camera.from_buffer_copy(c) for _ in range(2)]
    outs = [B.c_image_out(0x60000, 0x70000, 0x80000, None) for _ in range(2)]
    alloc, calls, keep = _alloc(fail=True)
    rc, m = _forward_batch(lib, g, cams, s, outs, alloc)
    assert rc == B.OMNIGS_ERR_ALLOC
    # one scratch allocation holding the records of both cameras
    assert len(calls) == 1 and calls[0][1] == B.OMNIGS_MEM_SCRATCH and calls[0][0] >= 2 * 1000 * 48


def test_forward_batch_bytes_host_query(lib):
    """The size query runs on the host: it grows by exactly 4 bytes per
    instance of capacity (the Gaussian id) plus the block-entry scratch
    sized by the same capacity, by the per-record buffers per Gaussian and
    camera, and rejects what omnigs_forward_batch rejects."""
    from paper_2404_03202_amd import scenes
    cams = [scenes.camera(w, h) for (w, h) in scenes.SERVE_RESOLUTIONS]
    q = lambda n, cs, cap: B.omnigs_forward_batch_bytes(n, cs, cap)
    base = q(100_000, cams[:1], 1 << 20)
    assert base > 100_000 * 48  # at least the blend records
    # linear in the capacity once the per-capacity buffers dominate (past 1.6M
    # keys the radix sort's blocks hold 6144 keys instead of 4096)
    d1 = q(100_000, cams[:1], 3 << 20) - q(100_000, cams[:1], 2 << 20)
    d2 = q(100_000, cams[:1], 4 << 20) - q(100_000, cams[:1], 3 << 20)
    assert abs(d1 - d2) <= 4096 and d1 >= 4 * (1 << 20)
    # more cameras: more records and tiles
    assert q(100_000, cams, 1 << 20) > q(100_000, cams[:2], 1 << 20) > base
    for bad in ((-1, cams[:1], 1), (10, cams[:1], 0), (10, [], 1), (10, cams * 5, 1)):
        with pytest.raises(B.OmnigsError):
            q(*bad)
    odd = dict(scenes.camera(64, 32), width=60)
    with pytest.raises(B.OmnigsError, match="multiple of 16"):
        q(10, [odd], 1)
