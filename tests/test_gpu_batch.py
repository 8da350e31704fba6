"""Batched forward (omnigs_forward_batch) and the continuous-batching server.

Every batched output must equal the render of its camera alone, bit for bit
(same records, same tile lists, same blend arithmetic), in both capacity
modes; sampled outputs are also checked against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2404_03202_amd import omnigs as B
from paper_2404_03202_amd import scenes
from paper_2404_03202_amd import serve

import parity

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FIELDS = ("image", "final_T", "n_contrib", "n_blended")


def to_dev(g):
    d = {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(DEV)
         for k, v in g.items() if k != "sh_degree"}
    d["sh_degree"] = g["sh_degree"]
    return d


def alone(gd, cam, settings=None):
    r = B.omnigs_forward(gd, cam, settings, with_blended=True)
    return dict(image=r.image, final_T=r.final_T, n_contrib=r.n_contrib, n_blended=r.n_blended), r.n_instances


def mixed_cameras():
    return [
        scenes.camera(128, 64),
        scenes.camera(96, 40, scenes.rot_y(1.1).T, [0.2, -0.1, 0.3]),          # ragged height
        scenes.camera(256, 128, scenes.rot_y(-2.5).T, [-0.4, 0.2, 0.1]),
        scenes.camera(16, 16, scenes.rot_y(0.3).T),                              # one tile
        scenes.camera(512, 256, np.eye(3), [0.1, 0.0, -0.2]),                    # yaw 0: seam wedge straddles
    ]


def assert_same(a, b, what):
    for k in FIELDS:
        if k in a and k in b:
            assert torch.equal(a[k], b[k]), f"{what}: {k} differs from the single-camera render"


@pytest.fixture(scope="module")
def room():
    return to_dev(scenes.room_scene(90, 30000, seam_fraction=0.3))


def test_batch_bit_identical_to_single(room):
    cams = mixed_cameras()
    singles, ms = zip(*[alone(room, c) for c in cams])
    res = B.omnigs_forward_batch(room, cams, with_blended=True)
    torch.cuda.synchronize()
    assert res.n_instances == sum(ms)
    assert int(res.overflow.item()) == 0
    for k, (o, s) in enumerate(zip(res.outs, singles)):
        assert_same(o, s, f"camera {k}")


def test_batch_capacity_mode(room):
    cams = mixed_cameras()
    ref = B.omnigs_forward_batch(room, cams, with_blended=True)
    M = ref.n_instances
    for cap in (M, 3 * M + 17):
        r = B.omnigs_forward_batch(room, cams, instance_capacity=cap, with_blended=True)
        torch.cuda.synchronize()
        assert r.n_instances == -1 and int(r.overflow.item()) == 0, cap
        for k, (o, s) in enumerate(zip(r.outs, ref.outs)):
            assert_same(o, s, f"capacity {cap}, camera {k}")
    # too small: flagged, no fault, outputs discarded
    for cap in (M - 1, M // 3, 1):
        r = B.omnigs_forward_batch(room, cams, instance_capacity=cap)
        torch.cuda.synchronize()
        assert int(r.overflow.item()) == 1, cap


def test_batch_max_size_and_limits(room):
    cams = [scenes.camera(64, 32, scenes.rot_y(0.4 * k).T, [0.05 * k, 0.0, -0.03 * k]) for k in range(B.OMNIGS_MAX_BATCH)]
    res = B.omnigs_forward_batch(room, cams, with_blended=True)
    for k, c in enumerate(cams):
        assert_same(res.outs[k], alone(room, c)[0], f"camera {k} of {len(cams)}")
    with pytest.raises(B.OmnigsError, match="batch 17"):
        B.omnigs_forward_batch(room, cams + cams[:1])


def test_batch_empty_and_culled_scene():
    bg = (0.25, 0.5, 0.75)
    empty = to_dev(dict(means=np.zeros((0, 3)), scales=np.zeros((0, 3)), quats=np.zeros((0, 4)),
                        opacities=np.zeros(0), sh=np.zeros((0, 16, 3)), sh_degree=3))
    cams = [scenes.camera(64, 32), scenes.camera(32, 20)]
    for cap in (0, 100):
        res = B.omnigs_forward_batch(empty, cams, dict(bg=bg), instance_capacity=cap)
        torch.cuda.synchronize()
        for o, c in zip(res.outs, cams):
            expect = np.broadcast_to(np.array(bg, np.float32)[:, None, None], (3, c["height"], c["width"]))
            np.testing.assert_array_equal(o["image"].cpu().numpy(), expect)
            assert (o["n_contrib"] == 0).all()
    g = scenes.shell_scene(91, 400)
    g["opacities"][:] = 1.0 / 300.0
    res = B.omnigs_forward_batch(to_dev(g), cams)
    assert res.n_instances == 0


def test_batch_oracle_parity():
    g = scenes.shell_scene(92, 3000)
    gd = to_dev(g)
    cams = [scenes.camera(128, 64), scenes.camera(96, 40, scenes.rot_y(2.0).T, [0.3, -0.4, 0.2]),
            scenes.camera(64, 32, scenes.rot_y(-0.7).T)]
    res = B.omnigs_forward_batch(gd, cams, dict(bg=(0.1, 0.3, 0.2)), with_blended=True)
    torch.cuda.synchronize()
    for k, c in enumerate(cams):
        orc = O.render(O.Scene(g, c, dict(bg=(0.1, 0.3, 0.2))))
        parity.check_image(res.outs[k]["image"].cpu().numpy(), orc, what=f"batched camera {k}",
                           gpu_T=res.outs[k]["final_T"].cpu().numpy(), gpu_nc=res.outs[k]["n_contrib"].cpu().numpy())


# ---------------------------------------------------------------- serving
SERVE_RES = ((128, 64), (256, 128), (512, 256), (1024, 512))


def test_serving_results_identical_alone(room):
    cams = scenes.serve_cameras(93, 48, SERVE_RES)
    # estimates far too small at first: the first batches overflow and are
    # retried with grown capacities
    srv = serve.Server(room, slots=2, max_batch=6, instance_estimate={r: 2000 for r in SERVE_RES})
    reqs = serve.make_requests(cams, scenes.arrival_times(93, len(cams), 4000.0))
    out = srv.run(reqs)
    print("serving", out)
    assert out["requests"] == len(cams)
    assert out["overflows"] >= 1 and out["mean_batch"] > 1.0
    assert all(r.done >= r.start >= r.arrival for r in reqs)
    for r in reqs:
        ref = alone(room, r.camera)[0]["image"]
        assert torch.equal(r.image, ref), f"request {r.rid} (batch of {r.batch_size}) differs from its render alone"


def test_serving_admission_by_footprint(room):
    cams = scenes.serve_cameras(94, 12, SERVE_RES)
    srv = serve.Server(room, slots=2, max_batch=8)
    srv.calibrate([scenes.camera(w, h) for (w, h) in SERVE_RES])
    smallest = min(srv.batch_bytes([r]) for r in serve.make_requests(cams))
    # a budget below any two requests' footprint: one request in flight at a time
    srv.budget = smallest + 1
    out = srv.run(serve.make_requests(cams))
    assert out["requests"] == 12 and out["mean_batch"] == 1.0
    srv = serve.Server(room, slots=1, max_batch=8, hbm_budget=64 << 30)
    srv.calibrate([scenes.camera(w, h) for (w, h) in SERVE_RES])
    out = srv.run(serve.make_requests(cams))
    assert out["mean_batch"] > 1.0


def test_footprint_matches_allocations(room):
    """The footprint the server admits by (the library's size query plus the
    outputs) equals what one batch takes from the caching allocator, up to
    the allocator's 512-byte rounding of each block."""
    cams = [scenes.camera(w, h, scenes.rot_y(0.3 * k).T, [0.1 * k, 0.0, 0.0]) for k, (w, h) in enumerate(SERVE_RES)]
    counts = [alone(room, c)[1] for c in cams]
    cap = int(1.1 * sum(counts)) + 1
    n = int(room["means"].shape[0])
    expect = serve.footprint(n, cams, cap)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    res = B.omnigs_forward_batch(room, cams, instance_capacity=cap)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    assert int(res.overflow) == 0
    blocks = 2 + 3 * len(cams) + 1  # two scratch arenas, three outputs per camera, the overflow word
    assert expect <= peak <= expect + 512 * blocks, (expect, peak)
    with pytest.raises(B.OmnigsError):
        B.omnigs_forward_batch_bytes(n, cams, 0)


def test_serving_sampled_oracle():
    g = scenes.room_scene(95, 4000, seam_fraction=0.3)
    gd = to_dev(g)
    cams = scenes.serve_cameras(95, 10, ((128, 64), (256, 128)))
    srv = serve.Server(gd, slots=2, max_batch=4)
    srv.calibrate([scenes.camera(128, 64), scenes.camera(256, 128)])
    reqs = serve.make_requests(cams)
    srv.run(reqs)
    for r in reqs[::3]:
        orc = O.render(O.Scene(g, r.camera))
        parity.check_image(r.image.cpu().numpy(), orc, what=f"served request {r.rid}")
