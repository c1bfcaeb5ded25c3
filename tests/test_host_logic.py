"""CPU tests of host-side logic: the batch autotuner's choice and cache, and argument
validation of the C ABI entry points (no GPU work is launched)."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2412_00291_amd", "libmapcore.so")


class _FakeBatch:
    def __init__(self):
        self.maps = []
        self.cfg = None

    def configure(self, sched, grid, use_graph):
        self.cfg = (sched, grid)

    def close(self):
        pass


def test_autotuner_picks_fastest_and_caches(tmp_path, monkeypatch):
    import time
    from paper_2412_00291_amd import autotune
    monkeypatch.setenv("MAPCORE_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")

    class _T:  # stands in for torch.cuda.synchronize
        class cuda:
            @staticmethod
            def synchronize():
                pass
    monkeypatch.setitem(__import__("sys").modules, "torch", _T)
    cost = {(0, 1024): 0.004, (0, 2048): 0.002, (1, 1024): 0.003}
    built = []

    def build():
        b = _FakeBatch()
        built.append(b)
        return b

    def run_step(b, k):
        time.sleep(cost[b.cfg])

    sched, grid, timings = autotune.tune("sig-a", build, run_step, n_steps=2, candidates=list(cost))
    assert (sched, grid) == (0, 2048) and len(built) == 3
    data = json.load(open(tmp_path / "tune.json"))
    assert data["gfx950|sig-a|median"]["grid"] == 2048
    built.clear()
    assert autotune.tune("sig-a", build, run_step, candidates=list(cost))[:2] == (0, 2048)
    assert not built  # served from the cache


def test_autotuner_mean_score_counts_every_step(tmp_path, monkeypatch):
    """A schedule that is fastest on most steps but slow on the rest wins by the median and
    loses by the mean; the two scores are cached apart, and an unknown score is refused."""
    import time
    from paper_2412_00291_amd import autotune
    monkeypatch.setenv("MAPCORE_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "_arch", lambda: "gfx950")

    class _T:
        class cuda:
            @staticmethod
            def synchronize():
                pass
    monkeypatch.setitem(__import__("sys").modules, "torch", _T)
    # seconds per step k = 1..5: (4, 2) is fast early and slow late, (4, 16) is even
    cost = {(4, 2): [0.001, 0.001, 0.001, 0.009, 0.009], (4, 16): [0.003] * 5}

    def build():
        return _FakeBatch()

    def run_step(b, k):
        if k > 0:
            time.sleep(cost[b.cfg][k - 1])

    sched, grid, t_med = autotune.tune("sig-b", build, run_step, n_steps=5, candidates=list(cost))
    assert (sched, grid) == (4, 2) and t_med[(4, 2)] < t_med[(4, 16)]
    sched, grid, t_mean = autotune.tune("sig-b", build, run_step, n_steps=5, candidates=list(cost), score="mean")
    assert (sched, grid) == (4, 16) and t_mean[(4, 2)] > t_mean[(4, 16)]
    data = json.load(open(tmp_path / "tune.json"))
    assert data["gfx950|sig-b|median"]["grid"] == 2 and data["gfx950|sig-b|mean"]["grid"] == 16
    with pytest.raises(ValueError):
        autotune.tune("sig-b", build, run_step, candidates=list(cost), score="max")


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_create_rejects_bad_parameters():
    from paper_2412_00291_amd import MAP_ERR_INVALID_ARG, map_create, map_last_error
    for args in ((0.0, 0.3, 1000, 19), (0.1, 0.0, 1000, 19), (0.1, 7.0, 1000, 19), (0.1, 0.3, 0, 19),
                 (0.1, 0.3, 1000, 0), (0.1, 0.3, 1000, 255), (float("nan"), 0.3, 1000, 19)):
        st, h = map_create(*args, device=0, stream=0)
        assert st == MAP_ERR_INVALID_ARG and not h.value
        assert "map_create" in map_last_error(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_null_handles_are_rejected():
    import ctypes
    from paper_2412_00291_amd import MAP_ERR_INVALID_ARG
    from paper_2412_00291_amd.mapcore import _lib
    assert _lib.map_sync(None) == MAP_ERR_INVALID_ARG
    assert _lib.map_integrate_lidar(None, None, None, None, None) == MAP_ERR_INVALID_ARG
    assert _lib.map_batch_step(None, None, 0, None, None) == MAP_ERR_INVALID_ARG
    assert _lib.map_set_schedule(None, 0, 0, 0) == MAP_ERR_INVALID_ARG
    _lib.map_destroy(None)
    _lib.map_batch_destroy(None)
    n = ctypes.c_int64(0)
    assert _lib.map_extract_mesh(None, 0, None, None, None, 0, ctypes.byref(n), None) == MAP_ERR_INVALID_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")
def test_every_entry_point_rejects_a_null_handle():
    """Each call that takes a map rejects a NULL map before any device work (status, or -1 /
    0 for the counting test-access calls); the calls without a map reject NULL or
    out-of-range arguments the same way.  Runs on the host alone."""
    import ctypes
    from paper_2412_00291_amd import MAP_ERR_INVALID_ARG as BAD
    from paper_2412_00291_amd.mapcore import _Quality, _lib
    h = ctypes.c_void_p(0)
    assert _lib.map_integrate_labels(None, None, None, None, None) == BAD
    assert _lib.map_integrate_labels_multi(None, 0, None, None, None, None) == BAD
    assert _lib.map_integrate_labels_lidar(None, None, None, None, None) == BAD
    assert _lib.map_integrate_logprobs(None, None, None, None, None) == BAD
    assert _lib.map_query_sdf(None, None, 0, None, None, None, None) == BAD
    assert _lib.map_range_image(None, None, None, 0, 1.0, 0.0, None, None, None) == BAD
    assert _lib.map_sdf_pose_adjoint(None, None, None, 0, 0, None, None, None, None) == BAD
    assert _lib.map_sdf_pose_adjoint_noalloc(None, None, None, 0, 0, None, None, None, None) == BAD
    assert _lib.map_stats(None, None) == BAD
    assert _lib.map_profile(None, 0) == BAD
    assert _lib.map_profile_read(None, None, None) == BAD
    assert _lib.map_set_dirty_bitmap(None, 0) == BAD
    assert _lib.map_set_distance(None, 0, 0.0) == BAD
    assert _lib.map_set_label_fusion(None, 0) == BAD
    assert _lib.map_batch_configure(None, 0, 1024, 0) == BAD
    # test access: -1 (or 0 blocks) for no map
    assert _lib.map_block_coords(None, None, 0) == -1
    assert _lib.map_touched_coords(None, None, 0) == -1
    assert _lib.map_download(None, 0, None, None, None, None, None) == -1
    assert _lib.map_download_aux(None, 0, None, None) == -1
    assert _lib.map_frame_normals(None, None, 0) == -1
    assert _lib.map_read_block(None, 0, 0, 0, None, None, None, None) == 0
    # no map: the batch needs maps and an output, the quality metrics an output and sizes
    assert _lib.map_batch_create(None, 1, ctypes.byref(h)) == BAD
    assert _lib.map_batch_create(None, 1, None) == BAD
    assert "map_batch_create" in _lib.map_last_error(None).decode()
    q = _Quality()
    assert _lib.map_mesh_quality(None, None, 0, None, None, 0, 0.1, 19, 0, None, None, None, None, None,
                                 None) == BAD
    assert _lib.map_mesh_quality(None, None, -1, None, None, 0, 0.1, 19, 0, None, None, None, None,
                                 ctypes.byref(q), None) == BAD
    assert _lib.map_mesh_quality(None, None, 5, None, None, 0, 0.1, 19, 0, None, None, None, None,
                                 ctypes.byref(q), None) == BAD
    assert _lib.map_mesh_quality(None, None, 0, None, None, 0, 0.0, 19, 0, None, None, None, None,
                                 ctypes.byref(q), None) == BAD
    assert "mesh_quality" in _lib.map_last_error(None).decode()


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and says so, before
    touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
