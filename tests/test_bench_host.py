"""Host-side logic of bench.py: kernel naming by work-group size and the lookup of counter traffic
per launch shape (no GPU)."""
import importlib.util
import os
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def info(segment, first_levels, threads):
    return types.SimpleNamespace(segment=segment, launch_first_level=first_levels,
                                 launch_threads=threads)


def test_kernel_names_follow_planned_work_group_size(bench):
    assert bench.launch_kernel_name("ig1", info(3072, [0, 5], [128, 128]), 0) == \
        "spd::step_kernel<true, 1, false, 128, true>"
    assert bench.launch_kernel_name("ig1", info(4096, [0, 4], [256, 256]), 1) == \
        "spd::step_kernel<false, 1, false, 256, true>"
    assert bench.launch_kernel_name("bd16", info(3072, [0, 5], [256, 256]), 1, planes=False) == \
        "spd::step_kernel<false, 5, false, 256, false>"


def test_planner_reports_work_group_size():
    """The planner's launch list carries each launch's work-group size and tile: IG(1) tiles of
    at most 3072 units on 128 threads, later launches on tiles no longer than their slots need."""
    from paper_1910_08324_amd import spd
    i = spd.plan(spd.Config("ig1", 8192, segment=3072, step_levels=5), 4096, 262144)
    assert [i.launch_threads[k] for k in range(i.n_launches)] == [128] * i.n_launches
    assert i.launch_tile[0] == 3072
    i = spd.plan(spd.Config("ig1", 8192, segment=4096, step_levels=4), 4096, 262144)
    th = [i.launch_threads[k] for k in range(i.n_launches)]
    tl = [i.launch_tile[k] for k in range(i.n_launches)]
    assert th == [256, 256, 128] and tl == [4096, 4096, 1024]
    for m in ("ig2", "ig3", "bd8", "bd16", "bd32"):
        i = spd.plan(spd.Config(m, 8192, segment=2048), 4096, 262144)
        assert all(i.launch_threads[k] == 256 for k in range(i.n_launches)), m
    i = spd.plan(spd.Config("exh", 256), 64, 65536)
    assert i.launch_threads[i.n_launches - 1] == 64 and i.launch_tile[i.n_launches - 1] == 0


def test_read_traffic_by_shape(bench, tmp_path, monkeypatch):
    f = tmp_path / "counters.txt"
    k128, k256 = ("spd::step_kernel<true, 1, false, 128, true>",
                  "spd::step_kernel<true, 1, false, 256, true>")
    f.write_text("\n".join([
        "# comment: ignored", "kernel | a | b", "method: ig1", f"kernel: {k128}", "segment: 3072",
        "step_levels: 4", "kernel_source_sha256_16: abc", "hbm_bytes_per_launch: 1.5e10",
        f"kernel@3072/5: {k128}", "hbm_bytes_per_launch@3072/5: 1.7e10",
        f"kernel@4096/4: {k256}", "hbm_bytes_per_launch@4096/4: 1.6e10"]) + "\n")
    monkeypatch.setattr(bench, "PMC_FILE", str(f))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.read_traffic("ig1", k128, (3072, 4)) == 1.5e10
    assert bench.read_traffic("ig1", k128, (3072, 5)) == 1.7e10
    assert bench.read_traffic("ig1", k256, (4096, 4)) == 1.6e10
    assert bench.read_traffic("ig1", k256, (6144, 4)) is None           # shape not measured
    assert bench.read_traffic("ig1", k256, (3072, 5)) is None           # other kernel at that shape
    assert bench.read_traffic("ig2", k128, (3072, 4)) is None           # other method
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "def")
    assert bench.read_traffic("ig1", k128, (3072, 4)) is None           # source changed since
