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


def info(segment, first_levels, n_out=262144):
    slots = [0] * 24
    slots[0] = n_out
    return types.SimpleNamespace(segment=segment, launch_first_level=first_levels, plane_slots=slots)


def test_step_threads(bench):
    # IG(1): 128 threads on tiles of at most 3072 units; later launches get tiles no longer than
    # their first level's slots need
    assert bench.step_threads("ig1", info(3072, [0, 5, 10]), 0) == 128
    assert bench.step_threads("ig1", info(4096, [0, 4, 8]), 0) == 256
    assert bench.step_threads("ig1", info(4096, [0, 4, 8]), 1) == 256      # 16384 slots: tile 4096
    assert bench.step_threads("ig1", info(4096, [0, 4, 8]), 2) == 128      # 1024 slots: tile 1024
    for m in ("ig2", "ig3", "bd8", "bd16", "bd32"):
        assert bench.step_threads(m, info(2048, [0, 4]), 0) == 256
    assert bench.launch_kernel_name("ig1", info(3072, [0, 5]), 0) == "spd::step_kernel<true, 1, false, 128>"
    assert bench.launch_kernel_name("bd16", info(3072, [0, 5]), 1) == "spd::step_kernel<false, 5, false, 256>"


def test_read_traffic_by_shape(bench, tmp_path, monkeypatch):
    f = tmp_path / "counters.txt"
    k128, k256 = "spd::step_kernel<true, 1, false, 128>", "spd::step_kernel<true, 1, false, 256>"
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
