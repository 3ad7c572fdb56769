"""bench.py's roofline bookkeeping on the host: the counted HBM traffic is
reported only for the kernel source and the kind of launch (one or two steps)
it was taken on, and the committed counter file names its commands."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(tmp_path, kernel_hash=None, **kw):
    v = {"steps_per_launch": 2, "hbm_bytes_per_launch": 123456789,
         "sq_insts_valu_per_dispatch": 1000}
    v.update(kw)
    d = {"kernel_hash": kernel_hash or bench._kernel_hash(), "variants": {"22": v}}
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "profiles" / "fused_step_d2q16_1024_counters.json").write_text(json.dumps(d))


def test_counters_need_the_same_source_launch_kind_and_variant(tmp_path, monkeypatch):
    h = bench._kernel_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_kernel_hash", lambda: h)
    _write(tmp_path)
    assert bench.counters_from_profile(2, 22)["hbm_bytes_per_launch"] == 123456789
    assert bench.counters_from_profile(1, 22) is None
    assert bench.counters_from_profile(2, 21) is None
    _write(tmp_path, kernel_hash="0" * 16)
    assert bench.counters_from_profile(2, 22) is None
    _write(tmp_path, steps_per_launch=None)
    assert bench.counters_from_profile(2, 22) is None


def test_counters_without_a_counter_file(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counters_from_profile(1, 0) is None


def test_committed_counter_file_is_complete():
    d = json.load(open(os.path.join(ROOT, "profiles", "fused_step_d2q16_1024_counters.json")))
    for k in ("kernel", "kernel_hash", "calibration", "variants", "commands"):
        assert k in d, k
    cal = d["calibration"]
    # the copy kernel of known size fixes bytes per counted KiB
    assert abs(cal["fetch_factor"] * cal["fetch_size_kib_per_dispatch"] * 1024
               - cal["bytes_read_per_dispatch"]) <= 1024
    assert abs(cal["write_factor"] * cal["write_size_kib_per_dispatch"] * 1024
               - cal["bytes_written_per_dispatch"]) <= 1024
    assert d["variants"]
    for name, v in d["variants"].items():
        for k in ("steps_per_launch", "grid_size", "fetch_size_kib_per_dispatch",
                  "write_size_kib_per_dispatch", "hbm_bytes_per_launch",
                  "algorithmic_bytes_per_launch", "sq_insts_valu_per_dispatch"):
            assert k in v, (name, k)
        want = (cal["fetch_factor"] * v["fetch_size_kib_per_dispatch"]
                + cal["write_factor"] * v["write_size_kib_per_dispatch"]) * 1024
        assert abs(v["hbm_bytes_per_launch"] - want) <= 1
        assert v["algorithmic_bytes_per_launch"] == 2 * 16 * 4 * 1024 * 1024 * v["steps_per_launch"]
    assert all(c.startswith("rocprofv3 --pmc ") for c in d["commands"])


def test_more_than_one_gpu_is_refused():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
