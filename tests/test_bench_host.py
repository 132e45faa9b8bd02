"""Host-side checks of bench.py: the one-GPU rule and the counter lookup that
fills roofline.traffic (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_committed_counters_are_used_while_they_match_the_kernel_source():
    """The committed counter summary is keyed to the kernel source it was taken
    from; bench.py reports its traffic only while the two agree."""
    with open(bench.COUNTERS) as fh:
        tab = json.load(fh)
    entry = tab["k_eso_fp64:grid100_k10000"]
    if entry["kernel_source_sha256_16"] != bench.kernel_source_hash():
        assert bench.measured_traffic("k_eso_fp64:grid100_k10000") is None
        pytest.skip("the counters predate the current kernel source (traffic is reported as null)")
    assert bench.measured_traffic("k_eso_fp64:grid100_k10000") == entry["bytes_per_launch"]
    # read + write, scaled by the plain copy's factors
    assert entry["bytes_per_launch"] == pytest.approx(entry["read_bytes"] + entry["write_bytes"])


def test_stale_or_missing_counters_give_no_traffic(tmp_path, monkeypatch):
    stale = tmp_path / "hbm_counters.json"
    stale.write_text(json.dumps({"k": {"kernel_source_sha256_16": "0" * 16,
                                       "bytes_per_launch": 1.0}}))
    monkeypatch.setattr(bench, "COUNTERS", str(stale))
    assert bench.measured_traffic("k") is None
    assert bench.measured_traffic("absent") is None
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "none.json"))
    assert bench.measured_traffic("k") is None


def test_cpu_baseline_reports_both_thread_counts_and_restores_them():
    import oracle
    from gen.instance import recipe_grid4_k8
    nt = oracle.num_threads()
    out = bench.cpu_baseline(recipe_grid4_k8(), 3, 2)
    assert out["kind"] == "oracle" and out["cores"] == nt and out["value"] > 0
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
    assert oracle.num_threads() == nt


class _FakeCtx:
    """Stands in for a context: z falls by 10x per pass from 1, one z-log entry
    per pass, FP32 for the first 4 passes then FP64."""

    def __init__(self):
        self.ev = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False

    def z(self, i):
        return 10.0 ** (-i)

    def solve(self, target, max_sweeps, window):
        a = b = 0
        while a + b < max_sweeps and not self.z(self.ev) <= target:
            self.ev += 1
            if self.ev <= 4:
                a += 1
            else:
                b += 1
        return a, b

    def residual(self):
        return {"evaluations": self.ev, "z": self.z(self.ev), "verdict": "feasible",
                "z_fp32_floor": 1e-12 if self.ev <= 4 else 0.0}

    def z_log(self, first, count):
        import numpy as np
        return np.array([self.z(i + 1) for i in range(first, first + count)])


class _FakePdr:
    FP64, FP32_BULK = 0, 1

    @staticmethod
    def device_synchronize():
        pass

    class Context:
        @staticmethod
        def from_instance(inst, **kw):
            return _FakeCtx()


def test_time_to_target_chunks_long_runs_and_keeps_the_ladder():
    """Runs split into solve calls of `chunk` passes report the same totals and
    ladder as one call (first pass at or below each decade)."""
    one = bench.time_to_target(_FakePdr, None, 0, 1, 1e-8, 100, chunk=100)
    many = bench.time_to_target(_FakePdr, None, 0, 1, 1e-8, 100, chunk=3)
    for r in (one, many):
        assert r["reached"] and (r["sweeps_fp32"], r["sweeps_fp64"]) == (4, 4)
        first = {k: v["sweeps"] for k, v in r["rungs"].items()}
        assert first == {"10000.0": 0, "1000.0": 0, "100.0": 0, "10.0": 0, "1.0": 0, "0.1": 0,
                         "0.01": 1, "0.0001": 3, "1e-06": 5, "1e-08": 7}
        assert r["handover_at_pass"] == 4 and "extrapolation" not in r
    # the FP32 floor is read after a call that ends in FP32
    assert one["z_fp32_floor"] is None and many["z_fp32_floor"] == 1e-12
    capped = bench.time_to_target(_FakePdr, None, 0, 1, 1e-8, 5, chunk=2)
    assert not capped["reached"] and capped["sweeps_fp32"] + capped["sweeps_fp64"] == 5


def test_time_to_target_wall_time_limit_and_extrapolation():
    """A run stopped by its time limit reports the rungs it reached and the
    passes still needed at its last measured descent rate, as an extrapolation."""
    r = bench.time_to_target(_FakePdr, None, 0, 1, 1e-8, 100, chunk=3, seconds=1e-12)
    assert not r["reached"] and r["sweeps_fp32"] + r["sweeps_fp64"] == 3
    assert r["rungs"]["0.01"]["sweeps"] == 1 and r["rungs"]["1e-06"] is None
    ex = r["extrapolation"]
    # z falls 10x per pass: from z = 1e-3 after 3 passes, 5 more passes to 1e-8
    assert "not measured" in ex["kind"]
    assert abs(ex["further_passes"] - 5.0) < 1e-9 and abs(ex["total_passes"] - 8.0) < 1e-9
