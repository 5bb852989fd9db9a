"""Host logic of the benchmark (no GPU): the batch sizing of the time-to-1% runs, the
algorithmic work behind the roofline figures, and the use of committed counter summaries."""
import json
import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1805_10164_amd import inputs  # noqa: E402


def test_next_batch_reaches_one_percent_in_one_more_batch():
    # sigma ~ 1/sqrt(n): with sigma/I = 4% after 4096 walkers, 1% needs 16x as many
    done, I, s = 4096, 2.0, 0.08
    b = bench.next_batch(done, I, s, 4096, 1 << 24)
    total = done + b
    assert total == int(1.2 * done * 16)
    assert s * math.sqrt(done / total) <= 0.01 * I


def test_next_batch_bounds():
    # at least the first batch, at most what the scratch holds, doubling without a sigma
    assert bench.next_batch(4096, 2.0, 0.0201, 4096, 1 << 24) >= 4096
    assert bench.next_batch(4096, 2.0, 10.0, 4096, 100_000) == 100_000 - 4096
    assert bench.next_batch(1024, 1.0, 0.0, 1024, 1 << 24) == 1024
    assert bench.next_batch(1024, 0.0, 0.5, 1024, 1 << 24) == 1024


def test_kernel_work_of_the_wire():
    wl = inputs.WIRE_W10_L100
    N, n, nE = wl.N, wl.N + 2, wl.n_energies
    # one alias entry (FP64 threshold + int32 alias) per step: 12 algorithmic bytes
    assert bench.kernel_work("walk_kernel", wl, 1e8) == ("hbm", 1e8 * 12 / 1e9, "GB")
    bound, amount, unit = bench.kernel_work("cholesky_kernel", wl, 0)
    assert (bound, unit) == ("mfma", "TFLOP")
    assert amount == pytest.approx(nE * (N ** 3 / 3 + 2 * N * N) / 1e12)
    _, amount, _ = bench.kernel_work("fullinv_kernel", wl, 0)
    assert amount == pytest.approx(nE * 8 * wl.W ** 3 * wl.L * (wl.L - 1) / 1e12)
    _, amount, _ = bench.kernel_work("alias_build_kernel", wl, 0)
    assert amount == pytest.approx(nE * (8 * N * N + 6 * n * n) / 1e9)
    assert bench.kernel_work("lead_sigma_kernel", wl, 0) is None


def test_roofline_fraction():
    wl = inputs.WIRE_W10_L100
    r = bench.roofline("walk_kernel", wl, 0.5, 1e8)
    assert r["achieved"] == pytest.approx(1.2 / 0.5e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
    # the packed 4-byte entries the walker reads, beside the algorithmic bytes
    assert r["steps_per_s"] == pytest.approx(1e8 / 0.5e-3)
    assert r["entry_gbs"] == pytest.approx(0.4 / 0.5e-3)
    assert r["entry_frac"] == pytest.approx(r["frac"] / 3)
    r = bench.roofline("cholesky_kernel", wl, 3.0, 0)
    assert r["unit"] == "TFLOP/s" and r["frac"] == pytest.approx(r["achieved"] / 78.6)


def test_traffic_rate():
    r = bench.add_traffic_rate({"traffic": 2e9, "avg_launch_ms": 0.5})
    assert r["traffic_gbs"] == pytest.approx(4000.0)
    assert r["traffic_frac_of_hbm_peak"] == pytest.approx(0.5)
    assert "traffic_gbs" not in bench.add_traffic_rate({"traffic": None, "avg_launch_ms": 0.5})
    r = bench.add_traffic_rate({"traffic": 2e9, "avg_launch_ms": 0.5, "unit": "GB/s",
                                "algorithmic_per_launch": 1.2e9})
    assert r["useful_fraction_of_traffic"] == pytest.approx(0.6)
    r = bench.add_traffic_rate({"traffic": 2e9, "avg_launch_ms": 0.5, "unit": "TFLOP/s",
                                "algorithmic_per_launch": 1e12})
    assert "useful_fraction_of_traffic" not in r


def test_measured_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    # a summary counts only while the kernel's source is the one that was profiled
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel v1")
    prof = tmp_path / "profiles"
    prof.mkdir()
    import hashlib
    rec = {"source": str(src), "source_sha256": hashlib.sha256(b"kernel v1").hexdigest(),
           "hbm_bytes_per_launch": 123.0}
    (prof / "k_kernel_w_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    monkeypatch.setattr(bench, "ROOT", "/")
    assert bench.measured_traffic("k_kernel", "w") == 123.0
    src.write_bytes(b"kernel v2")
    assert bench.measured_traffic("k_kernel", "w") is None
    assert bench.measured_traffic("missing_kernel", "w") is None


def test_committed_summaries_name_existing_sources():
    # every committed traffic summary points at a source file of the library
    prof = os.path.join(ROOT, "profiles")
    for f in os.listdir(prof):
        if f.endswith("_traffic.json"):
            rec = json.load(open(os.path.join(prof, f)))
            assert os.path.exists(os.path.join(ROOT, rec["source"])), f
            assert rec["hbm_bytes_per_launch"] > 0, f


def test_window_plan_holds_whole_steps_within_the_timer():
    for steps, per, cap in ((20, 66, 512), (3, 66, 512), (1, 512, 512), (100, 7, 512), (5, 1, 2)):
        plan = bench.window_plan(steps, per, cap)
        assert sum(plan) == steps and all(n * per <= cap for n in plan)
    with pytest.raises(RuntimeError):
        bench.window_plan(2, 600, 512)


class FakeTimes:
    """Stands in for the library's launch timer: records at most `cap` launches of a window
    and counts the rest as dropped, as the library does."""
    cap = 512

    def __init__(self):
        self.records, self.dropped = [], 0

    def __enter__(self):
        FakeTimes.current = self
        return self

    def __exit__(self, *exc):
        FakeTimes.current = None
        return False

    @classmethod
    def launch(cls, name, ms):
        w = cls.current
        if len(w.records) < cls.cap:
            w.records.append((name, ms))
        else:
            w.dropped += 1


def test_timed_records_cover_every_step(monkeypatch):
    # a step of 66 launches (8 of them walker launches of 0.5 ms) timed for 20 steps: every
    # launch is recorded, so per-launch figures and per-step sums cover all 20 steps
    monkeypatch.setattr(bench.M, "LaunchTimes", FakeTimes)

    def step():
        for i in range(66):
            FakeTimes.launch("walk_kernel" if i < 8 else "other_kernel", 0.5 if i < 8 else 0.1)

    rec = bench.timed_records(20, 66, step)
    assert len(rec) == 20 * 66
    pk = bench.per_kernel_table(rec, 20)
    assert pk["walk_kernel"]["launches"] == 160
    assert pk["walk_kernel"]["ms_per_launch"] == pytest.approx(0.5)
    assert pk["walk_kernel"]["ms_per_step"] == pytest.approx(4.0)
    assert sum(v["ms_per_step"] for v in pk.values()) == pytest.approx(4.0 + 58 * 0.1)


def test_a_window_that_drops_records_raises(monkeypatch):
    monkeypatch.setattr(bench.M, "LaunchTimes", FakeTimes)

    def step():
        for _ in range(66):
            FakeTimes.launch("k", 1.0)

    with FakeTimes() as lt:
        for _ in range(20):
            step()
    assert lt.dropped == 20 * 66 - 512
    with pytest.raises(RuntimeError):
        bench.require_complete(lt)
    # a plan that claims fewer launches per step than are issued also overflows and raises
    with pytest.raises(RuntimeError):
        bench.timed_records(20, 10, step)


def test_realized_errors_at_the_stop():
    r = bench.realized_errors([1.01, 0.98], [1.0], 1.0)
    assert r["mc_rel_err_at_stop"] == pytest.approx([0.01, 0.02])
    assert r["mc_rel_err_at_stop_max"] == pytest.approx(0.02)
    assert r["mc_energy_sampled_rel_err_at_stop"] == [0.0]
