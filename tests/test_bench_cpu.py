"""CPU checks of the benchmark's host logic: the roofline arithmetic, the
counter summaries it reads from profiles/ (and drops once the kernel sources
change), the exact-fit recovery measure, and the refusal of more than one
GPU.  No GPU call is made here."""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

MC_SOURCES = ["sabr_dev.h", "sabr_mc.h", "kernels_mc.hip"]


def test_roofline_arithmetic():
    """achieved = flops / time, frac = achieved / 157.3 TFLOP/s; the counter
    summary's traffic and issue rate are carried over."""
    r = bench.roofline(4.915e10 * 32, 0.0584, "sa_kernel", 10)
    assert r["achieved"] == pytest.approx(4.915e10 * 32 / 0.0584 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3)
    assert r["traffic"] is None and r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    r = bench.roofline(1.0e12, 0.5, "k", 1, {"traffic_bytes_per_launch": 123, "valu_insts_per_simd_cycle": 0.2,
                                              "valu_busy_rocprof": 0.8, "file": "profiles/x.md"})
    assert r["traffic"] == 123 and r["valu_insts_per_simd_cycle"] == 0.2 and r["counters_from"] == "profiles/x.md"
    assert "executed_fp32_tflops" not in r
    r = bench.roofline(1.0e12, 0.5, "k", 1, {"executed_fp32_flops_per_unit": 20.0}, units=1e10)
    assert r["executed_fp32_tflops"] == pytest.approx(20.0 * 1e10 / 0.5 / 1e12)
    assert r["executed_fp32_frac"] == pytest.approx(r["executed_fp32_tflops"] / 157.3)


@pytest.mark.parametrize("name,sources", [("counters_sa_kernel_static_surface.md", bench.SA_SOURCES),
                                          ("sa_kernel_dynamic_case1.md", bench.SA_SOURCES),
                                          ("counters_mc_crn_kernel_mc_calibration.md", MC_SOURCES)])
def test_counter_summaries_match_the_committed_sources(name, sources):
    """Every committed counter summary was taken on the kernel sources as they
    stand (its digest matches), and names a positive traffic per launch."""
    d = bench.counter_summary(name, sources)
    assert d is not None, name
    assert d["traffic_bytes_per_launch"] > 0
    assert 0 < d["valu_insts_per_simd_cycle"] < 1
    assert d["executed_fp32_flops_per_unit"] > 0 and d["unit"]


def test_counter_summary_dropped_when_sources_differ(tmp_path, monkeypatch):
    """A summary whose digest does not match the sources is not used."""
    line = {"sources": "0000000000000000", "traffic_bytes_per_launch": 1}
    (tmp_path / "c.md").write_text("# x\n\ncounters: %s\n" % json.dumps(line))
    monkeypatch.setattr(bench, "ROOT_PROFILES", str(tmp_path))
    assert bench.counter_summary("c.md", bench.SA_SOURCES) is None
    line["sources"] = bench.source_digest(bench.SA_SOURCES)
    (tmp_path / "c.md").write_text("counters: %s\n" % json.dumps(line))
    assert bench.counter_summary("c.md", bench.SA_SOURCES)["traffic_bytes_per_launch"] == 1
    assert bench.counter_summary("missing.md", bench.SA_SOURCES) is None


def test_exact_solutions_reproduce_the_surface(oracle):
    """The second exact fit the benchmark accepts for beta = 1 reproduces the
    oracle's vols of the surface (fits 20 and 22 of the workload); beta < 1
    or k >= 0 has the truth alone."""
    from paper_2407_20713_amd import inputs
    fits = inputs.surface_fits()
    gens, lb, ub = inputs.surface_true_params(len(fits))
    two = []
    for k, g in enumerate(fits):
        m = oracle.Market(g.T, g.fwd, g.offs, g.K)
        while True:
            x = inputs.draw_params(gens[k], lb, ub)
            v = oracle.model_vols(m, oracle.STATIC, x, g.meta["beta"])
            if np.all(np.isfinite(v)) and np.all(v > 0):
                break
        sols = bench.exact_solutions(x, g.meta["beta"], float(g.T[0]), lb, ub)
        if len(sols) > 1:
            two.append(k)
            v2 = oracle.model_vols(m, oracle.STATIC, sols[1], g.meta["beta"])
            np.testing.assert_allclose(v2, v, rtol=1e-13)
            assert np.max(np.abs(sols[1] - x)) > 0.05
    assert two == [20, 22]
    assert len(bench.exact_solutions([0.3, 0.2, 0.5], 0.5, 7.0, lb, ub)) == 1


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU: --gpus 2 exits with a message, before
    loading anything."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_latency_by_kind():
    """Serving latencies split by the kind of request, in milliseconds; kinds
    absent from the trace are left out."""
    lat = np.array([0.010, 0.020, 0.030, 1.0, 2.0])
    kind = np.array(["static", "static", "static", "mc", "mc"])
    d = bench.latency_by_kind(lat, kind)
    assert set(d) == {"static", "mc"}
    assert d["static"]["requests"] == 3 and d["static"]["p50_ms"] == pytest.approx(20.0)
    assert d["mc"]["p99_ms"] == pytest.approx(1990.0)
