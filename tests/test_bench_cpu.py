"""Host-side parts of bench.py, on the CPU: the algorithmic bytes per
cell-stage, the refusal of more than one GPU, and the profile summaries the
roofline figures are read from."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("dim,ncomp,precision,expect", [
    (1, 1, "fp64", 45.33), (1, 3, "fp64", 136.0), (1, 3, "mixed", 100.0),
    (2, 1, "fp64", 69.33), (2, 4, "fp64", 277.33), (2, 4, "mixed", 181.33)])
def test_algorithmic_bytes_per_cell_stage(dim, ncomp, precision, expect):
    """Stage 0 reads the state and writes the output and v^n (w^n); stages 1
    and 2 read the state and the step's base and write the output.  Averaged
    over the three stages."""
    avg = sum(bench.stage_bytes(dim, ncomp, precision, s) for s in range(3)) / 3.0
    assert abs(avg - expect) < 0.01, (dim, ncomp, precision, avg)
    # the same by hand for 2D Euler FP64: 96 B of state, 32 B of averages
    if (dim, ncomp, precision) == (2, 4, "fp64"):
        state, ubar, mom = 4 * 8 + 2 * 4 * 8, 4 * 8, 2 * 4 * 8
        assert bench.stage_bytes(2, 4, "fp64", 0) == state + state + mom
        assert bench.stage_bytes(2, 4, "fp64", 1) == state + (ubar + mom) + state


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.parametrize("dim", [1, 2])
def test_profile_summaries_parse(dim):
    """The committed counter summaries carry the figures bench.py reads: the
    source hash they were taken on, HBM bytes per launch and the flops per
    cell-stage of both precisions, with the algorithmic flops below the
    executed ones (the useful fraction of the lanes)."""
    rec = bench.recorded_counters(dim)
    assert rec["source_sha256"] and len(rec["source_sha256"]) == 16
    for prec in ("mixed", "fp64"):
        assert float(rec[f"hbm_bytes_per_launch_{prec}"]) > 0
        ex = float(rec[f"executed_flops_per_cell_stage_{prec}"])
        al = float(rec[f"algorithmic_flops_per_cell_stage_{prec}"])
        assert 0 < al < ex


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_traffic_reported_only_for_current_counters(precision):
    """Measured HBM bytes enter the line only when the counters were taken on
    the current kernel source and on the same workload, for either precision."""
    class Case:
        dim, name = 2, bench.COUNTERS[2][2]
    rec = {f"hbm_bytes_per_launch_{precision}": "1.5e9"}

    def roofline():
        return ({"bound": "alu", "avg_launch_ms": 0.5},
                {"achieved_algorithmic": 1000.0})
    roof, hbm = roofline()
    bench.attach_traffic(roof, hbm, rec, precision, Case, True)
    assert roof["traffic"] == 1.5e9 and roof["counters_current"] is True
    assert abs(hbm["achieved_measured"] - 3000.0) < 1e-9
    assert abs(hbm["measured_over_algorithmic"] - 3.0) < 1e-12
    roof, hbm = roofline()
    bench.attach_traffic(roof, hbm, rec, precision, Case, False)  # stale source hash
    assert roof["traffic"] is None and "achieved_measured" not in hbm
    Case.name = "euler2d-batch64"  # counters were taken on another workload
    roof, hbm = roofline()
    bench.attach_traffic(roof, hbm, rec, precision, Case, True)
    assert roof["traffic"] is None


@pytest.mark.parametrize("dim", [1, 2])
def test_committed_counters_are_those_of_the_current_sources(dim):
    """The counter summaries under profiles/ were taken on the kernel sources,
    the work-list builder and the per-file compiler flags as committed, so
    that bench.py reports their HBM traffic rather than null; a change to any
    of them must come with re-taken counters."""
    assert "paper_2402_03074_amd/build.py" in bench.COUNTERS[dim][3]
    assert bench.recorded_counters(dim)["source_sha256"] == bench.kernel_source_hash(dim)
