"""Host logic of bench.py (CPU): the use of the committed HBM-traffic summary and the
one-GPU guard."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STATS = dict(steps=100, rjs_steps=90, rvs_steps=10, rjs_fallbacks=0, rjs_trials=150, rvs_triggers=7)


class _Plan:
    def __init__(self, lds_cap):
        self.lds_cap = lds_cap


def _write(tmp_path, sha, stats=STATS, lds_cap=1024):
    p = tmp_path / "traffic.txt"
    keys = ",".join(f"{k}={stats[k]}" for k in bench.TRAFFIC_STATS)
    p.write_text(f"# comment: ignored\nkernel_sources_sha256: {sha}\nplan: 0.1,0,{lds_cap},2,1\n"
                 f"lds_cap: {lds_cap}\nstats: {keys}\nread_kib_per_launch: 1000.5\n"
                 "write_kib_per_launch: 24.5\nread_requests_per_launch: 8004\nwrite_requests_per_launch: 200\n")
    return str(p)


def test_traffic_used_only_for_the_same_kernel_and_decisions(tmp_path, monkeypatch):
    sha = bench.kernel_sources_sha256()
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _write(tmp_path, sha))
    t = bench.measured_traffic(_Plan(1024), dict(STATS, ended_early=3, alg_bytes=9))
    assert t == {"bytes": 1024.0 * 1025.0, "read_requests": 8004.0}
    # another launch decision (trial count) or, with eRVS steps, another LDS cap: no figure
    assert bench.measured_traffic(_Plan(1024), dict(STATS, rjs_trials=151)) is None
    assert bench.measured_traffic(_Plan(512), STATS) is None
    # without eRVS steps the LDS cap does not matter
    no_rvs = dict(STATS, rjs_steps=100, rvs_steps=0)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _write(tmp_path, sha, stats=no_rvs))
    assert bench.measured_traffic(_Plan(512), no_rvs) is not None
    # counters taken on other kernel sources: no figure
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _write(tmp_path, "0" * 64))
    assert bench.measured_traffic(_Plan(1024), STATS) is None
    # no summary at all
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic(_Plan(1024), STATS) is None


def test_committed_summary_parses():
    """The committed summary names every field bench.py reads."""
    kv = {}
    for line in open(os.path.join(ROOT, bench.TRAFFIC_FILE)):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    for k in ("kernel_sources_sha256", "lds_cap", "stats", "read_kib_per_launch", "write_kib_per_launch",
              "read_requests_per_launch"):
        assert k in kv, k
    rec = dict(x.split("=") for x in kv["stats"].split(","))
    assert set(rec) == set(bench.TRAFFIC_STATS)
    assert float(kv["read_kib_per_launch"]) > 0 and len(kv["kernel_sources_sha256"]) == 64


@pytest.mark.timeout(300)
def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU only" in r.stderr and r.stdout == ""


def test_one_off_share():
    """Shares of the one-off costs beside one job, and the jobs on a resident graph after
    which all of them fall below the paper's largest reported share (3.98 %)."""
    r = bench.one_off_share(prep_ms=1.0, profile_ms=9.0, index_ms=40.0, alias_ms=30.0, tune_ms=120.0, job_ms=10.0)
    assert r["paper_like_ms"] == 10.0 and r["all_ms"] == 191.0
    assert abs(r["paper_like_share_one_job"] - 0.5) < 1e-12
    assert abs(r["all_share_one_job"] - 191.0 / 201.0) < 1e-12
    k = r["jobs_for_all_below_3.98pct"]
    assert 191.0 / (191.0 + k * 10.0) < 0.0398 <= 191.0 / (191.0 + (k - 1) * 10.0)


def test_plan_argument_round_trip():
    """--plan text: a bench line's plan_arg reproduces its plan field for field; short
    forms take the library defaults; a wrong field count is refused."""
    p = bench.parse_plan("0.43,0,1024,2,1,64,0,1024,256,1")
    assert bench.plan_dict(p) == {"rho": float(p.rho), "d_lo": 0, "lds_cap": 1024, "bound": 2, "proposal": 1,
                                  "rjs_cap": 64, "grid": 0, "hub_deg": 1024, "hub_lanes": 256, "rvs_share": 1}
    assert bench.plan_dict(bench.parse_plan(bench.plan_arg(p))) == bench.plan_dict(p)
    q = bench.parse_plan("0.5,8,512")
    assert (q.bound, q.proposal, q.rjs_cap, q.hub_deg, q.hub_lanes, q.rvs_share) == (0, 0, 1024, 0, 64, 0)
    with pytest.raises(SystemExit):
        bench.parse_plan("0.5,8")
