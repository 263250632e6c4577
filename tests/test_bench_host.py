"""Host logic of the benchmark (no GPU): the one-GPU guard, the serving
statistics and the lookup of committed counter summaries."""
import glob
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "error" in json.loads(r.stdout.strip().splitlines()[-1])


def test_percentile_picks_an_observed_value():
    v = list(range(1, 1001))
    assert bench._pct(v, 0.5) == 501
    assert bench._pct(v, 0.99) == 990
    assert bench._pct([7], 0.99) == 7
    assert bench._pct([], 0.5) is None


def test_serve_stats_over_two_halves():
    def part(lat_ms, iters):
        lat = [x / 1e3 for x in lat_ms]
        return {"lat": lat, "ph": {"admit": [0.0] * len(lat), "run": lat}, "bytes": 1000 * len(lat), "span": 0.5,
                "iters": iters}

    a = part([1.0] * 99 + [5.0], 100)
    b = part([1.0] * 98 + [2.0, 3.0], 50)
    st = bench._serve_stats(100, [a, b], sizes=[1000, 3000])
    assert st["requests"] == 200
    assert st["requests_per_iteration"] == round(200 / 150, 3)
    # each half's own p99, then the p99 over both
    assert st["p99_halves_ms"] == [bench._pct(a["lat"], 0.99) * 1e3, bench._pct(b["lat"], 0.99) * 1e3]
    assert st["p99_ms"] == round(bench._pct(a["lat"] + b["lat"], 0.99) * 1e3, 3)
    assert st["GBps"] == round(200 * 1000 / 1.0 / 1e9, 2)
    assert st["offered_GBps"] == round(100 * 2000 / 1e9, 2)


def test_traffic_only_for_the_profiled_source_and_containers():
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "k_decode_*_traffic.json")))
    assert paths
    sha = bench._src_hash(os.path.join(ROOT, "paper_2411_05239_amd", "csrc", "decode.hip"))
    for path in paths:
        rec = json.load(open(path))
        name = os.path.basename(path)[len("k_decode_"):-len("_traffic.json")]
        wl = next(w for w in ("ckpt8b_delta_zg", "ckpt8b_delta", "ckpt8b", "fp32_256mb") if name.startswith(w))
        alg = rec["algorithmic_bytes_per_launch"]
        got = bench._traffic(wl, alg)
        if rec["decode_src_sha"] == sha:
            assert got == rec["hbm_bytes_per_launch"], path
        # other containers (another chunk size: other algorithmic bytes) get none
        assert bench._traffic(wl, alg + 1) is None
