"""Host-side logic of bench.py (no GPU): the algorithmic byte count of a
stage-kernel launch against a count written out here from its definition,
and the refusal of a run on more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stage_bytes_counts_each_datum_once():
    N, K, rb = 7, 3, 8
    npn = (N + 1) ** 2
    for k in range(5):
        reads = 3 + (3 if k > 0 else 0) + 4 + 2          # W, dU (not on the first stage), metric, b_x b_y
        writes = 3 + (3 if k < 4 else 0)                 # W, dU (not on the last stage)
        per_elem = 4 * (N + 1) + 1                       # face bathymetry, viscosity
        records = 12 * (N + 1) if k == 4 else 0          # last stage: face records (h, u, v)
        want = ((reads + writes) * npn * K + (per_elem + records) * K) * rb
        assert bench.stage_bytes(N, K, True, rb, k) == want
        assert bench.stage_bytes(N, K, False, rb, k) == want - K * rb
        assert bench.stage_bytes(N, K, True, rb, k, limiter=False) == want - records * K * rb
    # viscous elements add their face fluxes and viscous terms
    extra = bench.stage_bytes(N, K, True, rb, 2, n_visc=2) - bench.stage_bytes(N, K, True, rb, 2)
    assert extra == (16 * (N + 1) + 2 * npn) * 2 * rb
    # about 140 bytes per node on average over the five stages at N = 7 in FP64
    avg = sum(bench.stage_bytes(N, 262144, True, 8, k) for k in range(5)) / 5 / (262144 * npn)
    assert abs(avg - (138.53 + 96 * 8 / 64 / 5)) < 0.01


def test_stage_bytes_low_degree_fp64_reads_coordinates():
    """In FP64 at N <= 4 the stage kernel forms the metric terms from two
    coordinates per node instead of reading four metric terms; FP32 and
    N >= 5 read the four, FP32 also the four of each element's middle node
    (the stored ones are relative to them)."""
    K = 3
    for N in (2, 3, 4, 5, 8):
        npn = (N + 1) ** 2
        for rb, geo, geo_e in ((8, 2 if N <= 4 else 4, 0), (4, 4, 4)):
            per_elem = 4 * (N + 1) + geo_e + 1
            want = ((3 + 3 + geo + 2 + 3 + 3) * npn * K + per_elem * K) * rb
            assert bench.stage_bytes(N, K, True, rb, 2) == want
            assert bench.rhs_bytes(N, K, True, rb) == ((3 + geo + 2 + 3) * npn * K + per_elem * K) * rb


def test_dt_pass_bytes():
    N, K, rb = 7, 5, 8
    nf = N + 1
    # per element: CFL and viscous bound; per face node: record (3) and face geometry (3); face map 5 B per side
    assert bench.dt_pass_bytes(N, K, True, rb) == K * ((2 + 4 * nf * 6) * rb + 4 * 5)
    assert bench.dt_pass_bytes(N, K, False, rb) == K * ((1 + 4 * nf * 6) * rb + 4 * 5)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
