"""Host-side parts of bench.py (no GPU): the refusal of more than one GPU, the
CPU oracle worker of the multi-core baseline, and the modelled oracle time
of a bounded sample."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_cpu_worker_prints_its_modelled_time():
    core = sorted(os.sched_getaffinity(0))[0]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    p = subprocess.run([sys.executable, BENCH, "--cpu-worker", "--workload", "disk256", "--cpu-iters", "16",
                        "--cpu-arn", "1e6", "--cpu-core", str(core)], capture_output=True, text=True, timeout=300,
                       env=env)
    assert p.returncode == 0, p.stderr[-500:]
    rec = json.loads(p.stdout.strip().splitlines()[-1])
    assert rec["core"] == core
    assert rec["t_total"] > 0.0 and rec["spent"] > 0.0


def test_oracle_sample_scales_with_products_and_gram_schmidt_work():
    """The modelled time grows with the number of products the GPU solve
    used (one timed product per case, scaled by the count) and with the
    Gram-Schmidt work of its Krylov steps (a measured cost per unit)."""
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    wl = W.workload_disk256()
    t1, spent1, rows, mv, c = bench.oracle_sample(wl, [1], [0.0])
    # modelled counts far above the timing noise of the sampled rows
    t100, _, _, _, _ = bench.oracle_sample(wl, [100000], [0.0])
    assert rows == wl.problems[0].order and mv == wl.problems[0].order
    assert t100 > t1 > 0.0 and spent1 > 0.0 and c > 0.0
    units = 1e11
    ta, _, _, _, ca = bench.oracle_sample(wl, [1], [units])
    assert ta > t1 + 0.5 * ca * units


def test_gram_schmidt_units_of_restarted_gmres():
    """Step j of a cycle projects on j + 1 basis vectors: a run of s steps
    with restart m is full cycles of m(m+1)/2 and a last one of r(r+1)/2
    (r = s mod m), times n rows, summed over right-hand sides."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.arnoldi_units([3], 100, 10) == 6 * 10
    assert bench.arnoldi_units([127, 92], 100, 8192) == (5050 + 27 * 28 // 2 + 92 * 93 // 2) * 8192
    assert bench.arnoldi_units([200], 100, 1) == 2 * 5050
    assert bench.arnoldi_units([0], 100, 5) == 0


def test_oracle_full_solve_is_timed_end_to_end():
    """The disk of 256 elements is solved by the oracle in full (assembly,
    GMRES(50) to 1e-10, far field) and converges."""
    sys.path.insert(0, ROOT)
    import bench
    r = bench.oracle_full_solve()
    assert r["converged"] and r["seconds_per_solve"] > 0.0 and r["value"] == 1.0 / r["seconds_per_solve"]
    assert 5 <= r["gmres_iterations"] <= 50


def test_benchmark_matrices_have_128_byte_aligned_columns():
    """padded_ld rounds the order up to 8 complex128 / 16 complex64 entries
    and leaves multiples alone."""
    sys.path.insert(0, ROOT)
    import bench

    class P:  # precision constants as the binding defines them
        F64, F32 = 0, 1

    assert bench.padded_ld(14970, P.F64, P) == 14976
    assert bench.padded_ld(8192, P.F64, P) == 8192
    assert bench.padded_ld(602, P.F32, P) == 608
    assert bench.padded_ld(32768, P.F32, P) == 32768
    for n in range(1, 200):
        for prec, per, esz in ((P.F64, 8, 16), (P.F32, 16, 8)):
            ld = bench.padded_ld(n, prec, P)
            assert n <= ld < n + per and (ld * esz) % 128 == 0
