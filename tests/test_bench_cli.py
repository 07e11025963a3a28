"""bench.py's command line on the CPU: it imports, exposes its entry points,
and refuses more than one GPU with a message and exit status 2."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_entry_points():
    sys.path.insert(0, str(ROOT))
    import bench
    for name in ("main", "run_batch", "cpu_baseline", "cpu_baseline_pcg_rate", "spmm_bytes", "cheb_bytes",
                 "train_guess_network", "_check_physics"):
        assert callable(getattr(bench, name)), name
    # algorithmic bytes: matrix (values + indices) once, row pointers, X read and Y written
    assert bench.spmm_bytes(10, 30, 2) == 12 * 30 + 4 * 11 + 2 * 8 * 10 * 2


def test_traffic_lookup_never_raises_and_matches_committed_sources():
    """The roofline's traffic figure comes from the committed counter
    summaries; a record whose sources changed, an unknown workload or kernel
    gives None, and the record of the default workload (the 40-atom cluster on
    its P2 space) matches the current kernel sources."""
    import bench
    assert bench._traffic("no such kernel", "c2", 0, "fp64") is None
    assert bench._traffic("k_cheb_small<5, 4, 4, 256, 4, double>", "c1", 0, "fp64") is None
    t2 = bench._traffic(bench._kernel_name("cheb_step", 52, 4, 2009635), "c3", 0, "fp32ir", order=2)
    assert t2 is not None and 2e9 < t2 < 2e10, t2
    # the P1 summary may predate the current sources: then no figure, never a stale one
    t1 = bench._traffic(bench._kernel_name("cheb_step", 52, 4, 2004523), "c3", 0, "fp32ir", order=1)
    assert t1 is None or 1e9 < t1 < 5e9, t1


def test_physics_check_exits_on_invalid_results():
    """A step result with a wrong electron count, an inner loop stopped by its
    cap or overlapping orbitals ends bench.py with exit status 3; a valid one
    passes."""
    import pytest
    sys.path.insert(0, str(ROOT))
    import bench
    ok = {"eigenvalues_sorted": [-1.0, -0.5], "max_offdiag_overlap": 1e-4, "rho_integral": 4.0, "electrons": 4.0,
          "energy": -3.0, "inner_iters": 12, "inner_last_diff": 1e-11, "inner_converged": True}
    bench._check_physics(ok, 1e-2, "c2")
    for change in ({"rho_integral": 3.9}, {"inner_converged": False}, {"max_offdiag_overlap": 0.2},
                   {"eigenvalues_sorted": [float("nan"), -0.5]}):
        with pytest.raises(SystemExit) as e:
            bench._check_physics(dict(ok, **change), 1e-2, "c2")
        assert e.value.code == 3, change
