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
    for name in ("main", "run_batch", "cpu_baseline", "spmm_bytes", "cheb_bytes", "train_guess_network"):
        assert callable(getattr(bench, name)), name
    # algorithmic bytes: matrix (values + indices) once, row pointers, X read and Y written
    assert bench.spmm_bytes(10, 30, 2) == 12 * 30 + 4 * 11 + 2 * 8 * 10 * 2
