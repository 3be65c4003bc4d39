"""The relative scaled efficiency helper reproduces every percentage of Table 1."""
import os

from paper_2606_01433_amd.metrics import effic_rel, percentile

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")


def _rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        role, n, p, lev, t, eff, it = line.split()
        rows.append((role, float(n), int(p), int(lev), float(t), int(eff), float(it)))
    return rows


def test_table1_efficiencies():
    rows = _rows()
    assert len(rows) == 12
    for role, n, p, lev, t, eff, _ in rows:
        base = [r for r in rows if r[0] == role and r[2] == 2048 and r[3] == 3][0]
        got = 100.0 * effic_rel(t, n, p, base[4], base[1], base[2])
        assert abs(got - eff) <= 1.0, (role, n, p, lev, got, eff)


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert percentile(xs, 50) == 50 and percentile(xs, 99) == 99 and percentile([5.0], 99) == 5.0


def test_bench_traffic_entries_match_the_local_solve_source():
    """The HBM traffic bench.py attaches to its roofline was measured on the current local-solve source
    (otherwise it reports null): every recorded entry carries the hash of the kernel it was taken on."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    h = bench.local_solve_source_hash()
    assert bench.LOCAL_SOLVE_TRAFFIC
    for key, rec in bench.LOCAL_SOLVE_TRAFFIC.items():
        assert rec["source_hash"] == h, key
        assert rec["bytes"] > 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N > 1 exits with a message, before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
