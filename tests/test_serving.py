"""Continuous-batching service: results identical alone and in the mix; admission by footprint."""
import numpy as np
import pytest

from harness import unit_cube_problem, die_problem
from tests.conftest import cached


def _pool():
    return [cached(("srv", 0), lambda: die_problem(16, 8, 8, seed=0, levels=3)),
            cached(("srv", 1), lambda: die_problem(16, 8, 8, seed=5, levels=3, n_exp=0.3, lam=10.0)),
            cached(("srv", 2), lambda: unit_cube_problem(n=8, block=2, levels=3))]


def test_oversized_request_is_rejected_on_the_host():
    gdsw = pytest.importorskip("paper_2606_01433_amd.gdsw")
    try:
        gdsw.load_library()
    except RuntimeError as e:
        pytest.skip(str(e))
    from paper_2606_01433_amd.serving import Server, Request
    srv = Server.__new__(Server)           # host-side checks only: no scheduler thread, no GPU
    srv.budget = 1024
    srv._footprints = {}
    with pytest.raises(ValueError, match="more than the whole budget"):
        Server.submit(srv, Request(0, _pool()[0]))


@pytest.mark.gpu
def test_results_identical_alone_and_in_the_mix():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_01433_amd.serving import Server, Request
    pool = _pool()
    opts = [dict(tol=1e-8), dict(tol=1e-8, precision="mixed"), dict(tol=1e-10)]
    print("[gpu] serving alone", flush=True)
    alone = []
    srv = Server(max_active=1)
    for k, (P, o) in enumerate(zip(pool, opts)):
        alone.append(srv.submit(Request(k, P, **o)).wait(300))
    srv.close()
    print("[gpu] serving mix", flush=True)
    srv = Server(max_active=6)
    mix = [srv.submit(Request(10 + k, pool[k % 3], **opts[k % 3])) for k in range(9)]
    srv.drain(mix, 300)
    srv.close()
    assert srv.peak_active > 1
    for r in alone + mix:
        assert r.error is None, r.error
        assert r.info["converged"]
    for k, r in enumerate(mix):
        assert np.array_equal(r.x, alone[k % 3].x), k


@pytest.mark.gpu
def test_budget_queues_instead_of_failing():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_01433_amd.serving import Server, Request
    P = _pool()[0]
    probe = Server.__new__(Server)
    probe._footprints = {}
    fp = Server.footprint(probe, Request(0, P))
    srv = Server(budget_bytes=int(1.5 * fp), max_active=4)   # room for one request at a time
    print("[gpu] serving budget", flush=True)
    reqs = [srv.submit(Request(k, P)) for k in range(3)]
    srv.drain(reqs, 300)
    srv.close()
    assert srv.peak_active == 1
    assert all(r.error is None and r.info["converged"] for r in reqs)
    assert np.array_equal(reqs[0].x, reqs[2].x)
