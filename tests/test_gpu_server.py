"""GPU tests of the serving loop (acs_server_*): a mixed LP/SOCP request
stream with staggered arrivals, each result checked by the FP64 oracle and
equal to the same problem solved alone (bitwise: the pool path against a
batch of one, the worker path against acs_solve), admission under an HBM
budget, oversize rejection and cancellation."""
import time

import numpy as np
import pytest

from oracle.kkt import kkt_errors
from paper_2103_00736_amd import acs, synth

pytestmark = pytest.mark.gpu

SMALL_NNZ = 60_000


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert acs.lib().acs_init(0) == acs.ACS_OK, acs.lib().acs_last_error()


def _stream(k=10):
    """Serving-recipe requests (6 nonzeros per column, n = 3m, SOC sizes U{3..30}), small m."""
    rng = np.random.default_rng(11)
    out = []
    for i in range(k):
        kind = "socp" if i % 3 == 2 else "lp"
        m = int(np.exp(rng.uniform(np.log(300), np.log(6000))))
        out.append(synth.Request(i, 0.0, kind, m).problem())
    return out


def test_mixed_stream_matches_oracle_and_alone():
    probs = _stream()
    handles = [acs.Problem.from_synth(p) for p in probs]
    srv = acs.Server(hbm_budget=8 << 30, max_slots=64, small_nnz=SMALL_NNZ, workers=3, tick_iters=40)
    tickets = []
    for i, h in enumerate(handles):  # staggered arrivals: later ones join running ticks
        tickets.append(srv.submit(h, eps_kkt=1e-4))
        if i % 3 == 2:
            time.sleep(0.05)
    results = [srv.wait(t, 120_000) for t in tickets]
    st = srv.stats()
    print("stats", st)
    assert st["completed"] == len(probs) and st["running"] == 0 and st["bytes_in_use"] == 0
    for p, h, (x, y, z, info) in zip(probs, handles, results):
        rec = kkt_errors(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, x, y, z)
        path = "pool" if p.nnz <= SMALL_NNZ else "worker"
        print(f"{p.name} nnz={p.nnz} {path}: status={info.status} it={info.iterations} kkt={rec['kkt']:.2e} "
              f"lat={info.latency_ms:.1f}ms queue={info.queue_ms:.1f}ms")
        assert info.status == acs.SOLVED
        assert rec["kkt"] <= 1.05e-4
        if path == "pool":
            b = acs.Batch([h], eps_kkt=1e-4)
            b.run(20000)
            xa, ya, za, ia = b.result(0)
        else:
            xa, ya, za, ia = acs.solve(h, eps_kkt=1e-4)
        assert np.array_equal(x, xa) and np.array_equal(y, ya) and np.array_equal(z, za), p.name
        assert ia.iterations == info.iterations
    srv.close()


def test_budget_backpressure_and_rejection():
    probs = [synth.config3(i, m=m) for i, m in enumerate([400, 380, 360, 340, 320])]
    handles = [acs.Problem.from_synth(p) for p in probs]
    one = max(h.batch_device_bytes() for h in handles)  # every request goes to the pool here
    srv = acs.Server(hbm_budget=int(2.5 * one), max_slots=8, small_nnz=1 << 30, workers=1, tick_iters=25)
    tickets = [srv.submit(h) for h in handles]
    res = [srv.wait(t, 120_000) for t in tickets]
    st = srv.stats()
    assert st["peak_running"] <= 3
    assert all(r[3].status == acs.SOLVED for r in res)
    assert max(r[3].queue_ms for r in res) > 0.0
    big = acs.Problem.from_synth(synth.config3(0, m=3000))
    with pytest.raises(acs.AcsError) as ei:
        srv.submit(big)
    assert ei.value.code == acs.ACS_ERR_NOMEM
    srv.close()


def test_cancel():
    srv = acs.Server(hbm_budget=1 << 30, max_slots=1, small_nnz=1 << 30, workers=1, tick_iters=5)
    a = srv.submit(acs.Problem.from_synth(synth.config3(1, m=600)), max_iter=20000)
    b = srv.submit(acs.Problem.from_synth(synth.config3(2, m=600)))
    srv.cancel(b)  # still queued behind a: cancelled without running
    rb = srv.wait(b, 60_000)
    assert rb[3].status == acs.CANCELLED
    srv.cancel(a)
    ra = srv.wait(a, 60_000)
    assert ra[3].status in (acs.CANCELLED, acs.SOLVED)
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


def test_pool_k_iterations_match_oracle():
    """Requests stopped after 20 iterations on the server's pool path (the
    persistent kernel's ticks, other requests resident alongside): x, z and
    y of iteration 20 against 20 iterations of the literal FP64 oracle."""
    from oracle.alg2 import Algorithm2, default_parameters
    from tests._parity import assert_close, errors, fmt

    k = 20
    probs = [synth.config3(0, m=120), synth.socp_percol(80, 240, 3, 41, 3, 12, 0.8)]
    others = _stream(4)
    srv = acs.Server(hbm_budget=8 << 30, max_slots=64, small_nnz=10 ** 9, workers=1, tick_iters=7)
    handles = [acs.Problem.from_synth(p) for p in probs + others]
    tickets = [srv.submit(h, eps_kkt=1e-14, max_iter=(k if i < len(probs) else 60), cg_reduce=1e-7, cg_max=4000,
                          check_every=1000000) for i, h in enumerate(handles)]
    res = [srv.wait(t, 120_000) for t in tickets]
    srv.close()
    for p, (x, y, z, info) in zip(probs, res[:len(probs)]):
        t, L = default_parameters(p.soc_sizes)
        alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
        for _ in range(k):
            alg.step()
        errs = errors({"x": x, "z": z, "y": y}, {"x": alg.x, "z": alg.z, "y": alg.dual_multiplier()}, ("x", "z", "y"))
        print(f"{p.name}: status={info.status} it={info.iterations} {fmt(errs)}")
        assert info.status == acs.MAX_ITER and info.iterations == k
        assert_close(errs, 1e-5, p.name)
