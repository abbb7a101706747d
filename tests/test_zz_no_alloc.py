"""acs_solve_device_noalloc: the solve that allocates no device memory.

It must give the results of acs_solve_device (same kernels, same arithmetic;
only where the instance's arrays live differs), on two calls in a row, the
second on a smaller problem, so that the second runs over the first one's
leftovers in the shared scratch array.  Sizes beyond the array are refused
before any GPU work.
"""
import numpy as np
import pytest

from paper_2103_00736_amd import acs, synth

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def _solve_both(p, stream):
    import torch

    dev = torch.device("cuda:0")
    prob = acs.Problem.from_synth(p)
    out = {}
    with torch.cuda.stream(stream):
        for kind, fn in (("alloc", acs.solve_device), ("noalloc", acs.solve_device_noalloc)):
            xd = torch.full((p.n,), float("nan"), dtype=torch.float64, device=dev)
            yd = torch.full((p.m,), float("nan"), dtype=torch.float64, device=dev)
            zd = torch.full((p.n,), float("nan"), dtype=torch.float64, device=dev)
            info = fn(prob, xd.data_ptr(), yd.data_ptr(), zd.data_ptr(), stream=stream.cuda_stream,
                      eps_kkt=1e-4, max_iter=20000)
            out[kind] = (xd.cpu().numpy(), yd.cpu().numpy(), zd.cpu().numpy(), info)
    stream.synchronize()
    return out


def test_noalloc_matches_solve_device_on_two_calls_in_a_row():
    import torch

    assert acs.lib().acs_init(0) == acs.ACS_OK
    s = torch.cuda.Stream(device=torch.device("cuda:0"))
    big = synth.config3(10)                 # 320 x 800
    small = synth.config3(0, m=60)          # 60 x 150, solved second, over the first one's leftovers
    assert small.n < big.n and small.m < big.m
    for p in (big, small):
        prob = acs.Problem.from_synth(p)  # held: the handle dies with the object
        need = acs.lib().acs_problem_device_bytes(prob.handle, acs.PREC_MIXED)
        assert 0 < need <= SCRATCH_BYTES
        print(f"case {p.name}: m={p.m} n={p.n} nnz={p.nnz} device bytes {need}", flush=True)
        r = _solve_both(p, s)
        xa, ya, za, ia = r["alloc"]
        xn, yn, zn, inn = r["noalloc"]
        assert ia.status == inn.status == acs.SOLVED
        assert ia.iterations == inn.iterations and ia.cg_steps == inn.cg_steps
        assert ia.kkt == inn.kkt and ia.pobj == inn.pobj
        assert np.array_equal(xa, xn) and np.array_equal(ya, yn) and np.array_equal(za, zn)
        obj_err = abs(inn.pobj - p.p_star) / (1.0 + abs(p.p_star))
        print(f"  {p.name}: {inn.iterations} iterations, kkt {inn.kkt:.2e}, objective error {obj_err:.1e}",
              flush=True)
        assert inn.kkt <= 1e-4 and obj_err <= 1e-4


def test_noalloc_default_stream_and_refusals():
    import torch

    dev = torch.device("cuda:0")
    p = synth.config0()
    prob = acs.Problem.from_synth(p)
    xd = torch.zeros(p.n, dtype=torch.float64, device=dev)
    yd = torch.zeros(p.m, dtype=torch.float64, device=dev)
    zd = torch.zeros(p.n, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    # no stream: the library's own, set up once
    info = acs.solve_device_noalloc(prob, xd.data_ptr(), yd.data_ptr(), zd.data_ptr(), eps_kkt=1e-4)
    x, y, z, ref = acs.solve(prob, eps_kkt=1e-4)
    assert info.status == ref.status == acs.SOLVED and info.iterations == ref.iterations
    assert np.array_equal(xd.cpu().numpy(), x) and np.array_equal(zd.cpu().numpy(), z)
    assert np.array_equal(yd.cpu().numpy(), y)
    # larger than the scratch array: refused before any GPU work
    q = synth.lp_uniform(100_000, 400_000, 2_000_000, seed=7, name="too_big")
    qp = acs.Problem.from_synth(q)
    assert acs.lib().acs_problem_device_bytes(qp.handle, acs.PREC_MIXED) > SCRATCH_BYTES
    with pytest.raises(acs.AcsError) as e:
        acs.solve_device_noalloc(qp, 0, 0, 0)
    assert e.value.code == acs.ACS_ERR_NOMEM
    # the direct projection needs memory of its own
    with pytest.raises(acs.AcsError) as e:
        acs.solve_device_noalloc(prob, 0, 0, 0, projection=acs.PROJ_FACTOR)
    assert e.value.code == acs.ACS_ERR_ARG
    # a host pointer is refused
    host = np.zeros(p.n)
    with pytest.raises(acs.AcsError) as e:
        acs.solve_device_noalloc(prob, host.ctypes.data, 0, 0)
    assert e.value.code == acs.ACS_ERR_ARG
    # and the scratch still serves a solve afterwards
    info2 = acs.solve_device_noalloc(prob, xd.data_ptr(), yd.data_ptr(), zd.data_ptr(), eps_kkt=1e-4)
    assert info2.iterations == ref.iterations and np.array_equal(xd.cpu().numpy(), x)
