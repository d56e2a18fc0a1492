"""GPU tests of the serving loop (tsylv_submit / tsylv_poll).

* Continuous batching: requests of different (n, s, p) are submitted
  together; each result must be bitwise identical to the same solve run alone
  through the synchronous tsylv_gmres / tsylv_fom (the serving loop runs the
  same kernels and host arithmetic per request, with fixed-order
  reductions), and the small ones are checked against the oracle's
  Kronecker solution.
* Admission by HBM budget: with an arena that holds about two requests at a
  time, a burst of requests is queued, admitted as memory frees up, and all
  finish with the same results.
* A request larger than the whole arena fails with TSYLV_ENOMEM; unknown
  tickets give TSYLV_EINVAL.
"""

import time

import numpy as np
import pytest

from oracle import kron
from paper_2405_09233_amd import tsylv, workloads
from gpu_util import dev, host, say, rel


def make_requests(count, seed0=100):
    rng = np.random.default_rng(seed0)
    reqs = []
    for i in range(count):
        n = int(rng.integers(6, 60))
        s = int(rng.integers(1, 9))
        p = int(rng.integers(1, 9))
        method = tsylv.GMRES if i % 3 else tsylv.FOM
        reqs.append((n, s, p, method, workloads.dense_shifted(n, s, p, seed=seed0 + i)))
    return reqs


def wait_all(ctx, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            st, info = ctx.poll(t)
            if st != 2:  # TSYLV_PENDING
                out[t] = (st, info)
        assert time.time() - t0 < timeout, "serving loop did not finish"
        time.sleep(0.002)
    return out


def run_served(ctx, reqs, opts_kw):
    tensors, tickets = [], []
    for (n, s, p, method, (A, B, C)) in reqs:
        Ad, Bd, Cd = dev(A), dev(B), dev(C)
        Xd = tsylv.empty_device((n, s, p), "cuda:0")
        tensors.append((Ad, Bd, Cd, Xd))
        tickets.append(ctx.submit(Ad, Bd, Cd, Xd, method=method, **opts_kw))
    res = wait_all(ctx, tickets)
    return [(res[t][0], res[t][1], host(tensors[i][3])) for i, t in enumerate(tickets)]


def run_alone(ctx, req, opts_kw):
    n, s, p, method, (A, B, C) = req
    fn = ctx.gmres if method == tsylv.GMRES else ctx.fom
    X, info = fn(dev(A), dev(B), dev(C), **opts_kw)
    return info, host(X)


@pytest.mark.gpu
def test_batch_results_bitwise_equal_alone():
    say("serve: 12 mixed requests")
    ctx = tsylv.Context(1 << 30, device=0)
    reqs = make_requests(12)
    kw = dict(m=8, tol=1e-11, max_cycles=400)
    served = run_served(ctx, reqs, kw)
    for req, (st, info, X) in zip(reqs, served):
        assert st == 0, info.as_dict()
        info1, X1 = run_alone(ctx, req, kw)
        assert np.array_equal(X, X1), "served result differs from the solo run"
        assert info.steps == info1.steps and info.cycles == info1.cycles
        n, s, p, method, (A, B, C) = req
        if n * s * p <= 900:
            assert rel(X, kron.kron_solve(A, B, C)) <= 1e-8
    ctx.close()


@pytest.mark.gpu
def test_refined_requests_in_the_mix():
    say("serve: refined FP32 requests")
    ctx = tsylv.Context(1 << 30, device=0)
    reqs = [r for r in make_requests(6, seed0=300) if r[3] == tsylv.GMRES]
    kw = dict(refine=1, prec=tsylv.FP32, inner_m=8, tol=1e-10, max_outer=400)
    served = run_served(ctx, reqs, kw)
    for req, (st, info, X) in zip(reqs, served):
        assert st == 0, info.as_dict()
        info1, X1 = run_alone(ctx, req, kw)
        assert np.array_equal(X, X1)
    ctx.close()


@pytest.mark.gpu
def test_admission_by_arena_budget():
    say("serve: small arena")
    n, s, p = 48, 6, 4
    o = tsylv.default_opts(tsylv.GMRES, m=10)
    need = tsylv.workspace_bytes(tsylv.GMRES, n, s, p, o)
    ctx = tsylv.Context(int(2.5 * need) + 4096, device=0)
    reqs = [(n, s, p, tsylv.GMRES, workloads.dense_shifted(n, s, p, seed=500 + i))
            for i in range(6)]
    kw = dict(m=10, tol=1e-11, max_cycles=400)
    served = run_served(ctx, reqs, kw)
    for req, (st, info, X) in zip(reqs, served):
        assert st == 0, info.as_dict()
        _, X1 = run_alone(ctx, req, kw)
        assert np.array_equal(X, X1)
    ctx.close()


@pytest.mark.gpu
def test_oversized_request_and_bad_ticket():
    say("serve: oversized request")
    ctx = tsylv.Context(1 << 20, device=0)
    A, B, C = workloads.dense_shifted(200, 16, 8, seed=1)
    Ad, Bd, Cd = dev(A), dev(B), dev(C)
    Xd = tsylv.empty_device(C.shape, "cuda:0")
    t = ctx.submit(Ad, Bd, Cd, Xd)
    res = wait_all(ctx, [t])
    assert res[t][0] == -2
    st, _ = ctx.poll(t + 1000)
    assert st == -1
    ctx.close()


@pytest.mark.gpu
def test_close_with_requests_in_flight():
    say("serve: close while busy")
    ctx = tsylv.Context(1 << 30, device=0)
    keep = []
    for i in range(10):
        A, B, C = workloads.dense_shifted(64, 8, 4, seed=700 + i)
        Ad, Bd, Cd = dev(A), dev(B), dev(C)
        Xd = tsylv.empty_device(C.shape, "cuda:0")
        keep.append((Ad, Bd, Cd, Xd))
        ctx.submit(Ad, Bd, Cd, Xd, m=10, tol=1e-12)
    t0 = time.time()
    ctx.close()          # finishes admitted solves, cancels the queued ones
    assert time.time() - t0 < 60


@pytest.mark.gpu
@pytest.mark.parametrize("method", [tsylv.GMRES, tsylv.GMRES_BATCHED])
def test_submit_waits_for_work_on_the_context_stream(method):
    """Inputs written by device kernels on the context stream right before
    tsylv_submit (behind a long chain of products, so they are still being
    written when the request is admitted) are read only after those
    kernels: the served result is bitwise the synchronous solve's."""
    import torch
    say("submit after context-stream work", method)
    A, B, C = workloads.dense_shifted(96, 8, 4, seed=17)
    ctx = tsylv.Context(1 << 30, device=0)  # on torch's current stream
    try:
        srcA, srcB, srcC = dev(A), dev(B), dev(C)
        Xref, info = ctx.gmres(srcA, srcB, srcC, m=30, tol=1e-10)
        assert info.status == 0
        Xref = host(Xref)
        Ad = tsylv.empty_device(A.shape, "cuda:0")
        Bd = tsylv.empty_device(B.shape, "cuda:0")
        Cd = tsylv.empty_device(C.shape, "cuda:0")
        for t in (Ad, Bd, Cd):
            t.fill_(float("nan"))
        Xd = tsylv.empty_device(C.shape, "cuda:0")
        torch.cuda.synchronize()
        busy = torch.full((4096, 4096), 1e-4, dtype=torch.float32, device="cuda:0")
        for _ in range(40):
            busy = busy @ busy
        Ad.copy_(srcA)
        Bd.copy_(srcB)
        Cd.copy_(srcC)
        t = ctx.submit(Ad, Bd, Cd, Xd, method=method, m=30, tol=1e-10)
        st, info = wait_all(ctx, [t])[t]
        assert st == 0, info.as_dict()
        if method == tsylv.GMRES:
            assert np.array_equal(host(Xd), Xref)
        else:
            assert rel(host(Xd), Xref) <= 1e-8
        del busy
    finally:
        ctx.close()
