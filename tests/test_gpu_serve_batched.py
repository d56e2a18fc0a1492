"""GPU tests of serving in lockstep batches (requests of method
TSYLV_METHOD_GMRES_BATCHED through tsylv_submit / tsylv_poll).

* Requests that wait together are solved as one batch; every result must
  be bitwise the batch-of-one solve of its instance (tsylv_gmres_batch with
  that instance alone), with plain tGMRES requests interleaved in the queue
  (they split the batches), and the small ones match the oracle's Kronecker
  solution.
* Seed-only requests draw their instance on the device inside the batch.
* Admission by the arena: with an arena that holds a few instances at a
  time the queue drains in several batches with the same results.
* Malformed requests are rejected; closing the context with batches in
  flight finishes them.
* Plain tGMRES requests small enough for the single-workgroup solve join
  the batches, with the synchronous solve's bits.
* Batched requests above the size that tsylv_gmres_batch runs in lockstep
  (n s p > 2^18) are still served in lockstep batches (several batches in
  flight at once share nothing): every result converges, its true residual
  recomputed by tsylv_apply.
"""

import time

import numpy as np
import pytest

from oracle import kron
from paper_2405_09233_amd import tsylv, workloads
from gpu_util import dev, host, say, rel


def wait_all(ctx, tickets, timeout=120.0):
    out, t0 = {}, time.time()
    pending = list(tickets)
    while pending:
        for t in list(pending):
            st, info = ctx.poll(t)
            if st != 2:
                out[t] = (st, info)
                pending.remove(t)
        assert time.time() - t0 < timeout, "serving loop did not finish"
        time.sleep(0.001)
    return out


def make(count, seed0):
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(count):
        n, s, p = int(rng.integers(6, 80)), int(rng.integers(1, 13)), int(rng.integers(1, 10))
        out.append((n, s, p, workloads.dense_shifted(n, s, p, seed=seed0 + i)))
    return out


def submit_all(ctx, reqs, opts, plain_every=0):
    """Submits every instance as a GMRES_BATCHED request (and, with
    plain_every, every plain_every-th one also as a plain tGMRES request).
    Returns the batched requests' device tensors, their tickets, and the
    plain requests' tickets with their tensors (kept referenced)."""
    import torch
    batched, tickets, plain = [], [], []
    for i, (n, s, p, (A, B, C)) in enumerate(reqs):
        Ad, Bd, Cd = dev(A), dev(B), dev(C)
        X = torch.zeros_like(Cd)
        batched.append((Ad, Bd, Cd, X))
        tickets.append(ctx.submit(Ad, Bd, Cd, X, method=tsylv.GMRES_BATCHED, opts=opts))
        if plain_every and i % plain_every == 0:
            Xp = torch.zeros_like(Cd)
            plain.append((ctx.submit(Ad, Bd, Cd, Xp, method=tsylv.GMRES, m=20, tol=1e-10),
                          (Ad, Bd, Cd, Xp)))
    return batched, tickets, plain


@pytest.mark.gpu
def test_batched_requests_equal_batch_of_one():
    import torch
    say("serve batched: 24 requests with plain ones interleaved")
    c = tsylv.Context(4 << 30, device=0)
    try:
        reqs = make(24, 900)
        opts = tsylv.default_opts(tsylv.GMRES, m=30, tol=1e-11, max_cycles=100)
        batched, tickets, plain = submit_all(c, reqs, opts, plain_every=5)
        res = wait_all(c, tickets + [t for t, _ in plain])
        assert all(res[t][0] == 0 for t, _ in plain)
        for i, t in enumerate(tickets):
            st, info = res[t]
            assert st == 0, info.as_dict()
            Ad, Bd, Cd, X = batched[i]
            X1 = torch.zeros_like(Cd)
            i1 = c.gmres_batch([(Ad, Bd, Cd, X1)], opts=opts)[0]
            assert torch.equal(X, X1), i
            assert (info.steps, info.cycles, info.relres_true) == (i1.steps, i1.cycles,
                                                                   i1.relres_true)
        for i in range(3):
            n, s, p, (A, B, C) = reqs[i]
            assert rel(host(batched[i][3]), kron.kron_solve(A, B, C)) <= 1e-8
    finally:
        c.close()


@pytest.mark.gpu
def test_batched_seed_only_requests():
    import torch
    say("serve batched: seed-only requests")
    c = tsylv.Context(2 << 30, device=0)
    try:
        opts = tsylv.default_opts(tsylv.GMRES, m=30, tol=1e-10)
        shapes = [(40, 6, 5), (64, 12, 8), (25, 3, 2), (90, 16, 4)]
        Xs = [tsylv.empty_device(sh, "cuda:0").zero_() for sh in shapes]
        tickets = [c.submit(None, None, None, X, method=tsylv.GMRES_BATCHED, opts=opts,
                            seed=50 + k) for k, X in enumerate(Xs)]
        res = wait_all(c, tickets)
        for k, (sh, X, t) in enumerate(zip(shapes, Xs, tickets)):
            assert res[t][0] == 0, res[t][1].as_dict()
            A, B, C = c.generate(50 + k, *sh)
            X1 = torch.zeros_like(C)
            c.gmres_batch([(A, B, C, X1)], opts=opts)
            assert torch.equal(X, X1), k
    finally:
        c.close()


@pytest.mark.gpu
def test_large_batched_requests_served_in_lockstep():
    import torch
    say("serve batched: 12 seed-only requests of n s p = 327680")
    shape = (512, 32, 20)
    c = tsylv.Context(24 << 30, device=0)
    try:
        opts = tsylv.default_opts(tsylv.GMRES, m=30, tol=1e-9, max_cycles=200)
        Xs = [tsylv.empty_device(shape, "cuda:0").zero_() for _ in range(12)]
        tickets = [c.submit(None, None, None, X, method=tsylv.GMRES_BATCHED, opts=opts,
                            seed=700 + k) for k, X in enumerate(Xs)]
        res = wait_all(c, tickets, timeout=300.0)
        for k, (X, t) in enumerate(zip(Xs, tickets)):
            st, info = res[t]
            assert st == 0 and info.relres_true <= 1e-9, (k, info.as_dict())
            if k % 4 == 0:
                A, B, C = c.generate(700 + k, *shape)
                R = C - c.apply(A, B, X)
                r = (torch.linalg.norm(R) / torch.linalg.norm(C)).item()
                assert r <= 1.05e-9, (k, r)
    finally:
        c.close()


@pytest.mark.gpu
def test_batched_admission_by_arena_budget():
    import torch
    say("serve batched: small arena")
    reqs = make(12, 950)
    opts = tsylv.default_opts(tsylv.GMRES, m=20, tol=1e-10)
    probs = [(dev(A), dev(B), dev(C)) for _, _, _, (A, B, C) in reqs]
    one = max(tsylv.Context.batch_workspace_bytes(
        [(a, b, cc, torch.zeros_like(cc))], opts=opts) for a, b, cc in probs)
    c = tsylv.Context(3 * one + (1 << 20), device=0)
    try:
        Xs = [torch.zeros_like(cc) for _, _, cc in probs]
        tickets = [c.submit(a, b, cc, X, method=tsylv.GMRES_BATCHED, opts=opts)
                   for (a, b, cc), X in zip(probs, Xs)]
        res = wait_all(c, tickets)
        ref = tsylv.Context(1 << 30, device=0)
        try:
            for (a, b, cc), X, t in zip(probs, Xs, tickets):
                assert res[t][0] == 0, res[t][1].as_dict()
                X1 = torch.zeros_like(cc)
                ref.gmres_batch([(a, b, cc, X1)], opts=opts)
                assert torch.equal(X, X1)
        finally:
            ref.close()
    finally:
        c.close()


@pytest.mark.gpu
def test_batched_malformed_and_close_in_flight():
    import torch
    c = tsylv.Context(1 << 30, device=0)
    A, B, C = workloads.dense_shifted(10, 3, 4, seed=3)
    Ad, Bd, Cd = dev(A), dev(B), dev(C)
    X = torch.zeros_like(Cd)
    with pytest.raises(tsylv.TsylvError):
        c.submit(Ad, Bd, Cd, X, method=tsylv.GMRES_BATCHED, m=64)
    with pytest.raises(tsylv.TsylvError):
        c.submit(Ad, Bd, Cd, X, method=tsylv.GMRES_BATCHED, refine=1, prec=tsylv.FP32)
    o = tsylv.default_opts(tsylv.GMRES, x0_given=1)
    with pytest.raises(tsylv.TsylvError):
        c.submit(Ad, Bd, Cd, X, method=tsylv.GMRES_BATCHED, opts=o)
    keep = []
    for i in range(30):
        A, B, C = workloads.dense_shifted(48, 8, 4, seed=960 + i)
        t = (dev(A), dev(B), dev(C))
        Xi = torch.zeros_like(t[2])
        keep.append(t + (Xi,))
        c.submit(*t, Xi, method=tsylv.GMRES_BATCHED, m=10, tol=1e-12)
    t0 = time.time()
    c.close()  # finishes admitted batches, cancels the queued requests
    assert time.time() - t0 < 60


@pytest.mark.gpu
def test_served_batches_replay_recorded_graphs_while_the_caller_works(monkeypatch):
    """Served lockstep batches replay their step from a recorded HIP graph
    while the calling thread keeps the legacy default stream busy with its
    own kernels and synchronisations (the case that a stream capture on the
    worker could not survive): every result is bitwise the same as with the
    steps launched eagerly (TSYLV_BATCH_GRAPH=0), over several batches."""
    import torch
    say("serve batched: graph vs eager with caller work on the default stream")
    reqs = make(16, 1300)
    opts = tsylv.default_opts(tsylv.GMRES, m=30, tol=1e-11, max_cycles=100)
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("TSYLV_BATCH_GRAPH", mode)
        c = tsylv.Context(2 << 30, device=0)
        try:
            batched, tickets, _ = submit_all(c, reqs, opts)
            busy = torch.full((2048, 2048), 1e-4, dtype=torch.float32, device="cuda:0")
            pending = set(tickets)
            res = {}
            t0 = time.time()
            while pending:
                busy = busy @ busy  # the caller's own work on its stream
                torch.cuda.synchronize()
                for t in list(pending):
                    st, info = c.poll(t)
                    if st != 2:
                        res[t] = (st, info)
                        pending.discard(t)
                assert time.time() - t0 < 120, "serving loop did not finish"
            for t in tickets:
                assert res[t][0] == 0, res[t][1].as_dict()
            out[mode] = [host(b[3]) for b in batched]
        finally:
            c.close()
    for a, b in zip(out["1"], out["0"]):
        assert np.array_equal(a, b)
    n, s, p, (A, B, C) = reqs[0]
    assert rel(out["1"][0], kron.kron_solve(A, B, C)) <= 1e-8


@pytest.mark.gpu
def test_small_gmres_requests_join_batches():
    """Plain tGMRES requests small enough for the single-workgroup solve
    join the served batches (with GMRES_BATCHED requests of equal options,
    and with an initial guess): each result is bitwise the synchronous
    tsylv_gmres solve of its instance, with the same steps, cycles and
    residuals; larger tGMRES requests in the same queue run as single solves
    with the same guarantee.  Requests of one batch report the batch's wall
    time, so equal `seconds` show that batches formed."""
    import torch
    say("serve: small tGMRES requests in batches")
    c = tsylv.Context(2 << 30, device=0)
    try:
        rng = np.random.default_rng(1700)
        plain = tsylv.default_opts(tsylv.GMRES, m=30, tol=1e-11, max_cycles=100)
        guess = tsylv.default_opts(tsylv.GMRES, m=30, tol=1e-11, max_cycles=100, x0_given=1)
        items = []
        for i in range(56):
            if i in (13, 33, 50):
                n, s, p = 200, 12, 6  # n s p = 14400: beyond the one-workgroup solve
            else:
                n, s, p = (int(rng.integers(4, 25)), int(rng.integers(2, 9)),
                           int(rng.integers(2, 9)))
            A, B, C = workloads.dense_shifted(n, s, p, seed=1700 + i)
            Ad, Bd, Cd = dev(A), dev(B), dev(C)
            # runs of each kind (a batch is a run of requests with equal
            # options at the head of the queue)
            kind = "plain" if i < 24 else ("batched" if i < 40 else "guess")
            X0 = torch.zeros_like(Cd)  # the library layout (Cd's strides)
            if kind == "guess":
                X0.copy_(0.1 * torch.randn(Cd.shape, dtype=torch.float64, device="cuda:0"))
            X = torch.empty_like(X0)
            X.copy_(X0)
            items.append((kind, Ad, Bd, Cd, X0, X))
        torch.cuda.synchronize()
        tickets = []
        for kind, Ad, Bd, Cd, X0, X in items:
            method = tsylv.GMRES_BATCHED if kind == "batched" else tsylv.GMRES
            tickets.append(c.submit(Ad, Bd, Cd, X, method=method,
                                    opts=guess if kind == "guess" else plain))
        res = wait_all(c, tickets)
        secs = {}
        for (kind, Ad, Bd, Cd, X0, X), t in zip(items, tickets):
            st, info = res[t]
            assert st == 0, (kind, info.as_dict())
            if kind == "batched":
                X1 = torch.zeros_like(Cd)
                i1 = c.gmres_batch([(Ad, Bd, Cd, X1)], opts=plain)[0]
            else:
                X1 = X0.clone()
                _, i1 = c.gmres(Ad, Bd, Cd, X=X1, opts=guess if kind == "guess" else plain)
            assert torch.equal(X, X1), (kind, tuple(Cd.shape))
            assert (info.steps, info.cycles, info.relres_true) == (i1.steps, i1.cycles,
                                                                   i1.relres_true)
            if kind != "batched" and Cd.numel() <= 8192:
                secs[info.seconds] = secs.get(info.seconds, 0) + 1
        assert max(secs.values()) >= 2, secs
    finally:
        c.close()
