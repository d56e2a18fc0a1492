"""GPU tests of the batched lockstep tGMRES (tsylv_gmres_batch).

* Parity: a batch of small instances that covers every tile variant of the
  batched apply (s <= 16, 17..32, > 32), p = 1, odd and even p, solved to
  1e-12 and compared with the oracle's Kronecker solutions (bar 1e-9).
* Batch independence: an instance's X and record are bitwise the same
  alone and inside a batch, and with the step replayed from a HIP graph or
  launched eagerly (many replays per solve, host synchronisations between
  blocks of them).
* Against the single-instance tsylv_gmres on shapes of the batched
  workload (n a multiple of 32 in [256, 2048], s in [16, 128], p in
  {8, 16, 32}) with restarts: both to 1e-11, solutions within 1e-8.
* Per-instance stopping: instances that cannot converge in the cycles given
  report TSYLV_NOT_CONVERGED while the others converge; X0 is honoured.
* The executor by instance: small FP64 instances take the lockstep
  kernels, large ones and every refined solve (FP32 / BF16 inner cycles)
  the stream executor; a large instance's result is bitwise the synchronous
  tsylv_gmres solve, a refined batch's results are bitwise the refined
  single solves and match the oracle.
* Malformed batches are rejected.

Instances small enough for the single-workgroup executor are sent to the
lockstep kernels here (TSYLV_KRYLOV_TINY=0 for every test of this module):
that executor has its own tests (test_gpu_tiny.py).
"""

import os

import numpy as np
import pytest

from oracle import kron
from paper_2405_09233_amd import tsylv, workloads
from gpu_util import ctx, dev, host, say, rel

SMALL = [(12, 5, 4), (20, 18, 3), (9, 40, 2), (30, 6, 1), (16, 10, 5), (25, 3, 7)]


@pytest.fixture(autouse=True)
def _lockstep_and_stream_executors(monkeypatch):
    monkeypatch.setenv("TSYLV_KRYLOV_TINY", "0")


def _batch(shapes, seed0):
    import torch
    data, items = [], []
    for k, (n, s, p) in enumerate(shapes):
        A, B, C = workloads.dense_shifted(n, s, p, seed=seed0 + k)
        Ad, Bd, Cd = dev(A), dev(B), dev(C)
        X = torch.zeros_like(Cd)
        data.append((A, B, C))
        items.append((Ad, Bd, Cd, X))
    return data, items


@pytest.mark.gpu
def test_batch_matches_kronecker():
    say("batch vs kronecker", SMALL)
    data, items = _batch(SMALL, 300)
    infos = ctx().gmres_batch(items, m=30, tol=1e-12, max_cycles=50)
    for (A, B, C), (_, _, _, X), info in zip(data, items, infos):
        assert info.status == 0, info.as_dict()
        assert info.relres_true <= 1e-12
        assert rel(host(X), kron.kron_solve(A, B, C)) <= 1e-9


@pytest.mark.gpu
def test_alone_equals_in_batch_and_graph_equals_eager():
    import torch
    say("batch determinism")
    shapes = [(40, 12, 6), (64, 30, 4), (33, 50, 3), (50, 7, 1)]
    c = ctx()
    _, items = _batch(shapes, 400)
    infos = c.gmres_batch(items, m=8, tol=1e-11, max_cycles=100)  # several cycles
    assert all(i.status == 0 for i in infos)
    assert max(i.cycles for i in infos) > 1
    for k in range(len(shapes)):
        Ad, Bd, Cd, X = items[k]
        Xa = torch.zeros_like(Cd)
        ia = c.gmres_batch([(Ad, Bd, Cd, Xa)], m=8, tol=1e-11, max_cycles=100)[0]
        assert torch.equal(Xa, X), k
        assert (ia.steps, ia.cycles, ia.relres_true) == (infos[k].steps, infos[k].cycles,
                                                         infos[k].relres_true)
    os.environ["TSYLV_BATCH_GRAPH"] = "0"
    try:
        Xe = [torch.zeros_like(it[2]) for it in items]
        ie = c.gmres_batch([(a, b, cc, x) for (a, b, cc, _), x in zip(items, Xe)], m=8,
                           tol=1e-11, max_cycles=100)
    finally:
        del os.environ["TSYLV_BATCH_GRAPH"]
    for k in range(len(shapes)):
        assert torch.equal(Xe[k], items[k][3]), k
        assert ie[k].steps == infos[k].steps


@pytest.mark.gpu
def test_batched_workload_shapes_match_single_solves():
    import torch
    shapes = [(256, 16, 16), (512, 96, 8), (1024, 40, 8), (320, 128, 32)]
    say("batch vs single", shapes)
    c = ctx()
    _, items = _batch(shapes, 500)
    infos = c.gmres_batch(items, m=20, tol=1e-11, max_cycles=200)
    for (Ad, Bd, Cd, X), info in zip(items, infos):
        assert info.status == 0, info.as_dict()
        assert info.relres_true <= 1e-11
        Xs, i1 = c.gmres(Ad, Bd, Cd, m=20, tol=1e-11, max_cycles=200)
        assert i1.status == 0
        assert rel(host(X), host(Xs)) <= 1e-8
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_per_instance_stopping_and_x0():
    import torch
    say("batch stopping")
    c = ctx()
    _, items = _batch([(30, 6, 3), (40, 20, 5)], 600)
    infos = c.gmres_batch(items, m=2, tol=1e-12, max_cycles=1, raise_on_error=False)
    assert all(i.status == 1 for i in infos)  # TSYLV_NOT_CONVERGED
    assert all(i.cycles == 1 and i.steps == 2 for i in infos)
    # continue from the iterates: X0 given
    o = tsylv.default_opts(tsylv.GMRES, m=30, tol=1e-12, max_cycles=50)
    o.x0_given = 1
    infos2 = c.gmres_batch(items, opts=o)
    assert all(i.status == 0 for i in infos2)
    ref = [c.gmres(a, b, cc, m=30, tol=1e-12)[0] for a, b, cc, _ in items]
    for (_, _, _, X), Xr in zip(items, ref):
        assert rel(host(X), host(Xr)) <= 1e-9
    # one instance that converges at once (C = 0) next to one that does not
    A, B, C = workloads.dense_shifted(10, 4, 2, seed=7)
    Z = torch.zeros_like(dev(C))
    X0 = torch.zeros_like(Z)
    infos3 = c.gmres_batch([(dev(A), dev(B), Z, X0)] + [items[1]], m=30, tol=1e-12)
    assert infos3[0].status == 0 and infos3[0].steps == 0
    assert torch.count_nonzero(X0) == 0


@pytest.mark.gpu
def test_malformed_batches_are_rejected():
    c = ctx()
    _, items = _batch([(8, 3, 2)], 700)
    with pytest.raises(tsylv.TsylvError):
        c.gmres_batch(items, m=64)
    with pytest.raises(tsylv.TsylvError):
        c.gmres_batch([])


@pytest.mark.gpu
def test_mixed_batch_executors_by_instance():
    """FP64 batch with small instances (lockstep) and large ones (n s p >
    2^18: the stream executor): the large ones are bitwise the synchronous
    tsylv_gmres solves, the small ones bitwise their batch-of-one solves."""
    import torch
    shapes = [(512, 96, 8), (30, 6, 3), (1024, 40, 8), (40, 20, 5)]
    say("batch executors", shapes)
    c = ctx()
    _, items = _batch(shapes, 800)
    infos = c.gmres_batch(items, m=20, tol=1e-11, max_cycles=200)
    for k, ((Ad, Bd, Cd, X), info) in enumerate(zip(items, infos)):
        assert info.status == 0, info.as_dict()
        n, s, p = shapes[k]
        if n * s * p > (1 << 18):
            Xs, i1 = c.gmres(Ad, Bd, Cd, m=20, tol=1e-11, max_cycles=200)
            assert torch.equal(Xs, X), k
            assert i1.steps == info.steps
        else:
            X1 = torch.zeros_like(Cd)
            c.gmres_batch([(Ad, Bd, Cd, X1)], m=20, tol=1e-11, max_cycles=200)
            assert torch.equal(X1, X), k


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [tsylv.FP32, tsylv.BF16])
def test_refined_batch(prec):
    """Refined batches (FP64 refinement around inner tGMRES cycles in FP32
    or BF16): every instance bitwise its refined single solve, within 1e-7
    of the oracle's Kronecker solution for the small ones, relres 1e-10."""
    import torch
    shapes = [(30, 6, 3), (12, 5, 4), (256, 48, 8), (9, 40, 2)]
    say("refined batch", prec, shapes)
    data, items = _batch(shapes, 900)
    c = ctx()
    o = tsylv.default_opts(tsylv.GMRES, m=30, refine=1, prec=prec, inner_m=20, inner_tol=1e-4,
                           tol=1e-10, max_outer=300)
    infos = c.gmres_batch(items, opts=o)
    for k, ((A, B, C), (Ad, Bd, Cd, X), info) in enumerate(zip(data, items, infos)):
        assert info.status == 0, (k, info.as_dict())
        assert info.relres_true <= 1e-10 and info.outer >= 1
        Xs, _ = c.gmres(Ad, Bd, Cd, opts=o)
        assert torch.equal(Xs, X), k
        if A.shape[0] * B.shape[0] * A.shape[2] <= 900:
            assert rel(host(X), kron.kron_solve(A, B, C)) <= 1e-7
