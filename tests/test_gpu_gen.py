"""GPU tests of the on-device instance generator (tsylv_generate) and of
serving requests that carry only a seed.

* tsylv_generate against the host evaluation of the same counter-based
  definition (workloads.philox_instance): the Philox words are integers, so
  any slip in the counter map, the key or the Box-Muller pairing shows as an
  O(1) difference; what remains is the rounding of log, sin and cos
  (bar: 1e-13 absolute on values of size ~1).
* A request with A, B and C NULL draws its instance inside the setup
  transforms; the tube transform of a generated tube runs the same fma
  sequence as that of the stored tensor, so its result is bitwise the
  synchronous solve of the tsylv_generate output -- for tGMRES, tFOM, the
  BF16-refined solve and the t-Bartels-Stewart solve.
* On a small instance the served solution matches the oracle's Kronecker
  solve of the host-generated instance.
* Malformed requests (some of A, B, C NULL, p > 64 with generation) are
  rejected.
"""

import ctypes
import time

import numpy as np
import pytest

from oracle import kron
from paper_2405_09233_amd import tsylv, workloads
from gpu_util import ctx, dev, host, say, rel


def wait(c, t, timeout=120.0):
    t0 = time.time()
    while True:
        st, info = c.poll(t)
        if st != 2:
            return st, info
        assert time.time() - t0 < timeout, "serving loop did not finish"
        time.sleep(0.001)


@pytest.mark.gpu
@pytest.mark.parametrize("seed,n,s,p", [(0, 5, 5, 1), (3, 50, 7, 9), (12345, 33, 20, 64),
                                        (2**63 + 5, 130, 3, 67), (7, 1, 1, 3)])
def test_generate_matches_host_definition(seed, n, s, p):
    say("generate", seed, n, s, p)
    A, B, C = ctx().generate(seed, n, s, p)
    Ah, Bh, Ch = workloads.philox_instance(seed, n, s, p)
    for got, ref in ((A, Ah), (B, Bh), (C, Ch)):
        g = host(got)
        assert g.shape == ref.shape
        assert np.max(np.abs(g - ref)) <= 1e-13


@pytest.mark.gpu
@pytest.mark.parametrize("method,refined,n,s,p", [
    (tsylv.GMRES, False, 100, 12, 7), (tsylv.FOM, False, 64, 16, 64), (tsylv.GMRES, False, 40, 6, 1),
    (tsylv.GMRES, True, 300, 24, 9), (tsylv.TBS, False, 20, 9, 6)])
def test_generated_request_equals_synchronous(method, refined, n, s, p):
    import torch
    say("generated request", method, refined, n, s, p)
    c = ctx()
    seed = 1000 + n + s + p
    if refined:
        o = tsylv.default_opts(method, refine=1, prec=tsylv.BF16, inner_m=16, tol=1e-10)
    else:
        o = tsylv.default_opts(method, m=20, tol=1e-10)
    A, B, C = c.generate(seed, n, s, p)
    Xs = torch.zeros_like(C)
    if method == tsylv.TBS:
        Xs, info_s = c.tbs(A, B, C, Xs, opts=o)
    elif method == tsylv.FOM:
        Xs, info_s = c.fom(A, B, C, Xs, opts=o)
    else:
        Xs, info_s = c.gmres(A, B, C, Xs, opts=o)
    assert info_s.status == 0, info_s.as_dict()
    Xg = torch.zeros_like(C)
    st, info = wait(c, c.submit(None, None, None, Xg, method=method, opts=o, seed=seed))
    assert st == 0, info.as_dict()
    assert info.relres_true == info_s.relres_true
    assert torch.equal(Xg, Xs)


@pytest.mark.gpu
def test_generated_request_matches_oracle():
    import torch
    say("generated request vs oracle")
    c = ctx()
    n, s, p, seed = 12, 4, 5, 77
    X = tsylv.empty_device((n, s, p), "cuda:0")
    X.zero_()
    o = tsylv.default_opts(tsylv.GMRES, m=60, tol=1e-12)
    st, info = wait(c, c.submit(None, None, None, X, opts=o, seed=seed))
    assert st == 0, info.as_dict()
    A, B, C = workloads.philox_instance(seed, n, s, p)
    assert rel(host(X), kron.kron_solve(A, B, C)) <= 1e-9
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_malformed_generated_requests_are_rejected():
    c = ctx()
    lib = tsylv.load()
    A, B, C = c.generate(1, 8, 3, 2)
    X = tsylv.empty_device((8, 3, 2), "cuda:0")
    req = tsylv.Request()
    req.method = tsylv.GMRES
    req.n, req.s, req.p = 8, 3, 2
    req.A, req.B, req.C = A.data_ptr(), None, C.data_ptr()
    req.X = X.data_ptr()
    req.opts = tsylv.default_opts(tsylv.GMRES)
    ticket = ctypes.c_uint64()
    assert lib.tsylv_submit(c.handle, ctypes.byref(req), ctypes.byref(ticket)) == -1
    X65 = tsylv.empty_device((8, 3, 65), "cuda:0")
    with pytest.raises(tsylv.TsylvError):
        c.submit(None, None, None, X65, seed=3)
    with pytest.raises(ValueError):
        c.submit(None, None, None, X)  # no seed
