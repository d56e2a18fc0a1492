"""GPU test of the allocation-free apply (tsylv_apply_noalloc): called
through the C ABI twice in a row on one stream, the second call with a
smaller input, each result equals tsylv_apply's on the same operands (the
same kernels with the default tiles: bit for bit), in every precision; the
static scratch is shared by the calls, so the second call also shows that
nothing of the first call's contents leaks into it.  Sizes beyond the
scratch are rejected with TSYLV_ESCRATCH before anything is enqueued."""

import numpy as np
import pytest

from paper_2405_09233_amd import tsylv
from gpu_util import dev, host, say


def _operands(n, s, p, seed):
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((n, n, p)))
    B = np.asfortranarray(rng.standard_normal((s, s, p)))
    X = np.asfortranarray(rng.standard_normal((n, s, p)))
    return A, B, X


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [tsylv.FP64, tsylv.FP32, tsylv.BF16])
def test_noalloc_apply_matches_tsylv_apply(prec):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = tsylv.Context(2 << 30, device=0)
    try:
        for n, s, p in [(300, 70, 9), (57, 13, 4)]:  # second call smaller
            say("noalloc apply", prec, n, s, p)
            A, B, X = _operands(n, s, p, seed=n + s + p + prec)
            Ad, Bd, Xd = dev(A), dev(B), dev(X)
            ref = host(ctx.apply(Ad, Bd, Xd, prec=prec))
            Y = tsylv.apply_noalloc(Ad, Bd, Xd, prec=prec)
            torch.cuda.synchronize()
            got = host(Y)
            assert np.array_equal(got, ref), np.abs(got - ref).max()
    finally:
        ctx.close()


@pytest.mark.gpu
def test_noalloc_apply_rejects_sizes_beyond_the_scratch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cap = tsylv.noalloc_scratch_bytes()
    assert cap == 256 << 20
    n, s, p = 2048, 8, 16  # Fourier planes of A alone: 512 MiB
    assert tsylv.workspace_bytes(tsylv.APPLY, n, s, p) > cap
    A = tsylv.empty_device((n, n, p), "cuda:0")
    B = tsylv.empty_device((s, s, p), "cuda:0")
    X = tsylv.empty_device((n, s, p), "cuda:0")
    with pytest.raises(tsylv.TsylvError) as e:
        tsylv.apply_noalloc(A, B, X)
    assert e.value.status == -7
