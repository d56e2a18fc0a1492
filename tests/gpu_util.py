"""Helpers shared by the GPU tests (context creation, transfers)."""

import sys

import numpy as np
import pytest

from paper_2405_09233_amd import tsylv

_CTX = {}


def ctx(arena_gb=24):
    """One library context per process, on cuda:0 with a torch-owned arena."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    key = arena_gb
    if key not in _CTX:
        _CTX[key] = tsylv.Context(int(arena_gb * (1 << 30)), device=0)
    return _CTX[key]


def dev(a):
    return tsylv.to_device(a, "cuda:0")


def host(t):
    return tsylv.to_host(t)


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


_WORKLOADS = {}


def workload(name):
    """A named full-size workload of paper_2405_09233_amd.workloads
    (``cd_4096``: n = 4096, s = 64, p = 32; ``cd_8192``: n = 8192, s = 128,
    p = 64, 34 GB of FP64 A), generated once per test process on the host."""
    if name not in _WORKLOADS:
        from paper_2405_09233_amd import workloads
        say("generating workload", name)
        _WORKLOADS[name] = getattr(workloads, name)(seed=0)
    return _WORKLOADS[name]
