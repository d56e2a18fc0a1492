"""CPU checks of the C-ABI library: it loads, exports every function that
include/tsylv.h declares, and the ctypes structures of the binding have the
sizes and field offsets the C compiler gives the header's structs.  No
compute call is made (there is no GPU here)."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2405_09233_amd import tsylv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsylv.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsylv_[a-z_]+)\s*\(", src)))


def test_library_exports_header_functions():
    lib = tsylv.load()
    names = header_functions()
    assert "tsylv_gmres" in names and "tsylv_poll" in names
    for name in names:
        assert hasattr(lib, name), name
    assert names == tsylv.EXPORTED


def test_struct_layout_matches_header(tmp_path):
    c = r'''
#include <stdio.h>
#include <stddef.h>
#include "tsylv.h"
#define F(T, f) printf("%s.%s %zu\n", #T, #f, offsetof(T, f));
int main(void) {
  printf("tsylv_opts %zu\n", sizeof(tsylv_opts));
  printf("tsylv_info %zu\n", sizeof(tsylv_info));
  printf("tsylv_request %zu\n", sizeof(tsylv_request));
  printf("tsylv_problem %zu\n", sizeof(tsylv_problem));
  F(tsylv_opts, tol) F(tsylv_opts, inner_tol) F(tsylv_opts, res_hist) F(tsylv_opts, res_hist_cap)
  F(tsylv_info, relres_true) F(tsylv_info, seconds) F(tsylv_info, fom_fallback)
  F(tsylv_request, n) F(tsylv_request, A) F(tsylv_request, X) F(tsylv_request, opts)
  F(tsylv_request, gen_seed) F(tsylv_problem, p) F(tsylv_problem, A) F(tsylv_problem, X)
  return 0;
}
'''
    cf = tmp_path / "layout.c"
    cf.write_text(c)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(cf), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    got = {k: int(v) for k, v in got.items()}
    assert got["tsylv_opts"] == ctypes.sizeof(tsylv.Opts)
    assert got["tsylv_info"] == ctypes.sizeof(tsylv.Info)
    assert got["tsylv_request"] == ctypes.sizeof(tsylv.Request)
    assert got["tsylv_problem"] == ctypes.sizeof(tsylv.Problem)
    for key, val in got.items():
        if "." in key:
            sname, field = key.split(".")
            cls = {"tsylv_opts": tsylv.Opts, "tsylv_info": tsylv.Info,
                   "tsylv_request": tsylv.Request, "tsylv_problem": tsylv.Problem}[sname]
            assert getattr(cls, field).offset == val, key


def test_default_opts_and_workspace_query():
    o = tsylv.default_opts(tsylv.GMRES)
    assert (o.m, o.max_cycles, o.tol, o.prec) == (30, 500, 1e-8, tsylv.FP64)
    assert tsylv.default_opts(tsylv.TBA).m == 10
    n, s, p = 4096, 64, 32
    b = tsylv.workspace_bytes(tsylv.GMRES, n, s, p, o)
    assert b >= 8 * (p * n * n + (o.m + 3) * n * s * p)
    assert tsylv.workspace_bytes(tsylv.GMRES, 0, s, p, o) == 0
    assert tsylv.workspace_bytes(tsylv.APPLY, 8, 6, 4, None) > 0


def test_batch_workspace_query(monkeypatch):
    """The batch plan's byte count without a device: each lockstep
    instance's Fourier setup and basis plus the shared tables; an instance
    small enough for the single-workgroup executor (run after the lockstep
    batch, in a workspace of its own) needs its setup and basis; malformed
    batches give 0."""
    probs = (tsylv.Problem * 2)()
    shapes = [(100, 8, 5), (40, 3, 2)]
    for k, (n, s, p) in enumerate(shapes):
        probs[k].n, probs[k].s, probs[k].p = n, s, p
        probs[k].A = probs[k].B = probs[k].C = probs[k].X = 4096  # never dereferenced
    o = tsylv.default_opts(tsylv.GMRES, m=20)
    lib = tsylv.load()
    floors = [8 * (p * n * n + p * s * s + 3 * p * p + (o.m + 4) * n * s * p)
              for n, s, p in shapes]
    b = lib.tsylv_batch_workspace_bytes(2, probs, ctypes.byref(o))
    assert b >= max(floors)
    monkeypatch.setenv("TSYLV_KRYLOV_TINY", "0")  # both instances in lockstep
    b = lib.tsylv_batch_workspace_bytes(2, probs, ctypes.byref(o))
    assert b >= sum(floors)
    monkeypatch.delenv("TSYLV_KRYLOV_TINY")
    assert lib.tsylv_batch_workspace_bytes(0, probs, ctypes.byref(o)) == 0
    o.m = 64  # beyond the batch's restart limit
    assert lib.tsylv_batch_workspace_bytes(2, probs, ctypes.byref(o)) == 0
    # refined batches run as concurrent single solves: their workspaces
    o = tsylv.default_opts(tsylv.GMRES, refine=1, prec=tsylv.FP32)
    single = [tsylv.workspace_bytes(tsylv.GMRES, n, s, p, o) for n, s, p in [(100, 8, 5), (40, 3, 2)]]
    assert lib.tsylv_batch_workspace_bytes(2, probs, ctypes.byref(o)) == sum(single)


def test_strerror():
    lib = tsylv.load()
    assert lib.tsylv_strerror(0) == b"ok"
    assert b"invalid" in lib.tsylv_strerror(-1)


def test_invalid_arguments_rejected_without_gpu():
    lib = tsylv.load()
    assert lib.tsylv_destroy(None) == -1
    assert lib.tsylv_gmres(None, 4, 2, 2, None, None, None, None, None, None) == -1
    h = ctypes.c_void_p()
    assert lib.tsylv_create(ctypes.byref(h), 0, None, None, 0) == -1


def test_tbs_workspace_bounds(monkeypatch):
    """tsylv_workspace_bytes of the direct solve: its own up to n, s = 64,
    past it that of the tGMRES(30) that stands in for it; the batched form
    likewise (the larger of its direct and tGMRES parts), 0 for a malformed
    instance.  Host-only, no GPU call."""
    assert tsylv.workspace_bytes(tsylv.TBS, 8, 6, 4) > 0
    assert tsylv.workspace_bytes(tsylv.TBS, 64, 64, 33) > 0
    g = tsylv.default_opts(tsylv.GMRES)
    for n, s in ((65, 6), (8, 65), (300, 80)):
        assert tsylv.workspace_bytes(tsylv.TBS, n, s, 4) == tsylv.workspace_bytes(
            tsylv.GMRES, n, s, 4, g)
    small = tsylv.workspace_bytes(tsylv.TBS, 8, 6, 4)
    assert tsylv.workspace_bytes(tsylv.TBS, 8, 6, 8) > small
    lib = tsylv.load()
    probs = (tsylv.Problem * 3)()
    for k, (n, s, p) in enumerate([(8, 6, 4), (65, 6, 4), (30, 3, 2)]):
        probs[k].n, probs[k].s, probs[k].p = n, s, p
        probs[k].A = probs[k].B = probs[k].C = probs[k].X = 4096  # never dereferenced
    direct = lib.tsylv_tbs_batch_workspace_bytes(1, probs)
    assert direct > 0
    monkeypatch.setenv("TSYLV_KRYLOV_TINY", "0")  # the tGMRES part in lockstep
    mixed = lib.tsylv_tbs_batch_workspace_bytes(3, probs)
    both = (tsylv.Problem * 1)(probs[1])
    krylov = lib.tsylv_batch_workspace_bytes(1, both, ctypes.byref(g))
    assert mixed >= max(direct, krylov) and krylov > 0
    probs[2].n = 0
    assert lib.tsylv_tbs_batch_workspace_bytes(3, probs) == 0


def test_default_apply_variant_is_host_logic():
    """The tile variant an untuned apply takes (host logic, no GPU): capped
    64 x 16 tiles for FP64 at small s from n = 2048 on, the 32-deep
    uncapped ones below, capped 64 x 32 up to s = 64, 64 x 64 beyond; bad
    precisions and sizes are rejected."""
    v = tsylv.apply_default_variant
    assert v(tsylv.FP64, 4096, 16) == 15 and v(tsylv.FP64, 1024, 16) == 9
    assert v(tsylv.FP64, 4096, 64) == 10 and v(tsylv.FP64, 8192, 128) == 13
    assert v(tsylv.FP32, 4096, 64) == 1 and v(tsylv.FP32, 8192, 128) == 3
    for prec in (tsylv.FP64, tsylv.FP32, tsylv.BF16):
        for n, s in ((8, 1), (300, 24), (4096, 200)):
            assert 0 <= v(prec, n, s) < tsylv.apply_variants(prec)
    with pytest.raises(tsylv.TsylvError):
        v(7, 100, 10)
    with pytest.raises(tsylv.TsylvError):
        v(tsylv.FP64, 0, 10)
