"""The C-ABI library loads and exports every symbol include/slicq.h declares;
host-only calls (plan design, parameter validation) work without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "slicq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1210_0084_amd as sq
    return sq.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("nsgt_plan", "slicq_analyze", "slicq_synthesize", "slicq_adjoint", "slicq_analyze_batched"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_plan_info_host_only(lib):
    import paper_1210_0084_amd as sq
    p = sq.Plan(44100, 110, 11025, 12, 8192, 1024)
    assert p.K == 81 and p.nbands == 83 and p.coefs_per_slice == 10208
    assert p.num_slices(0) == 0 and p.num_slices(1) == 2 and p.num_slices(8192) == 2 and p.num_slices(8193) == 4


@pytest.mark.parametrize("args", [
    (44100, 0, 100, 12, 4096, 512),          # fmin <= 0
    (44100, 200, 100, 12, 4096, 512),        # fmin >= fmax
    (44100, 100, 1000, 12, 4000, 512),       # 2N not a power of two
    (44100, 100, 1000, 12, 4096, 2048),      # M >= N
    (44100, 100, 1000, 12, 4096, 511),       # N - M odd
    (44100, 100, 1000, 0, 4096, 512),        # B < 1
    (44100, 5, 1000, 12, 256, 32),           # empty / colliding bands
])
def test_invalid_parameters_are_rejected(lib, args):
    import paper_1210_0084_amd as sq
    with pytest.raises(sq.SlicqError, match="-1"):
        sq.Plan(*args)


def test_calls_before_upload_fail_cleanly(lib):
    import paper_1210_0084_amd as sq
    p = sq.Plan(44100, 110, 11025, 12, 8192, 1024)
    rc = lib.slicq_analyze(p._h, 0, ctypes.c_void_p(16), 100, ctypes.c_void_p(16), 10 ** 6, ctypes.c_void_p(16),
                           10 ** 9, None)
    assert rc == -6 and b"upload" in lib.slicq_last_error()
    b = ctypes.c_size_t()
    assert lib.slicq_workspace_size(p._h, 0, 10, ctypes.byref(b)) == 0 and b.value > 0
    assert lib.nsgt_plan_table_bytes(p._h, 1, ctypes.byref(b)) == 0 and b.value > 0
    assert lib.slicq_workspace_size(p._h, 7, 10, ctypes.byref(b)) == -1


def test_prepared_batch_validation_host_only(lib):
    # every check of slicq_batch_create that fails returns before any device work
    import paper_1210_0084_amd as sq
    p = sq.Plan(44100, 110, 11025, 12, 8192, 1024)
    P = ctypes.c_void_p
    h = P()
    dummy = P(16)                         # never dereferenced: the calls below fail validation first
    assert lib.slicq_batch_tasks_bytes(-1) == 0
    need = lib.slicq_batch_tasks_bytes(10)
    assert need >= 10 * 96
    # nsig <= 0 / total <= 0
    assert lib.slicq_batch_create(p._h, dummy, dummy, 0, 10, 100, 100, dummy, need, None, ctypes.byref(h)) == -1
    assert lib.slicq_batch_create(p._h, dummy, dummy, 2, 0, 100, 100, dummy, need, None, ctypes.byref(h)) == -1
    # negative bounds, null buffers, null handle output
    assert lib.slicq_batch_create(p._h, dummy, dummy, 2, 10, -1, 100, dummy, need, None, ctypes.byref(h)) == -1
    assert lib.slicq_batch_create(p._h, None, dummy, 2, 10, 100, 100, dummy, need, None, ctypes.byref(h)) == -1
    assert lib.slicq_batch_create(p._h, dummy, dummy, 2, 10, 100, 100, dummy, need, None, None) == -1
    # tasks buffer too small
    assert lib.slicq_batch_create(p._h, dummy, dummy, 2, 10, 100, 100, dummy, need - 1, None, ctypes.byref(h)) == -4
    assert h.value is None
    # calls on a null batch handle
    assert lib.slicq_analyze_batch(None, 0, dummy, 1, dummy, 1, dummy, 1 << 20, None) == -1
    assert lib.slicq_synthesize_batch(None, 0, dummy, 1, dummy, 1, dummy, 1 << 20, None) == -1
    lib.slicq_batch_destroy(None)


def test_full_length_plan_host_only(lib):
    # plan checks and table sizes of the full-length transform need no device
    import paper_1210_0084_amd as sq
    p = sq.Plan(44100, 200, 22000, 48, 4096, 1024, window="blackman_harris")
    f = sq.FullPlan(p, 1 << 20, "slicq")
    assert f.nbands == 2 * p.K + 2 and f.L == 1 << 20
    assert all(int(m) == int(p.M[k if k < p.nbands else 2 * p.K + 2 - k]) * 256 for k, m in enumerate(f.M))
    assert not f.painless                                  # this lattice aliases a few bands
    g = sq.FullPlan(p, 1 << 16, "painless")
    assert g.painless and all(g.M >= g.lengths)
    b = ctypes.c_size_t()
    assert lib.nsgt_full_workspace_size(f._h, 0, ctypes.byref(b)) == 0 and b.value >= 8 * (f.L + 2 * f.coef_count)
    assert lib.nsgt_full_table_bytes(f._h, 1, ctypes.byref(b)) == 0 and b.value > 0
    rc = lib.nsgt_full_analyze(f._h, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), 10 ** 8, ctypes.c_void_p(16),
                               10 ** 10, None)
    assert rc == -6 and b"upload" in lib.slicq_last_error()
    for L, lat in ((3000, 0), (2048, 0), (1 << 25, 0), (1 << 16, 2)):
        with pytest.raises(sq.SlicqError, match="-1"):
            sq.FullPlan(p, L, "slicq") if lat != 2 else lib_call_bad_lattice(lib, p)


def lib_call_bad_lattice(lib, p):
    import paper_1210_0084_amd as sq
    h = ctypes.c_void_p()
    sq._check(lib.nsgt_full_plan(p._h, 1 << 16, 2, ctypes.byref(h)))
