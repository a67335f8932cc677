"""CPU-only checks of the C-ABI library: it loads, exports every function that
include/ea.h declares, and rejects malformed descriptions before it touches a
device.  No compute call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1403_4560_amd import binding, workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ea.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ea_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # and the binding covers the same set
    assert sorted(n for n, _, _ in binding._SIGS) == names


def _desc(work, **over):
    arrs = dict(sid=np.ascontiguousarray(work.sample_id, dtype=np.uint32),
                L=np.ascontiguousarray(work.L, dtype=np.int32),
                nT=np.ascontiguousarray(work.n_temps, dtype=np.int32),
                beta=np.ascontiguousarray(work.beta, dtype=np.float64),
                h=np.ascontiguousarray(work.h, dtype=np.float32),
                J=np.ascontiguousarray(work.J), spins=np.ascontiguousarray(work.spins0, dtype=np.int8))
    arrs.update(over)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p).value
    d = binding.Desc(len(arrs["L"]), p(arrs["sid"]), p(arrs["L"]), p(arrs["nT"]), p(arrs["beta"]),
                     p(arrs["h"]), int(over.get("jkind", work.jkind)), p(arrs["J"]), p(arrs["spins"]),
                     1, int(over.get("m", 10)), int(over.get("start", 0)), int(over.get("tier", 0)))
    return d, arrs


def _create(d):
    h = ctypes.c_void_p()
    st = binding.load().ea_create_ensemble(ctypes.byref(d), None, ctypes.byref(h))
    return st, h, binding.load().ea_last_error().decode()


@pytest.fixture
def small():
    return W.make_workload([4, 4], 3, (0.5, 2.0), [0.3, 0.2])


def test_rejects_odd_L(small):
    d, keep = _desc(small, L=np.array([4, 5], dtype=np.int32))
    st, h, msg = _create(d)
    assert st == -5 and not h.value and "odd" in msg


def test_rejects_bad_spin(small):
    sp = small.spins0.copy()
    sp[7] = 0
    d, keep = _desc(small, spins=sp)
    st, h, msg = _create(d)
    assert st == -1 and "spin" in msg


def test_rejects_off_grid_coupling(small):
    J = small.J.copy()
    J[3] = np.float32(0.1)
    d, keep = _desc(small, J=J)
    st, h, msg = _create(d)
    assert st == -1 and "grid" in msg


def test_rejects_large_coupling(small):
    J = small.J.copy()
    J[0] = np.float32(8.0)
    d, keep = _desc(small, J=J)
    assert _create(d)[0] == -1


def test_rejects_pm1_alphabet():
    w = W.make_workload([4], 2, (0.5, 2.0), 0.4, jkind=W.J_PM1)
    J = w.J.copy()
    J[1] = 2
    d, keep = _desc(w, J=J)
    st, h, msg = _create(d)
    assert st == -1 and "+-1" in msg


def test_rejects_bad_beta(small):
    b = small.beta.copy()
    b[1] = b[0] * 0.5
    d, keep = _desc(small, beta=b)
    assert _create(d)[0] == -1
    b = small.beta.copy()
    b[0] = np.nan
    d, keep = _desc(small, beta=b)
    assert _create(d)[0] == -1


def test_rejects_bad_sizes(small):
    d, keep = _desc(small, nT=np.array([3, 0], dtype=np.int32))
    assert _create(d)[0] == -1
    d, keep = _desc(small, L=np.array([4, 34], dtype=np.int32))
    assert _create(d)[0] == -1
    d, keep = _desc(small, m=-1)
    assert _create(d)[0] == -1


def test_null_handles_are_rejected():
    lib = binding.load()
    assert lib.ea_sweep_pt(None, 1) == -4
    assert lib.ea_measure(None, 0, None, None, None) == -4
    assert lib.ea_create_ensemble(None, None, None) == -1
    lib.ea_destroy(None)


def test_rejects_unknown_tier(small):
    d, keep = _desc(small, tier=4)
    st, h, msg = _create(d)
    assert st == -1 and not h.value and "tier" in msg


def test_rejects_beta_beyond_the_acceptance_bound(small):
    b = small.beta.copy()
    b[-1] = 2.0 ** 21
    d, keep = _desc(small, beta=b)
    st, h, msg = _create(d)
    assert st == -1 and not h.value and "2^20" in msg


def test_query_sizes_and_bind_reject_null_arguments(small):
    lib = binding.load()
    n = ctypes.c_size_t(7)
    assert lib.ea_query_sizes(None, ctypes.byref(n)) == -1
    d, keep = _desc(small)
    assert lib.ea_query_sizes(ctypes.byref(d), None) == -1
    d, keep = _desc(small, L=np.array([4, 5], dtype=np.int32))
    assert lib.ea_query_sizes(ctypes.byref(d), ctypes.byref(n)) == -5 and n.value == 0
    assert lib.ea_bind_buffers(None, None, 0) == -4
