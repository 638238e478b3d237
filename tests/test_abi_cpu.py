"""The C-ABI library loads and exports every symbol include/aco.h declares, and
its host-side logic (sizes, argument checks, gamma schedule) behaves, without
touching a GPU: every call here returns before the first HIP runtime call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aco.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aco_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("aco_create", "aco_transition", "aco_construct", "aco_update", "aco_run",
                     "aco_destroy", "aco_last_error", "aco_workspace_bytes"):
        assert required in names
    text = open(HEADER).read()
    assert "torch" not in text.lower().replace("pytorch", "")
    assert 'extern "C"' in text


def test_library_exports_every_declared_symbol():
    from paper_2404_04895_amd import _native
    L = _native.lib()
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(_declared_functions()) <= set(_native.SIGNATURES)


def test_sizes_are_pure():
    from paper_2404_04895_amd import _native
    L = _native.lib()
    assert L.aco_leading_dim(1) == 64 and L.aco_leading_dim(64) == 64
    assert L.aco_leading_dim(65) == 128 and L.aco_leading_dim(5000) == 5056
    assert L.aco_workspace_bytes(2, 10) == 0
    assert L.aco_workspace_bytes(_native.MAX_CITIES + 1, 10) == 0
    assert L.aco_workspace_bytes(10, 0) == 0
    b = L.aco_workspace_bytes(5000, 5000)
    assert b % 256 == 0
    # four padded FP32 matrices + tours + succ/pred dominate
    assert b >= 4 * 5000 * 5056 * 4 + 3 * 5000 * 5000 * 4
    assert L.aco_workspace_bytes(100, 10) < L.aco_workspace_bytes(100, 20)


def test_argument_errors_before_any_device_call():
    from paper_2404_04895_amd import _native
    L = _native.lib()
    out = ctypes.c_void_p(123)
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: the checks fail first
    ws = ctypes.c_void_p(0x200000)

    def create(n=10, alpha=1.0, beta=2.0, rho=0.5, Q=1.0, m_max=10, ws_ptr=ws, nbytes=1 << 30,
               dist=fake):
        return L.aco_create(dist, n, alpha, beta, rho, Q, m_max, ws_ptr, nbytes, None,
                            ctypes.byref(out))

    assert create(n=2) == _native.ACO_EINVAL
    assert create(n=_native.MAX_CITIES + 1) == _native.ACO_EINVAL
    assert create(m_max=0) == _native.ACO_EINVAL
    assert create(alpha=-1.0) == _native.ACO_EINVAL
    assert create(beta=float("nan")) == _native.ACO_EINVAL
    assert create(rho=0.0) == _native.ACO_EINVAL
    assert create(rho=1.5) == _native.ACO_EINVAL
    assert create(Q=0.0) == _native.ACO_EINVAL
    assert create(dist=None) == _native.ACO_EINVAL
    assert create(ws_ptr=None) == _native.ACO_EINVAL
    assert create(ws_ptr=ctypes.c_void_p(0x200010)) == _native.ACO_EINVAL  # misaligned
    assert create(nbytes=1) == _native.ACO_ENOMEM
    assert out.value is None
    assert b"workspace" in L.aco_last_error()
    assert L.aco_create(fake, 10, 1.0, 2.0, 0.5, 1.0, 10, ws, 1 << 30, None, None) == \
        _native.ACO_EINVAL
    # calls on a NULL context
    assert L.aco_transition(None, 1.0) == _native.ACO_EINVAL
    assert L.aco_construct(None, 1, 0, 0) == _native.ACO_EINVAL
    assert L.aco_update(None, 1.0) == _native.ACO_EINVAL
    assert L.aco_run(None, 1, 0, 1, None, None) == _native.ACO_EINVAL
    assert L.aco_deposit_scale(None) == -1
    assert L.aco_sorted_prefix(None) == 0
    assert L.aco_batch_sorted_walk_stats(None, None) == _native.ACO_EINVAL
    assert L.aco_sorted_rows(None) is None and L.aco_sorted_cities(None) is None
    assert L.aco_uniforms(0, 0, 0, 0, -1, None, None) == _native.ACO_EINVAL
    L.aco_destroy(None)


def test_gamma_schedule_matches_oracle():
    import oracle
    from paper_2404_04895_amd import gamma_schedule
    for T in (1, 2, 3, 10, 100, 200, 500):
        for t in list(range(0, min(T + 2, 60))) + [T - 1, T, T + 5]:
            for gmax, gmin in ((1.5, 1.0), (2.0, 0.5), (1.0, 1.0)):
                assert gamma_schedule(t, T, gmax, gmin) == oracle.gamma(t, T, gmax, gmin), \
                    (t, T, gmax, gmin)


def test_product_path_does_not_reach_the_oracle():
    """The package and its library never import, link or load the oracle."""
    pkg = os.path.join(ROOT, "paper_2404_04895_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), os.path.join(dirpath, f)


def test_batch_and_setter_argument_errors_before_any_device_call():
    from paper_2404_04895_amd import _native
    L = _native.lib()
    i32 = lambda *v: (ctypes.c_int32 * len(v))(*v)
    i64 = lambda *v: (ctypes.c_int64 * len(v))(*v)
    u64 = lambda *v: (ctypes.c_uint64 * len(v))(*v)
    # sizes: empty batch, an instance below 3 cities or above the maximum, no ants
    assert L.aco_batch_workspace_bytes(i32(10), i32(10), 0) == 0
    assert L.aco_batch_workspace_bytes(i32(10, 2), i32(10, 10), 2) == 0
    assert L.aco_batch_workspace_bytes(i32(_native.MAX_CITIES + 1), i32(4), 1) == 0
    assert L.aco_batch_workspace_bytes(i32(10), i32(0), 1) == 0
    assert L.aco_batch_workspace_bytes(i32(10, 3), i32(10, 1), 2) > 0
    out = ctypes.c_void_p(123)
    fake = ctypes.c_void_p(0x100000)
    ws = ctypes.c_void_p(0x200000)

    def create(n, m, count, offsets=None):
        offsets = offsets or i64(*([0] * max(count, 1)))
        return L.aco_batch_create(fake, offsets, n, m, u64(*([0] * max(count, 1))), count, 1.0,
                                  2.0, 0.5, 1.0, None, ws, 1 << 30, None, ctypes.byref(out))

    assert create(i32(10), i32(10), 0) == _native.ACO_EINVAL            # empty batch
    assert create(i32(10, 2), i32(10, 10), 2) == _native.ACO_EINVAL     # n = 2
    assert create(i32(10), i32(0), 1) == _native.ACO_EINVAL             # no ants
    assert create(i32(10), i32(10), 1, i64(-1)) == _native.ACO_EINVAL   # bad offset
    assert out.value is None
    # the selection, walk and bounds setters on a NULL context
    assert L.aco_set_selection(None, 0) == _native.ACO_EINVAL
    assert L.aco_set_sorted_walk(None, 4) == _native.ACO_EINVAL
    assert L.aco_set_tau_bounds(None, 0.0, 1.0) == _native.ACO_EINVAL
    assert L.aco_set_schedule(None, -1) == _native.ACO_EINVAL
