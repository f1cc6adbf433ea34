"""CPU-side checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects bad configurations on the host before any launch."""
import ctypes
import os
import re

import pytest

from paper_2603_14982_amd import lbm

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lbm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 15
    L = lbm.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lbm.EXPORTS)


def _cfg(**kw):
    base = dict(levels=2, n=(64, 64, 64), bc=(0,) * 6, tau0=0.6, max_blocks=600)
    base.update(kw)
    return lbm.make_config(**base)


def test_buffer_sizes():
    L = lbm.lib()
    c = _cfg()
    pool = L.lbm_pool_bytes(ctypes.byref(c))
    assert pool == 2 * 601 * 10 * 512 * 4  # 600 slots + the all-zero slot
    c16 = _cfg(storage="bf16", scale=[64.0] * 10)
    assert L.lbm_pool_bytes(ctypes.byref(c16)) == pool // 2
    assert L.lbm_meta_bytes(ctypes.byref(c)) > 600 * (27 * 4 + 2 * 512)


@pytest.mark.parametrize("kw,msg", [
    (dict(tau0=0.5), "tau0"),
    (dict(levels=0), "levels"),
    (dict(levels=6), "levels"),
    (dict(n=(60, 64, 64)), "multiple"),
    (dict(levels=3, n=(48, 64, 64)), "multiple"),
    (dict(bc=(0, 1, 0, 0, 0, 0)), "pairs"),
    (dict(bc=(7, 7, 0, 0, 0, 0)), "boundary"),
    (dict(max_blocks=0), "max_blocks"),
    (dict(storage="bf16", scale=[0.0] * 10), "scales"),
    (dict(n=(1 << 20, 1 << 20, 1 << 20)), "too large"),
    (dict(bc=(1, 4, 0, 0, 0, 0), log_inflow=(3, 0.1, 0.0)), "log inflow"),
    (dict(bc=(1, 4, 0, 0, 0, 0), log_inflow=(2, -0.1, 0.0)), "log inflow"),
    (dict(bc=(1, 4, 0, 0, 0, 0), log_inflow=(2, float("nan"), 0.0)), "log inflow"),
])
def test_invalid_configurations_are_rejected_on_host(kw, msg):
    L = lbm.lib()
    c = _cfg(**kw)
    assert L.lbm_pool_bytes(ctypes.byref(c)) == 0
    h = ctypes.c_void_p()
    st = L.lbm_create(ctypes.byref(c), None, None, 0, ctypes.byref(h))
    assert st == -1
    assert msg in L.lbm_last_error(None).decode()
    assert not h.value


def test_open_boundary_configuration_accepted_and_unknown_profile_rejected():
    L = lbm.lib()
    c = _cfg(bc=(1, 4, 0, 0, 3, 3), log_inflow=(2, 0.05, 4.0))
    assert L.lbm_pool_bytes(ctypes.byref(c)) > 0
    c.inflow_profile = 2
    assert L.lbm_pool_bytes(ctypes.byref(c)) == 0
    h = ctypes.c_void_p()
    assert L.lbm_create(ctypes.byref(c), None, None, 0, ctypes.byref(h)) == -1
    assert "inflow profile" in L.lbm_last_error(None).decode()


def test_coupling_configuration():
    L = lbm.lib()
    plain = L.lbm_meta_bytes(ctypes.byref(_cfg()))
    c = _cfg(coupling=True)
    assert L.lbm_meta_bytes(ctypes.byref(c)) >= plain + 601 * 4 * 512 * 4  # fields of every slot
    c.coupling = 2
    assert L.lbm_meta_bytes(ctypes.byref(c)) == 0
    h = ctypes.c_void_p()
    assert L.lbm_create(ctypes.byref(c), None, None, 0, ctypes.byref(h)) == -1
    assert "coupling" in L.lbm_last_error(None).decode()


def test_missing_buffers_rejected():
    L = lbm.lib()
    c = _cfg()
    h = ctypes.c_void_p()
    assert L.lbm_create(ctypes.byref(c), None, None, 0, ctypes.byref(h)) == -1
    assert "pool" in L.lbm_last_error(None).decode()


def test_null_context_calls_fail_cleanly():
    L = lbm.lib()
    assert L.lbm_step(None, 1) == -1
    assert L.lbm_remesh(None, None, 0) == -1
    assert L.lbm_destroy(None) == -1
    out = ctypes.c_int64()
    assert L.lbm_num_blocks(None, 0, ctypes.byref(out)) == -1
    assert L.lbm_set_option(None, 0, 16384) == -1
    assert L.lbm_set_coupling(None, None, None, 0) == -1
    assert L.lbm_scalar_advance(None, 1.0, 0.0, None) == -1
    assert L.lbm_scalar_set(None, None, None, 0) == -1
    assert L.lbm_scalar_get(None, None, None) == -1


def test_null_context_state_and_adjoint_calls_fail_cleanly():
    L = lbm.lib()
    assert L.lbm_state_bytes(None) == 0
    assert L.lbm_adjoint_work_bytes(None, 1) == 0
    assert L.lbm_adjoint_steps(None, None, 0, 1, None, None, None, 0) == -1
    assert L.lbm_step_record(None, 1, None, 0) == -1
    assert L.lbm_adjoint_reverse(None, None, None, None, 0) == -1
    assert L.lbm_save(None, None, 0) == -1
    assert L.lbm_load(None, None, 0) == -1
    assert L.lbm_adjoint_step(None, None, 0, None, None, None, 0) == -1
    lo = (ctypes.c_int32 * 3)(0, 0, 0)
    assert L.lbm_loss_ke_grad(None, 0, lo, lo, None) == -1
