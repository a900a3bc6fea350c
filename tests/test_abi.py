"""CPU checks of the C-ABI library: it loads without a GPU and exports every
function include/hipib.h declares; configuration defaults; argument errors that
the host rejects before touching the device."""
import ctypes as C

import pytest


def test_library_exports_every_declared_symbol():
    from paper_2503_22695_amd import hipib
    L = hipib.lib()
    names = hipib.exported_names()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_default_config_values():
    from paper_2503_22695_amd import hipib
    cfg = hipib.default_config()
    assert (cfg.mg_pre, cfg.mg_post, cfg.mg_coarse_sweeps, cfg.mg_max_cycles) == (2, 2, 0, 50)
    assert cfg.mg_rtol == 1e-10 and cfg.convection == 1 and cfg.precision == hipib.FP64
    assert cfg.deterministic == 0 and cfg.mg_krylov == 1


@pytest.mark.parametrize("n", [7, 20, 40, 2048])
def test_create_rejects_bad_sizes_on_host(n):
    """n must be 4*2^k or 6*2^k (every multigrid level even); checked before any
    device call."""
    from paper_2503_22695_amd import hipib
    cfg = hipib.default_config(n=n)
    h = C.c_void_p()
    st = hipib.lib().hipib_create(C.byref(cfg), None, C.byref(h))
    assert st == hipib.E_INVAL and not h.value
    assert b"n =" in hipib.lib().hipib_last_error()


def test_null_context_is_an_error():
    from paper_2503_22695_amd import hipib
    L = hipib.lib()
    assert L.hipib_fe_force(None, None, 0.0, None) == hipib.E_INVAL
    assert L.hipib_advance(None, None, None, None, 0.0, 1, 0.0, 0.0) == hipib.E_INVAL
    assert L.hipib_destroy(None) == hipib.OK


def test_cavity_pressure_waveform():
    """hipib_cavity_pressure is the load hipib_advance applies: p0 sin^2(pi t / T),
    zero for p0 = 0 or T <= 0 (host function, no GPU)."""
    import math
    from paper_2503_22695_amd import hipib
    for p0, T, t in [(1.0, 0.05, 0.0125), (2.5, 0.05, 0.05), (1.0, 0.05, 0.0), (0.7, 1.0, 0.3)]:
        sn = math.sin(math.pi * t / T)
        assert hipib.cavity_pressure(p0, T, t) == p0 * sn * sn
    assert hipib.cavity_pressure(1.0, 0.05, 0.025) == 1.0
    assert hipib.cavity_pressure(0.0, 0.05, 0.01) == 0.0
    assert hipib.cavity_pressure(1.0, 0.0, 0.01) == 0.0
    assert hipib.cavity_pressure(1.0, -1.0, 0.01) == 0.0
