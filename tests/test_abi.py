"""Host-side checks of the C ABI: the library loads, exports every entry
point include/ile.h declares, and rejects bad configurations before touching
a device.  No compute calls (these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_1902_04934_amd import ile, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ile.LIB_PATH):
        from paper_1902_04934_amd import build
        build.build()
    return ile.lib()


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "ile.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ile_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(L):
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for s in range(8):
        assert L.ile_status_string(s)
    assert L.ile_status_string(ile.ILE_OK) == b"ok"


def _cfg(**kw):
    modes = (ile.Mode * 2)(ile.Mode(2, 2), ile.Mode(2, -2))
    base = dict(n_det=2, n_lm=2, modes=modes, srate_hz=4096.0, n_t=201,
                d_ref_mpc=100.0, gmst_rad=0.0, earth_radius_m=6378e3,
                t_ref_max_s=0.01, precision=0, device=0, stream=None)
    base.update(kw)
    cfg = ile.Config(base["n_det"], base["n_lm"], base["modes"], base["srate_hz"],
                     base["n_t"], base["d_ref_mpc"], base["gmst_rad"],
                     base["earth_radius_m"], base["t_ref_max_s"], base["precision"],
                     base["device"], base["stream"])
    return cfg, modes


@pytest.mark.parametrize("bad", [
    dict(n_t=200), dict(n_t=0), dict(n_det=0), dict(n_det=5), dict(n_lm=0),
    dict(n_lm=33), dict(srate_hz=0.0), dict(d_ref_mpc=-1.0), dict(t_ref_max_s=-1e-3),
    dict(precision=7), dict(earth_radius_m=0.0),
])
def test_create_rejects_bad_config(L, bad):
    cfg, _keep = _cfg(**bad)
    h = C.c_void_p()
    assert L.ile_create(C.byref(cfg), C.byref(h)) == ile.ILE_E_ARG
    assert not h.value


def test_create_rejects_bad_modes(L):
    modes = (ile.Mode * 2)(ile.Mode(2, 3), ile.Mode(2, -2))
    cfg, _ = _cfg(modes=modes)
    h = C.c_void_p()
    assert L.ile_create(C.byref(cfg), C.byref(h)) == ile.ILE_E_ARG
    modes = (ile.Mode * 1)(ile.Mode(9, 0))
    cfg, _ = _cfg(modes=modes, n_lm=1)
    assert L.ile_create(C.byref(cfg), C.byref(h)) == ile.ILE_E_ARG


def test_null_arguments(L):
    assert L.ile_create(None, None) == ile.ILE_E_ARG
    assert L.ile_eval(None, None, 0, None) == ile.ILE_E_ARG
    assert L.ile_set_data(None, None, 0, 0.0, None, None, None) == ile.ILE_E_ARG
    assert L.ile_sync(None) == ile.ILE_E_ARG
    L.ile_destroy(None)


def test_create_without_gpu_reports_device(L):
    """With a valid config, creation either succeeds (GPU present) or says
    ILE_E_DEVICE (none, as in the build container)."""
    cfg, _keep = _cfg()
    h = C.c_void_p()
    st = L.ile_create(C.byref(cfg), C.byref(h))
    assert st in (ile.ILE_OK, ile.ILE_E_DEVICE)
    if st == ile.ILE_OK:
        L.ile_destroy(h)


def test_binding_raises_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(ile, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(ile, "_lib", None)
    with pytest.raises(ImportError):
        ile.lib()


def test_binding_types_every_declared_symbol(L):
    """The ctypes binding gives every declared entry point its argument
    types (an untyped call would pass Python ints as 32-bit C ints and
    truncate pointers)."""
    missing = [n for n in declared_symbols() if getattr(L, n).argtypes is None]
    assert not missing, missing
