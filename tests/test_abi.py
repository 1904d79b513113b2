"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/hh.h, and rejects malformed descriptors before touching a
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="hh.h"):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hh_[a-z0-9_]+)\s*\(", txt)))


def _lib():
    from paper_2601_21407_amd import hh
    return hh


def test_library_exports_every_declared_symbol():
    hh = _lib()
    names = _declared()
    assert "hh_init" in names and "hh_step_n" in names and "hh_backward" in names
    assert "hh_syn_propagate" in names
    for nm in names:
        assert hasattr(hh.lib, nm), nm
    assert set(hh.exported_symbols()) <= set(names)


def test_probe_library_is_separate():
    """The measurement probes (include/hh_probe.h) live in libhh_probe.so,
    not in the product library."""
    hh = _lib()
    from paper_2601_21407_amd import probe
    names = _declared("hh_probe.h")
    assert names == ["hh_probe_barrier", "hh_probe_barrier_bytes", "hh_probe_issue"]
    for nm in names:
        assert hasattr(probe.lib, nm), nm
        with pytest.raises(AttributeError):
            getattr(hh.lib, nm)


def test_struct_sizes_match_header_layout():
    hh = _lib()
    assert ctypes.sizeof(hh.Rate) == 20
    assert ctypes.sizeof(hh.Gate) == 44
    assert ctypes.sizeof(hh.Channel) == 44
    assert ctypes.sizeof(hh.Input) == 56
    assert ctypes.sizeof(hh.Outputs) == 40


def test_status_strings():
    hh = _lib()
    for s in range(-7, 1):
        assert hh.lib.hh_status_string(s)
    assert hh.lib.hh_status_string(-1) == b"invalid argument or descriptor"


@pytest.mark.parametrize("mutate", [
    lambda d: setattr(d, "dt", -1.0),
    lambda d: setattr(d, "C_m", 0.0),
    lambda d: setattr(d, "n_gates", 9),
    lambda d: setattr(d.gates[0].r[0], "form", 7),
    lambda d: setattr(d.gates[1], "kind", 3),
    lambda d: setattr(d.gates[0].r[1], "K", 0.0),
    lambda d: setattr(d.channels[0], "n_gates", 5),
    lambda d: d.channels[1].gate.__setitem__(0, 3),
    lambda d: d.channels[1].expo.__setitem__(0, -1),
    lambda d: setattr(d, "v_method", 2),
])
def test_malformed_descriptor_rejected(mutate):
    hh = _lib()
    from paper_2601_21407_amd import workloads as W
    d = hh.desc_from_model(W.classic_hh())
    mutate(d)
    h = ctypes.c_void_p()
    assert hh.lib.hh_init(ctypes.byref(h), ctypes.byref(d), 10, 1, None, None) == -1
    assert not h.value


def test_bad_sizes_rejected():
    hh = _lib()
    from paper_2601_21407_amd import workloads as W
    d = hh.desc_from_model(W.classic_hh())
    h = ctypes.c_void_p()
    assert hh.lib.hh_init(ctypes.byref(h), ctypes.byref(d), 0, 1, None, None) == -2
    assert hh.lib.hh_init(ctypes.byref(h), ctypes.byref(d), 1 << 30, 4, None, None) == -2
    assert hh.lib.hh_init(None, ctypes.byref(d), 10, 1, None, None) == -1
    assert hh.lib.hh_step_n(None, None, 0, 1, None, None, None) == -1
