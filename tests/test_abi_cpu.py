"""The C-ABI library loads without a GPU, exports every function that include/*.h declares, and
its host-only random-choice decisions agree with the oracle's independent Philox."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import oracle
import paper_2103_08932_amd as tl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(tlsph_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def library():
    if not os.path.exists(tl.LIB_PATH):
        from paper_2103_08932_amd import build
        build.build()
    return tl.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tlsph_create_body", "tlsph_set_material", "tlsph_set_loads", "tlsph_set_damping",
                     "tlsph_relax_until", "tlsph_get_displacement", "tlsph_destroy_body", "tlsph_step"):
        assert required in names


def test_every_declared_symbol_is_exported(library):
    missing = [n for n in declared_functions() if not hasattr(library, n)]
    assert not missing, missing


def test_version_and_error_strings(library):
    assert "gfx950" in tl.version()
    assert isinstance(tl.last_error(), str)


def test_decisions_match_oracle(library):
    for seed, alpha in ((0, 0.2), (1, 0.2), (7, 0.5), (123456789, 0.05), (3, 1.0)):
        got = tl.damping_decisions(seed, alpha, 0, 3000)
        ref = np.array([oracle.damped_decision(seed, n, alpha) for n in range(3000)], np.uint8)
        assert np.array_equal(got, ref), (seed, alpha)
    got = tl.damping_decisions(5, 0.2, 10**12, 100)
    ref = np.array([oracle.damped_decision(5, 10**12 + q, 0.2) for q in range(100)], np.uint8)
    assert np.array_equal(got, ref)


def test_decisions_reject_bad_alpha(library):
    with pytest.raises(tl.TLSPHError):
        tl.damping_decisions(0, 0.0, 0, 10)
    with pytest.raises(tl.TLSPHError):
        tl.damping_decisions(0, 1.5, 0, 10)


def test_create_body_rejects_bad_arguments_before_device_work(library):
    h = ctypes.c_void_p()
    desc = tl._BodyDesc()
    assert library.tlsph_create_body(ctypes.byref(desc), ctypes.byref(h)) == tl.E_INVALID
    assert "NULL" in tl.last_error()
    X = np.zeros((3, 2))
    desc.X0 = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    desc.dim = 4
    desc.n = 3
    assert library.tlsph_create_body(ctypes.byref(desc), ctypes.byref(h)) == tl.E_INVALID
    assert "dim" in tl.last_error()
    desc = tl._BodyDesc(2, 3, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, -1.0, 1.3, 1000.0, 32, None,
                        tl._Allocator())
    assert library.tlsph_create_body(ctypes.byref(desc), ctypes.byref(h)) == tl.E_INVALID
    desc.dp = 0.002
    desc.precision = 16
    assert library.tlsph_create_body(ctypes.byref(desc), ctypes.byref(h)) == tl.E_INVALID
    assert not h.value


def test_server_rejects_bad_arguments_before_device_work(library):
    h = ctypes.c_void_p()
    alloc = tl._Allocator()
    assert library.tlsph_server_create(1 << 30, 0, 32, None, alloc, ctypes.byref(h)) == tl.E_INVALID
    assert "max_slots" in tl.last_error()
    assert library.tlsph_server_create(1 << 30, 65, 32, None, alloc, ctypes.byref(h)) == tl.E_INVALID
    assert library.tlsph_server_create(1 << 30, 8, 16, None, alloc, ctypes.byref(h)) == tl.E_INVALID
    assert "precision" in tl.last_error()
    assert library.tlsph_server_create(1024, 8, 32, None, alloc, ctypes.byref(h)) == tl.E_INVALID
    assert "budget" in tl.last_error()
    assert not h.value
    t = ctypes.c_int64()
    q = tl._Request()
    assert library.tlsph_server_submit(None, ctypes.byref(q), ctypes.byref(t)) == tl.E_INVALID
    done = ctypes.c_int()
    assert library.tlsph_server_wait(None, 1, 0.0, ctypes.byref(done), None, None) == tl.E_INVALID
    assert library.tlsph_server_error(None, 1) == b""


def test_null_body_calls_are_rejected(library):
    """Every call that takes a body handle rejects NULL with TLSPH_E_INVALID before any device work."""
    import numpy as np
    out = np.zeros(4)
    assert library.tlsph_set_damping_scheme(None, tl.PARTICLE) == tl.E_INVALID
    assert library.tlsph_set_damping(None, 1.0, 0.0, 0.0, 0.2, 1) == tl.E_INVALID
    assert library.tlsph_set_material(None, tl.NEOHOOKE, 1e6, 0.3) == tl.E_INVALID
    assert library.tlsph_get_von_mises(None, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == tl.E_INVALID
    assert library.tlsph_get_von_mises_noalloc(None, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == \
        tl.E_INVALID
    assert "NULL" in tl.last_error()
