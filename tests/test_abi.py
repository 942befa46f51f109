"""The C-ABI library loads and exports every function include/vie.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'vie.h')
LIB = os.path.join(ROOT, 'paper_1903_07884_amd', 'libvie.so')


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    return sorted(set(re.findall(r'\b(?:vie_status|const char \*)\s*(\w+)\s*\(', text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ('vie_create', 'vie_matvec', 'precond_setup', 'precond_apply', 'vie_solve', 'vie_last_error'):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason='libvie.so not built')
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason='libvie.so not built')
def test_binding_names_match_header():
    from paper_1903_07884_amd import vie
    assert sorted(vie.EXPORTS) == declared_functions()
    vie.load(LIB)


@pytest.mark.skipif(not os.path.exists(LIB), reason='libvie.so not built')
def test_argument_errors_before_device_work():
    """Checks that return before any HIP call: usable without a GPU."""
    from paper_1903_07884_amd import vie
    lib = vie.load(LIB)
    out = ctypes.c_void_p(123)
    chi = (ctypes.c_double * 2)(0.0, 0.0)
    for grid, dx, k in (((0, 1, 1), 1e-8, 1.0), ((2, -1, 1), 1e-8, 1.0), ((1, 1, 1), 0.0, 1.0),
                        ((1, 1, 1), 1e-8, -1.0), ((1, 1, 1), float('nan'), 1.0)):
        g = (ctypes.c_int32 * 3)(*grid)
        st = lib.vie_create(g, dx, k, ctypes.cast(chi, ctypes.c_void_p), None, None, ctypes.byref(out))
        assert st == -1 and out.value is None
        assert lib.vie_last_error().decode().startswith('vie_create')
    assert lib.vie_create(None, 1e-8, 1.0, None, None, None, ctypes.byref(out)) == -1
    assert lib.vie_matvec(None, None, None, 1, 0, None) == -1
    assert lib.precond_apply(None, None, None, 1, 0, None) == -1
    assert lib.vie_solve(None, None, None, None, 1, None, None, None) == -1
    assert lib.precond_setup(None, None, None, ctypes.byref(out)) == -1 and out.value is None
    assert lib.vie_destroy(None) == 0 and lib.precond_destroy(None) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason='libvie.so not built')
def test_server_argument_errors_before_device_work():
    """The serving calls reject NULL handles and bad options before touching the device."""
    from paper_1903_07884_amd import vie
    lib = vie.load(LIB)
    out = ctypes.c_void_p(123)
    bad = vie.ServerOpts(-1, 0, 0)
    assert lib.vie_server_create(ctypes.byref(bad), ctypes.byref(out)) == -1 and out.value is None
    assert lib.vie_last_error().decode().startswith('vie_server_create')
    assert lib.vie_server_create(None, None) == -1
    rid = ctypes.c_int64()
    assert lib.vie_server_submit(None, None, None, None, ctypes.byref(rid)) == -1
    assert lib.vie_server_wait(None, 1, None) == -1
    done = ctypes.c_int32()
    assert lib.vie_server_query(None, 1, ctypes.byref(done)) == -1
    assert lib.vie_server_info_get(None, None) == -1
    assert lib.vie_server_destroy(None) == 0
