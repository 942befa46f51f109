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
