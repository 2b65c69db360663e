"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that the headers under include/ declare, and rejects
invalid problem descriptions before touching the device."""
import ctypes as ct
import os
import re

import pytest

from paper_2502_09758_amd import _lib as L
from paper_2502_09758_amd import build as B

INCLUDE = os.path.join(B.ROOT, "include")


@pytest.fixture(scope="module")
def lib():
    if not B.built():
        B.build()
    return L.lib()


def declared():
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if f.endswith(".h"):
            text = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, f)).read(), flags=re.S)
            names |= set(re.findall(r"\b(maid(?:1d)?_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_binding_exports():
    assert declared() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared():
        assert hasattr(lib, name), name


def _desc(**kw):
    d = dict(H=32, W=32, C=1, K=5, dtype=0, boundary=0, reg=0, alpha=1e-3, eps_tv=1e-2, beta=0.0, h1_w0=1.0)
    d.update(kw)
    return L.maid_desc(**d)


@pytest.mark.parametrize("bad,msg", [
    (dict(K=4), "odd"), (dict(K=33), "odd"), (dict(K=0), "odd"), (dict(K=7, H=5), "exceed"),
    (dict(C=0), "C must"), (dict(C=4), "C must"), (dict(dtype=2), "dtype"), (dict(reg=3), "reg"),
    (dict(alpha=-1.0), "alpha"), (dict(alpha=float("nan")), "alpha"), (dict(eps_tv=0.0), "eps_tv"),
    (dict(beta=-1.0), "beta"), (dict(H=0), "H and W"), (dict(boundary=1), "periodic"), (dict(boundary=2), "boundary"),
    (dict(C=3, kc=2), "kc"), (dict(C=1, kc=3), "kc"), (dict(kc=-1), "kc"),
])
def test_create_rejects_invalid_descriptions(lib, bad, msg):
    h = ct.c_void_p(123)
    rc = lib.maid_create(ct.byref(_desc(**bad)), ct.byref(h))
    assert rc == L.EINVAL
    assert h.value is None
    assert msg in lib.maid_last_error(None).decode()


def test_null_arguments_rejected(lib):
    assert lib.maid_create(None, None) == L.EINVAL
    assert lib.maid_lower_solve(None, None, None, None, 0.0, 1, None, None, None, None) == L.EINVAL
    assert lib.maid_step(None, None, None, None, None, None, None) == L.EINVAL
    lib.maid_destroy(None)
