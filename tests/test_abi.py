"""Host-side checks of the C ABI library (no GPU needed)."""

import os
import re

import pytest

from paper_2601_03935_amd import gsis as G
from paper_2601_03935_amd import warmstart as WS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("gsis.h", "gsis_warmstart.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(gsis_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_matches_binding_list():
    assert _declared() == sorted(G.EXPORTS + WS.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = G.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_default_opts():
    o = G.default_opts()
    assert o.scheme == G.GSIS_GSIS and o.precision == G.GSIS_FP32
    assert o.kin_sweeps == 8 and o.max_inner == 100 and o.n_precond == 10 and o.limiter_K == 10.0
    o2 = G.default_opts(precision="fp64", scheme="cis", tol=1e-8)
    assert o2.precision == G.GSIS_FP64 and o2.scheme == G.GSIS_CIS and o2.tol == 1e-8


def test_mlp_argument_errors():
    L = WS._lib()
    import ctypes as C

    h = C.c_void_p()
    assert L.gsis_mlp_create(0, 0, 8, 2, 1, 0, C.byref(h)) == G.GSIS_E_ARG
    assert L.gsis_mlp_create(0, 3, 8, 65, 1, 0, C.byref(h)) == G.GSIS_E_ARG
    assert L.gsis_mlp_forward(None, 1, None, None) == G.GSIS_E_ARG
    assert L.gsis_mlp_forward_noalloc(None, 1, None, None) == G.GSIS_E_ARG
    assert L.gsis_mlp_num_params(None) == G.GSIS_E_ARG


def test_null_handle_errors():
    L = G.lib()
    assert L.gsis_set_stream(None, None) == G.GSIS_E_ARG
    assert L.gsis_kinetic_step(None) == G.GSIS_E_ARG
    assert L.gsis_last_error(None) == b"null handle"
