"""Host-side checks of the C ABI library (no GPU needed)."""

import os
import re

import pytest

from paper_2601_03935_amd import gsis as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "gsis.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsis_[a-z_]+)\s*\(", text)))


def test_header_matches_binding_list():
    assert _declared() == sorted(G.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = G.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_default_opts():
    o = G.default_opts()
    assert o.scheme == G.GSIS_GSIS and o.precision == G.GSIS_FP32
    assert o.kin_sweeps == 8 and o.max_inner == 100 and o.n_precond == 10 and o.limiter_K == 5.0
    o2 = G.default_opts(precision="fp64", scheme="cis", tol=1e-8)
    assert o2.precision == G.GSIS_FP64 and o2.scheme == G.GSIS_CIS and o2.tol == 1e-8


def test_null_handle_errors():
    L = G.lib()
    assert L.gsis_set_stream(None, None) == G.GSIS_E_ARG
    assert L.gsis_kinetic_step(None) == G.GSIS_E_ARG
    assert L.gsis_last_error(None) == b"null handle"
