"""The C-ABI library loads on a CPU-only host and exports every entry point
that include/esdg.h declares (no compute calls: there is no GPU here)."""
import os
import re

from paper_1804_02221_amd import esdg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "esdg.h")).read()
    return sorted(set(re.findall(r"\b(esdg_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    L = esdg.lib()
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_header():
    # every declared entry point has a ctypes signature in the binding
    src = open(os.path.join(ROOT, "paper_1804_02221_amd", "esdg.py")).read()
    for n in declared():
        assert f'"{n}"' in src, n


def test_default_params_host_only():
    p = esdg.default_params(7)
    assert p.g == 9.81 and p.h_tol == 1e-4 and p.cfl == 0.5
    assert p.sigma_min < p.sigma_max
    assert esdg.lib().esdg_abi_version() == 103
