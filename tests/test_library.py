"""CPU checks of the C ABI library: it loads and exports every symbol that
include/hgks.h declares (no compute calls: there is no GPU here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "hgks.h")).read()
    decl = r"^(?:hgks_status|void|int64_t|size_t|const char\*)\s+\*?(hgks_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, txt, flags=re.M)))


def test_header_lists_entry_points():
    syms = declared_symbols()
    for s in ("hgks_create", "hgks_load_mesh", "hgks_residual", "hgks_jv", "hgks_implicit_step",
              "hgks_solve_steady", "hgks_set_bc", "hgks_set_freestream"):
        assert s in syms


def test_library_exports_all_declared_symbols():
    from paper_2304_09485_amd import hgks
    if not os.path.exists(hgks.LIB_PATH):
        pytest.skip("libhgks.so not built")
    L = hgks.load_library()
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert missing == []
    assert sorted(hgks.SYMBOLS) == declared_symbols()


def test_default_options_match_paper():
    from paper_2304_09485_amd import hgks
    if not os.path.exists(hgks.LIB_PATH):
        pytest.skip("libhgks.so not built")
    o = hgks.default_options()
    assert (o.krylov_dim, o.restarts, o.jacobi_sweeps) == (10, 3, 2)
    assert (o.cfl, o.tau_eps, o.tau_C, o.gamma, o.gamma_lin) == (10.0, 0.1, 1.0, 1.4, 0.025)
