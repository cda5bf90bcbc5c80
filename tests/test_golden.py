"""Golden values the paper prints, checked against the oracle's defaults and
the internal-degree-of-freedom formula of Sec. 2."""
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def load():
    out = {}
    with open(os.path.join(HERE, "golden", "paper_parameters.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val = line.split()[:2]
            out[name] = float(val)
    return out


def test_oracle_defaults_match_paper(oracle_lib):
    g = load()
    o = oracle_lib.default_options()
    for k in ("tau_eps", "tau_C", "gamma", "gamma_lin", "krylov_dim", "restarts", "jacobi_sweeps", "cfl"):
        assert getattr(o, k) == pytest.approx(g[k]), k
    assert (5 - 3 * g["gamma"]) / (g["gamma"] - 1) == pytest.approx(g["K_internal"])
