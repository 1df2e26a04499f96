"""The CPU oracle against facts fixed by the paper and by mathematics (CPU only)."""
import pytest

import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(None)


@pytest.mark.parametrize("k", [256, 4096, 16384])
def test_plain_oracle_true_error(k):
    """How far the plain oracle is from the exact product, measured against the pinned
    doubled-precision reference: far below the 1e-13 parity bar at every k."""
    import numpy as np

    import oracle
    import synth
    m, n = 24, 20
    p = synth.problem(97, k, "N", "N", m, n, k, ld_rule=lambda r: max(1, r))
    plain, dd = p["C"].copy(), p["C"].copy()
    assert oracle.dgemm("N", "N", m, n, k, 1.0, p["A"], m, p["B"], k, 1.0, plain, m) == 0
    assert oracle.dgemm_dd("N", "N", m, n, k, 1.0, p["A"], m, p["B"], k, 1.0, dd, m) == 0
    D = np.zeros(m * n)
    assert oracle.absden("N", "N", m, n, k, 1.0, p["A"], m, p["B"], k, 1.0, p["C"], m, D, m) == 0
    err = float(np.max(np.abs(plain[: m * n] - dd[: m * n]) / D))
    print(f"[plain oracle true error] k={k}: {err:.2e}")
    assert err <= 1e-14
