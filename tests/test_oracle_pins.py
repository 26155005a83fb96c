"""Oracle pins (CPU).  Tolerances (in tests/oracle_pins.PINS): exact for counts and
orderings; float64 rounding (1e-12 relative) for identities that hold exactly; looser
where an iteration or a finite difference sets the accuracy."""
import pytest

from tests import oracle_pins as P


@pytest.mark.parametrize("name,fn,kw,tol", P.PINS, ids=[p[0] for p in P.PINS])
def test_pin(name, fn, kw, tol):
    err = fn(**kw)
    assert err <= tol, f"{name}: error {err:.3e} > {tol:.1e}"
