"""The FP64 oracle against closed forms, invariants and brute force (CPU)."""

import inspect
import sys

import pytest

import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


def test_every_oracle_function_is_run_by_a_pin():
    """A function of the oracle that no pin executes is unpinned: its
    mistakes would pass every check.  Trace the pins and require each
    function defined in an oracle module to be entered at least once."""
    from oracle import adjoint, analytic, das, dbclip, fir, moments

    modules = (das, adjoint, analytic, dbclip, fir, moments)
    called = set()

    def prof(frame, event, arg):
        if event == "call":
            called.add((frame.f_code.co_filename, frame.f_code.co_name))

    sys.setprofile(prof)
    try:
        for pin in P.ALL_PINS:
            pin()
    finally:
        sys.setprofile(None)
    missing = [f"{m.__name__}.{name}" for m in modules
               for name, fn in inspect.getmembers(m, inspect.isfunction)
               if fn.__module__ == m.__name__ and (fn.__code__.co_filename, name) not in called]
    assert not missing, f"oracle functions no pin runs: {missing}"
