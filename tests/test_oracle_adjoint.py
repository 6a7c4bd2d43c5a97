"""Pins of the oracle's adjoint of the density response (CPU only): second
divided differences against 50-digit decimal arithmetic, the vector-Jacobian
product against finite differences of the forward oracle, and self-adjointness
of the response; plus planted mistakes that the pins must catch."""
import numpy as np

import oracle
import oracle.lrdm_oracle as Lo
from tests import pins as P


def test_second_divided_differences_50_digit_decimal():
    assert P.pin_second_divided_differences_decimal() < 1e-9


def test_vjp_matches_finite_differences():
    assert P.pin_vjp_fd() < 1e-8


def test_vjp_self_adjoint():
    assert P.pin_vjp_self_adjoint() < 1e-12


ORIG_D = Lo.second_divided_differences
ORIG_FD = Lo.fermi_derivatives


def _patch(mp, name, fn):
    mp.setattr(Lo, name, fn)
    mp.setattr(oracle, name, fn)


def test_planted_transposed_second_differences_is_caught(monkeypatch):
    _patch(monkeypatch, "second_divided_differences", lambda e, mu, kT: ORIG_D(e, mu, kT).T)
    assert P.pin_vjp_fd() > 1e-6


def test_planted_dropped_taylor_term_is_caught(monkeypatch):
    def bad(e, mu, kT):
        f1, f2, f3, _ = ORIG_FD(e, mu, kT)
        return f1, f2, f3, 0.0 * f3
    _patch(monkeypatch, "fermi_derivatives", bad)
    assert P.pin_second_divided_differences_decimal() > 1e-9


def test_planted_wrong_fermi_shift_in_adjoint_is_caught(monkeypatch):
    orig = Lo.fermi_shift
    calls = {"n": 0}

    def bad(Hp, fp):
        # the adjoint's second call per direction (nu) returns a wrong value
        calls["n"] += 1
        v = orig(Hp, fp)
        return -v if calls["n"] % 2 == 0 else v
    monkeypatch.setattr(Lo, "fermi_shift", bad)
    _, g, Psi, eps, ne, kT, dV, G = P._vjp_case(1, seed=3)
    gdV, _, _ = Lo.density_response_vjp(Psi, eps, g, ne, kT, dV, G, 1)
    monkeypatch.setattr(Lo, "fermi_shift", orig)
    ref = Lo.density_response(Psi, eps, g, ne, kT, G, 1)[0]
    assert np.linalg.norm(gdV - ref) / np.linalg.norm(ref) > 1e-6
