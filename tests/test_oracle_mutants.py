"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each mutant is a one-line change of oracle/oracle.cpp (a dropped term, a
wrong sign, a swapped index, a transposed operand, a wrong factor), built
into a temporary library and loaded in place of the real one; the pin suite
of tests/test_oracle_pins.py is then run against it and at least one pin
must fail.  The real oracle is restored afterwards.
"""
import inspect
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.cpp")

MUTANTS = {
    "drop the phi32 term of P_ee":
        ("u3 * u1 * (sn31 * sn31) +\n                      u3 * u2 * (sn32 * sn32));",
         "u3 * u1 * (sn31 * sn31));"),
    "wrong sign of the CP (Im) term":
        ("p += 2.0 * x.imag() * std::sin(2.0 * half_phase);",
         "p -= 2.0 * x.imag() * std::sin(2.0 * half_phase);"),
    "swapped mass-splitting index":
        ("const double half_phase = (K_PHASE * L) / E * dm2[i][j];",
         "const double half_phase = (K_PHASE * L) / E * dm2[j][i];"),
    "wrong |U_e1|^2":
        ("const T u1 = (1.0 - s12) * (1.0 - s13);", "const T u1 = (1.0 - s12) * (1.0 + s13);"),
    "transposed smearing matrix":
        ("acc += tb.R[(size_t)i * nb + j] * (th[4] * mu0[j]);",
         "acc += tb.R[(size_t)j * nb + i] * (th[4] * mu0[j]);"),
    "wrong GL weight":
        ("const double wi = 2.0 / ((1.0 - x * x) * dpn * dpn);",
         "const double wi = 2.0 / ((1.0 + x * x) * dpn * dpn);"),
    "wrong quadrature weight scale":
        ("w[k] = h * wt[i];", "w[k] = 2.0 * h * wt[i];"),
    "chi2 without its factor 2":
        ("*out = 2.0 * acc;", "*out = acc;"),
    "wrong sign of d P / d dm21":
        ("dp[0] = -4.0 * (u2 * u1 * T21 * q - u3 * u2 * T32 * q);",
         "dp[0] = -4.0 * (u2 * u1 * T21 * q + u3 * u2 * T32 * q);"),
    "IBD threshold not clamped":
        ("if (x <= me) return 0.0;", "if (x <= 0.0) return 0.0;"),
    "resolution without sqrt2":
        ("const double den = sqrt2 * sig;", "const double den = sig;"),
    "adjoint uses R instead of R^T":
        ("for (int i = 0; i < nb; ++i) acc += tb.R[(size_t)i * nb + j] * gnu[i];",
         "for (int i = 0; i < nb; ++i) acc += tb.R[(size_t)j * nb + i] * gnu[i];"),
    "phase constant off in the 5th digit":
        ("constexpr double K_PHASE = 1266.9326794198487;",
         "constexpr double K_PHASE = 1266.9426794198487;"),
    "spectrum quadratic term linear in E":
        ("std::exp(a[0] + a[1] * E + a[2] * E * E + a[3] * E * E * E)",
         "std::exp(a[0] + a[1] * E + a[2] * E + a[3] * E * E * E)"),
    "spectrum cubic term quadratic in E":
        ("std::exp(a[0] + a[1] * E + a[2] * E * E + a[3] * E * E * E)",
         "std::exp(a[0] + a[1] * E + a[2] * E * E + a[3] * E * E)"),
    "spectrum constant term dropped":
        ("std::exp(a[0] + a[1] * E + a[2] * E * E + a[3] * E * E * E)",
         "std::exp(a[1] * E + a[2] * E * E + a[3] * E * E * E)"),
    "CP phase of the mixing matrix with the opposite sign":
        ("const cplx eid = std::polar(1.0, dcp);   // e^{+i delta}\n"
         "  const cplx emid = std::polar(1.0, -dcp); // e^{-i delta}",
         "const cplx eid = std::polar(1.0, -dcp);\n"
         "  const cplx emid = std::polar(1.0, dcp);"),
    "baseline weight ignored":
        ("acc += wr * pee_point<double>(E[i], L[r], theta[0], theta[1], theta[2], theta[3]);",
         "acc += pee_point<double>(E[i], L[r], theta[0], theta[1], theta[2], theta[3]);"),
    "bin integration without its weights":
        ("acc += (w ? w[k] : 1.0) * x[v * npts + k];", "acc += x[v * npts + k];"),
    "smearing transform contracts against the reversed vector":
        ("acc += r * x[v * n_in + c];", "acc += r * x[v * n_in + (n_in - 1 - c)];"),
    "d chi2 / d nu with the wrong sign of the data term":
        ("dchi2_dnu[v * nb + i] = 2.0 * (1.0 - dv[i] / nv[i]);",
         "dchi2_dnu[v * nb + i] = 2.0 * (1.0 + dv[i] / nv[i]);"),
}


def _pin_calls():
    """Every pin of the suite, with one representative argument per parameter."""
    calls = []
    for name, fn in inspect.getmembers(pins, inspect.isfunction):
        if not name.startswith("test_"):
            continue
        params = inspect.signature(fn).parameters
        args = {}
        for p in params:
            args[p] = {"L": 1300.0, "n": 5, "order": 5, "n_sub": 4, "which": "mini_multiL"}[p]
        calls.append((name, fn, args))
    return calls


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of '{name}' not found exactly once"
    mut = tmp_path / "mut.cpp"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / f"lib_{abs(hash(name))}.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                    "-fPIC", "-shared", str(mut), "-o", str(lib)], check=True)
    return str(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    lib = _build(tmp_path, name, old, new)
    monkeypatch.setattr(oracle, "_LIBPATH", lib)
    monkeypatch.setattr(oracle, "_lib", None)
    caught = []
    try:
        for pin, fn, args in _pin_calls():
            try:
                fn(**args)
            except (AssertionError, oracle.OracleError, FloatingPointError, ValueError):
                caught.append(pin)
                break
    finally:
        monkeypatch.setattr(oracle, "_lib", None)
    assert caught, f"no pin catches the mutant '{name}'"


def test_unmutated_oracle_passes_every_pin_call():
    for pin, fn, args in _pin_calls():
        fn(**args)
