"""The paper's printed condition numbers and iteration counts (Tables 1-4)
reproduced by the oracle (paper mode: unrestarted left-preconditioned GMRES,
x0 = 0, tolerance 1e-7; kappa = 2-norm condition number of P^{-1} M; the
diagonal factor on the tau D side)."""
import json
import os

import pytest

from oracle import examples as ex

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)["rows"]


T1 = load("table1_example1.json")
T2 = load("table2_example1.json")
T34 = load("tables34_examples23.json")


@pytest.mark.parametrize("row", T1, ids=lambda r: f"n{r['n1p1']}-a{r['alpha']}")
def test_table1_kappa(row):
    s, _ = ex.ex1_system(row["n1p1"] - 1, row["alpha"])
    assert ex.kappa(s) == pytest.approx(row["I_kappa"], abs=0.05)
    assert ex.kappa(s, "tau", "right") == pytest.approx(row["PF_kappa"], abs=0.05)


@pytest.mark.parametrize("row", [r for r in T1 if r["n1p1"] <= 128], ids=lambda r: f"n{r['n1p1']}-a{r['alpha']}")
def test_table1_iterations(row):
    n = row["n1p1"] - 1
    _, _, it_i = ex.run_ex1(n, row["alpha"], solver="gmres", prec="none")
    _, _, it_p = ex.run_ex1(n, row["alpha"], solver="gmres", prec="tau", dside="right")
    assert it_i == pytest.approx(row["I_it"], abs=1e-9)   # exact
    assert it_p == pytest.approx(row["PF_it"], abs=0.1)   # printed to one decimal


@pytest.mark.parametrize("row", T2, ids=lambda r: f"n{r['n1p1']}-a{r['alpha']}")
def test_table2(row):
    n = row["n1p1"] - 1
    s, _ = ex.ex1_system(n, row["alpha"])
    assert ex.kappa(s, "tri") == pytest.approx(row["tri_kappa"], abs=0.05)
    assert ex.kappa(s, "tilde") == pytest.approx(row["tilde_kappa"], abs=0.05)
    _, _, it_t = ex.run_ex1(n, row["alpha"], solver="gmres", prec="tri")
    _, _, it_p = ex.run_ex1(n, row["alpha"], solver="gmres", prec="tilde")
    assert it_t == pytest.approx(row["tri_it"], abs=1e-9)
    assert it_p == pytest.approx(row["tilde_it"], abs=0.1)


@pytest.mark.parametrize("row", T34, ids=lambda r: f"ex{r['example']}-n{r['n']}")
def test_tables3_4(row):
    n, beta = row["n"], row["beta"]
    s, _, _ = ex.ex2_system(n, 1.8, beta)
    assert ex.kappa(s) == pytest.approx(row["I_kappa"], abs=0.05)
    assert ex.kappa(s, "tau", "right") == pytest.approx(row["PF_kappa"], abs=0.05)
    _, _, it_i = ex.run_ex2(n, 1.8, beta, solver="gmres", prec="none")
    _, _, it_p = ex.run_ex2(n, 1.8, beta, solver="gmres", prec="tau", dside="right")
    assert it_i == pytest.approx(row["I_it"], abs=0.1)
    assert it_p == pytest.approx(row["PF_it"], abs=0.1)


def test_discretisation_orders():
    """Example 1 is first order in h (Section 1.2), Example 2 second order
    (Section 1.3 weights with Crank-Nicolson): halving h halves / quarters the
    error against the exact solution at T = 1."""
    e = []
    for n in (63, 127):
        u, ue, _ = ex.run_ex1(n, 1.2)
        e.append(abs(u - ue).max())
    assert e[0] < 0.04 and 1.8 < e[0] / e[1] < 2.2
    e = []
    for n in (16, 32):
        u, ue, _ = ex.run_ex2(n)
        e.append(abs(u - ue).max())
    assert e[0] < 0.1 and 3.4 < e[0] / e[1] < 4.6
