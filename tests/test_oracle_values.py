"""Oracle values pinned against closed forms, textbook limits and
deterministic quadrature (all independent of the Monte Carlo pipeline)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import references as R


def test_free_gas_matches_printed_T0(golden):
    g = golden["fermi_energy_T0"]
    # T0 = E_F of one species at n0/2; (3/5) E_F is the free-gas energy per particle
    EF = R.free_gas_per_particle(g["n0"], 0.5) / 0.6
    assert abs(EF - g["value_MeV"]) < 0.5 * 10 ** (-g["printed_digits"])
    # neutron matter at n = 0.08 has the same Fermi momentum
    assert R.free_gas_per_particle(0.08, 0.0) == pytest.approx(0.6 * EF, rel=1e-12)


@pytest.mark.parametrize("q,x,n", [(2, 0.0, 0.08), (4, 0.5, 0.16), (4, 0.3, 0.16), (4, 0.0, 0.12)])
def test_first_order_contact_closed_form(q, x, n):
    val = R.first_order(n, x, q=q, Cy=0.0, Lambda=1e8)
    assert val == pytest.approx(R.contact_first_order(n, x, q=q), rel=1e-12)


def test_lee_yang_coefficient(golden):
    """Medium-subtracted second order for a contact interaction reproduces the
    Huang-Yang/Lee-Yang (kF a)^2 coefficient: pins the 1/4 prefactor, spin sum,
    (2pi)^-9 measure, Pauli geometry and denominators of the quadrature."""
    val = R.lee_yang_x2(1.0, n_k=12, n_pp=12, n_cp=8, n_p=16, n_c=12, n_phi=4)
    assert val == pytest.approx(golden["huang_yang_coefficient"]["value"], rel=2e-6)
    # independent of kF and of the coupling (dimensionless ratio)
    val2 = R.lee_yang_x2(0.6, C0=-0.02, n_k=12, n_pp=12, n_cp=8, n_p=16, n_c=12, n_phi=4)
    assert val2 == pytest.approx(val, rel=1e-9)


def test_second_order_quadrature_converged():
    a = R.second_order_pnm(0.08, n_k=12, n_pp=12, n_cp=8, n_p=16, n_c=12, n_phi=16)
    b = R.second_order_pnm(0.08, n_k=16, n_pp=16, n_cp=12, n_p=24, n_c=16, n_phi=24)
    assert abs(a - b) < 1e-4 * abs(b)
    assert b < 0.0


def _z(r, ref):
    return (r.mean - ref) / r.sigma


@pytest.mark.parametrize("n", [0.04, 0.12, 0.20])
def test_mc_first_order_pnm(n):
    ref = R.first_order(n, 0.0)
    r, I, V, e = O.integrate(O.problem(1, density=n, seed=1), 1 << 16, 8)
    assert abs(_z(r, ref)) < 3.0


def test_mc_first_order_nuclear():
    ref = R.first_order(0.16, 0.3, q=4)
    r, I, V, e = O.integrate(O.problem(1, density=0.16, proton_fraction=0.3, q=4,
                                       label_method=1), 1 << 16, 8)
    assert abs(_z(r, ref)) < 3.0


def test_mc_second_order_pnm_and_seed_stability():
    ref = R.second_order_pnm(0.08, n_k=16, n_pp=16, n_cp=12, n_p=24, n_c=16, n_phi=24)
    zs = []
    for seed in (1, 2, 3, 4):
        r, I, V, e = O.integrate(O.problem(2, density=0.08, seed=seed), 1 << 18, 10)
        zs.append(_z(r, ref))
    assert all(abs(z) < 3.0 for z in zs), zs
    # z-scores of independent seeds are N(0,1)-like
    assert sum(z * z for z in zs) < 16.0
