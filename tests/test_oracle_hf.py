"""Pins of the oracle's Hartree-Fock spectrum (eq:spe): the self-energy
quadrature against the first-order energy (E1 = 1/2 sum_i n_i Sigma_i,
an independent lens-volume quadrature), the contact-interaction closed form,
quadrature convergence, the spline, and the cancellation of a constant
self-energy in every energy denominator (each cut has as many holes as
particles of each isospin)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import references as R


def _e1_from_sigma(pb, ng=40):
    """(1/n) sum_tau 2 spins int_{k<kF_tau} d^3k/(2pi)^3 Sigma_tau(k) / 2."""
    xg, wg = np.polynomial.legendre.leggauss(ng)
    kf = O.fermi_momenta(pb)
    total = 0.0
    for t in range(2 if pb.q == 4 else 1):
        if kf[t] <= 0:
            continue
        ks = 0.5 * kf[t] * (xg + 1.0)
        ws = 0.5 * kf[t] * wg
        acc = sum(w * k * k * O.hf_sigma(pb, t, k, 48) for k, w in zip(ks, ws))
        total += 4.0 * math.pi / (2 * math.pi) ** 3 * acc
    return total / pb.density


@pytest.mark.parametrize("n,x,q", [(0.08, 0.0, 2), (0.16, 0.3, 4), (0.12, 0.5, 4)])
def test_hf_self_energy_gives_first_order_energy(n, x, q):
    pb = O.problem(1, 0, density=n, proton_fraction=x, q=q)
    e1 = R.first_order(n, x, q=q)
    assert abs(_e1_from_sigma(pb) - e1) < 1e-9 * abs(e1)


@pytest.mark.parametrize("n,x,q", [(0.1, 0.0, 2), (0.16, 0.25, 4)])
def test_hf_contact_closed_form(n, x, q):
    # V = hbar c C0 (no Yukawa, regulator scale far above every momentum):
    # Sigma_tau = hbar c C0 (n - n_tau / 2)
    pb = O.problem(1, 0, density=n, proton_fraction=x, q=q, Cy=0.0, Lambda=1e3)
    hc = O.DEFAULTS["hbarc"] * O.DEFAULTS["C0"]
    dens = [(1 - x) * n, x * n]
    for t in range(2 if q == 4 else 1):
        for k in (0.0, 0.7, 1.9, 3.0):
            assert abs(O.hf_sigma(pb, t, k, 32) - hc * (n - dens[t] / 2)) < 1e-10 * abs(hc * n)


def test_hf_quadrature_converged():
    pb = O.problem(2, 0, density=0.16, proton_fraction=0.3, q=4)
    for t in (0, 1):
        for k in (0.0, 0.5, 1.2, 1.45, 2.0, 4.0, 9.0):
            a, b = O.hf_sigma(pb, t, k, 64), O.hf_sigma(pb, t, k, 128)
            assert abs(a - b) <= 1e-13 * max(1.0, abs(b)), (t, k, a, b)


def test_hf_spline_nodes_and_accuracy():
    pb = O.problem(2, 0, density=0.16, proton_fraction=0.3, q=4, spectrum=1)
    h = pb.hf_kmax / pb.hf_n
    y, _ = pb._hf_keep
    for t in (0, 1):
        for i in (0, 1, 17, 200, pb.hf_n):
            assert O.hf_spline(pb, t, i * h) == pytest.approx(y[t, i], abs=1e-12)
        # between the nodes the spline follows the quadrature to 1e-7 MeV
        for k in np.linspace(0.013, 5.0, 37):
            assert abs(O.hf_spline(pb, t, k) - O.hf_sigma(pb, t, k)) < 1e-7
    assert O.hf_spline(pb, 0, pb.hf_kmax + 3.0) == y[0, -1]
    assert abs(y[0, -1]) < 1e-12


@pytest.mark.parametrize("order,did,q,n,x", [(2, 0, 2, 0.1, 0.0), (3, 1, 2, 0.12, 0.0),
                                            (2, 0, 4, 0.16, 0.3), (3, 2, 4, 0.16, 0.2)])
def test_hf_constant_self_energy_cancels(order, did, q, n, x):
    # contact interaction: Sigma_tau is constant in k, and every cut has as many
    # holes as particles of each isospin, so the HF integrand equals the free one
    kw = dict(Cy=0.0, Lambda=1e3, kcut_extra=0.0005)
    free = O.problem(order, did, density=n, proton_fraction=x, q=q, **kw)
    hf = O.problem(order, did, density=n, proton_fraction=x, q=q, spectrum=1, **kw)
    grid = O.uniform_grid(3 * (order + 1))
    w0, _ = O.sample_values(free, grid, 0, 0, 3000)
    w1, c1 = O.sample_values(hf, grid, 0, 0, 3000)
    assert np.count_nonzero(w0) > 50
    assert np.all(np.abs(w1 - w0) <= 1e-9 * c1 + 1e-300)


def test_hf_changes_the_second_order_energy():
    # with the regulated Yukawa interaction Sigma depends on k, so the HF
    # integrand differs from the free one (a sign that the spectrum is used)
    free = O.problem(2, 0, density=0.08)
    hf = O.problem(2, 0, density=0.08, spectrum=1)
    grid = O.uniform_grid(9)
    w0, _ = O.sample_values(free, grid, 0, 0, 2000)
    w1, _ = O.sample_values(hf, grid, 0, 0, 2000)
    nz = w0 != 0
    assert np.median(np.abs(w1[nz] / w0[nz] - 1.0)) > 1e-3


# ---------------------------------------------------------------------------
# The HF spectrum inside the second-order denominators, pinned by an
# independent reduced-dimension quadrature (references.second_order)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,x,q", [(0.08, 0.0, 2), (0.12, 0.1, 4)])
def test_hf_self_energy_two_quadratures(n, x, q):
    # the oracle integrates over the partner momentum k' (|k'|, angle); the
    # reference over the transfer |k - k'| with the solid angle in closed form
    pb = O.problem(1, 0, density=n, proton_fraction=x, q=q)
    ks = np.array([0.0, 0.3, 0.9, 1.2, 1.6, 2.5, 4.0])
    for t in range(2 if q == 4 else 1):
        ref = R.hf_self_energy(ks, n, x, q, t, ng=96)
        for k, r in zip(ks, ref):
            assert abs(O.hf_sigma(pb, t, k) - r) < 1e-10 * max(1.0, abs(r)), (t, k)


def test_general_second_order_quadrature_matches_neutron_matter_one():
    # two separately written quadratures of Eq. (2) (the neutron-matter one is
    # itself pinned by the Lee-Yang coefficient)
    a = R.second_order_pnm(0.08, n_k=16, n_pp=16, n_cp=12, n_p=24, n_c=16, n_phi=24)
    b = R.second_order(0.08, n_k=24, n_pp=14, n_cp=14, n_p=16, n_c=14)
    assert abs(a - b) < 3e-5 * abs(a)


@pytest.mark.parametrize("spectrum", ["free", "hf"])
def test_general_second_order_quadrature_converged(spectrum):
    a = R.second_order(0.12, 0.1, 4, spectrum=spectrum, n_k=12, n_pp=8, n_cp=8, n_p=10, n_c=8)
    b = R.second_order(0.12, 0.1, 4, spectrum=spectrum)
    assert abs(a - b) < 5e-4 * abs(b)


def test_nuclear_quadrature_neutron_limit_and_symmetry():
    # x = 0 nuclear matter is neutron matter; x <-> 1 - x is a relabelling
    a = R.second_order(0.08, 0.0, 2, spectrum="hf")
    b = R.second_order(0.08, 0.0, 4, spectrum="hf")
    assert abs(a - b) < 1e-12 * abs(a)
    c = R.second_order(0.16, 0.2, 4, spectrum="hf")
    d = R.second_order(0.16, 0.8, 4, spectrum="hf")
    assert abs(c - d) < 1e-12 * abs(c)


@pytest.mark.parametrize("n,x,q", [(0.08, 0.0, 2), (0.12, 0.1, 4), (0.16, 0.3, 4)])
def test_mc_second_order_hf_against_quadrature(n, x, q):
    """The oracle's Monte Carlo with the HF spectrum (spline tables, per-line
    isospin in every denominator) agrees with the quadrature within 3 sigma,
    while the free-spectrum value is many sigma away.  At x = 0.1 exchanging
    the neutron and proton self-energies moves the quadrature by 4% (25
    sigma here), averaging them by 2%."""
    ref = R.second_order(n, x, q, spectrum="hf")
    free = R.second_order(n, x, q, spectrum="free")
    pb = O.problem(2, 0, density=n, proton_fraction=x, q=q, spectrum=1, seed=1)
    r, I, V, e = O.integrate(pb, 1 << 18, 10)
    assert abs(r.mean - ref) < 3.0 * r.sigma, (r.mean, r.sigma, ref)
    assert abs(r.mean - free) > 30.0 * r.sigma


def test_mc_second_order_nuclear_free_against_quadrature():
    ref = R.second_order(0.16, 0.3, 4)
    pb = O.problem(2, 0, density=0.16, proton_fraction=0.3, q=4, seed=2)
    r, I, V, e = O.integrate(pb, 1 << 18, 10)
    assert abs(r.mean - ref) < 3.0 * r.sigma, (r.mean, r.sigma, ref)


@pytest.mark.parametrize("order,did,n,x", [(2, 0, 0.16, 0.2), (3, 2, 0.12, 0.35)])
def test_hf_mirror_proton_fraction(order, did, n, x):
    # exchanging neutrons and protons relabels every isospin sum: the HF
    # integrand at x equals the one at 1 - x sample by sample
    a = O.problem(order, did, density=n, proton_fraction=x, q=4, spectrum=1)
    b = O.problem(order, did, density=n, proton_fraction=1.0 - x, q=4, spectrum=1)
    grid = O.uniform_grid(3 * (order + 1))
    wa, ca = O.sample_values(a, grid, 0, 0, 600)
    wb, _ = O.sample_values(b, grid, 0, 0, 600)
    assert np.count_nonzero(wa) > 20
    assert np.all(np.abs(wa - wb) <= 1e-12 * ca + 1e-300)
