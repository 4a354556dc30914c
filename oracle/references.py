"""Deterministic reference values for the MBPT energy integrals.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy/scipy,
fp64, written from the definitions in the paper's Sec. "Many-body
expressions" (Eqs. (1)-(5), eq:Dijkabc and the sum shorthand below
Eq. (5)) and from
textbook results:

* ``free_gas_per_particle``: kinetic part of the first-order energy with a free
  spectrum, (3/5) hbar^2 kF^2 / 2m per species.
* ``first_order``: the first-order two-body term 1/2 sum_ij <ij|V(1-P12)|ij>
  reduced to a 1-D integral over the relative momentum p: the centre-of-mass
  integral is the volume of the lens cut out of two Fermi spheres whose centres
  are 2p apart.
* ``second_order_pnm``: Eq. (2) in neutron matter as a 5-D Gauss-Legendre
  integral over (K, p', cos theta', p, cos theta) with the azimuth done by the
  trapezoidal rule, using rotational invariance and analytic Pauli limits.
* ``lee_yang_x2``: the same machinery for a contact interaction with the
  vacuum second-Born term added back (medium-subtracted second order); its
  ratio to (3/5) E_F (kF a)^2 is the Huang-Yang/Lee-Yang coefficient
  4 (11 - 2 ln 2) / (21 pi^2).
"""
import math

import numpy as np

HBARC = 197.3269804


def fermi_momentum(n_species):
    """kF = (3 pi^2 n_tau)^(1/3) for one species density n_tau [fm^-3]."""
    return (3.0 * math.pi ** 2 * n_species) ** (1.0 / 3.0)


def free_gas_per_particle(density, x, hbar2_m=41.47):
    """T/A = (3/5) (hbar^2/2m) [(1-x) kF_n^2 + x kF_p^2]  [MeV]."""
    kn = fermi_momentum((1.0 - x) * density)
    kp = fermi_momentum(x * density)
    return 0.6 * 0.5 * hbar2_m * ((1.0 - x) * kn ** 2 + x * kp ** 2)


def lens_volume(R1, R2, d):
    """Volume of the intersection of two balls of radii R1, R2, centres d apart."""
    R1, R2, d = float(R1), float(R2), float(d)
    if R1 <= 0.0 or R2 <= 0.0:
        return 0.0
    if d >= R1 + R2:
        return 0.0
    if d <= abs(R1 - R2):
        r = min(R1, R2)
        return 4.0 / 3.0 * math.pi * r ** 3
    return (math.pi * (R1 + R2 - d) ** 2
            * (d * d + 2.0 * d * (R1 + R2) - 3.0 * (R1 - R2) ** 2) / (12.0 * d))


def _V_pair(p, C0, Cy, mpi, Lam, reg_exp, hbarc):
    """Direct V(p, p) and exchange V(p, -p) for relative momentum magnitude p."""
    f2 = math.exp(-2.0 * (p / Lam) ** reg_exp)
    vd = hbarc * (C0 + Cy / (mpi * mpi)) * f2
    ve = hbarc * (C0 + Cy / (4.0 * p * p + mpi * mpi)) * f2
    return vd, ve


def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def _gl_interval(a, b, n):
    x, w = _gl(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def first_order(density, x, q=2, C0=-1.0, Cy=-2.0, mpi=0.7, Lambda=2.0, reg_exp=4.0,
                hbarc=HBARC, npts=200):
    """First-order (two-body) energy per particle [MeV].

    E1/V = 1/2 sum_{labels} int d^3k_i d^3k_j/(2pi)^6 n_i n_j <ij|V(1-P12)|ij>
         = (2pi)^-6 int 4 pi p^2 dp * 1/2 [ g_d sum_{ti,tj} 8 Lens(kF_ti, kF_tj, 2p) V_d
                                            - g_e sum_t 8 Lens(kF_t, kF_t, 2p) V_e ]
    with g_d = 4 spin pairs and g_e = 2 equal-spin states.  q=2 is neutron
    matter (one isospin), q=4 spin x isospin.
    """
    if q == 2:
        kfs = [fermi_momentum(density)]
        if x != 0.0:
            raise ValueError("neutron matter needs x = 0")
    else:
        kfs = [fermi_momentum((1.0 - x) * density), fermi_momentum(x * density)]
    pairs = [(a, b) for a in kfs for b in kfs]
    pmax = max(kfs)
    # breakpoints where the lens formula changes branch
    bps = {0.0, pmax}
    for a, b in pairs:
        for v in (abs(a - b) / 2.0, (a + b) / 2.0):
            if 0.0 < v < pmax:
                bps.add(v)
    bps = sorted(bps)
    total = 0.0
    for lo, hi in zip(bps[:-1], bps[1:]):
        ps, ws = _gl_interval(lo, hi, npts)
        for p, w in zip(ps, ws):
            vd, ve = _V_pair(p, C0, Cy, mpi, Lambda, reg_exp, hbarc)
            direct = 4.0 * sum(8.0 * lens_volume(a, b, 2 * p) for a, b in pairs)
            exch = 2.0 * sum(8.0 * lens_volume(a, a, 2 * p) for a in kfs)
            total += w * 4.0 * math.pi * p * p * 0.5 * (direct * vd - exch * ve)
    return total / (2.0 * math.pi) ** 6 / density


def contact_first_order(density, x, q=2, C0=-1.0, hbarc=HBARC):
    """Unregulated contact, first order: E/V = V0 [rho^2/2 - (rho_n^2 + rho_p^2)/4]
    for spin x isospin; neutron matter gives V0 rho^2 / 4."""
    V0 = C0 * hbarc
    rn, rp = (1.0 - x) * density, x * density
    if q == 2:
        return V0 * density / 4.0
    return V0 * (0.5 * density ** 2 - 0.25 * (rn ** 2 + rp ** 2)) / density


# --------------------------------------------------------------------------
# Second order, neutron matter: reduced-dimension quadrature
# --------------------------------------------------------------------------

def _graded(a, b, n, power=3, at="lo"):
    """Gauss-Legendre nodes on [a, b] clustered at one end by a power map."""
    t, w = _gl_interval(0.0, 1.0, n)
    ws = (b - a) * power * t ** (power - 1) * w
    if at == "lo":
        return a + (b - a) * t ** power, ws
    return b - (b - a) * t ** power, ws


def _ls_pnm(p, pp, pdotpp, C0, Cy, mpi, Lam, reg_exp, hbarc):
    """Spin-summed <ij|V(1-P12)|ab><ab|V(1-P12)|ij> in neutron matter:
    4 Vd^2 + 4 Ve^2 - 4 Vd Ve with Vd = V(p, p'), Ve = V(p, -p')."""
    f = np.exp(-(p / Lam) ** reg_exp - (pp / Lam) ** reg_exp)
    q2m = p * p + pp * pp - 2.0 * pdotpp
    q2p = p * p + pp * pp + 2.0 * pdotpp
    vd = hbarc * (C0 + Cy / (q2m + mpi * mpi)) * f
    ve = hbarc * (C0 + Cy / (q2p + mpi * mpi)) * f
    return 4.0 * vd * vd + 4.0 * ve * ve - 4.0 * vd * ve


def _second_order_core(kF, hbar2_m, ls_fn, n_k=24, n_pp=24, n_cp=16, n_p=32, n_c=24,
                       n_phi=32, pcut=None, vacuum=False):
    """E2/V [MeV fm^-3] of Eq. (2) in neutron matter,

       E2/V = 1/4 (2pi)^-9 int d^3K d^3p' d^3p n_i n_j (1-n_a)(1-n_b) LS / D,

    K = k_i + k_j = k_a + k_b along z, p' = (k_i - k_j)/2 in the xz plane,
    p = (k_a - k_b)/2, D = (hbar^2/m)(p'^2 - p^2).  Holes need
    K p'|cos theta'| < kF^2 - K^2/4 - p'^2, particles need
    K p |cos theta| <= K^2/4 + p^2 - kF^2.  The integrand is even under
    (cos theta, cos theta') -> -(cos theta, cos theta'), so cos theta' >= 0 is
    integrated and doubled.

    vacuum=True (constant LS only) adds the vacuum second-Born piece
    LS (m/hbar^2)/p^2 over all p; where both particle factors are 1
    (p > K/2 + kF) the sum of the two pieces, LS (m/hbar^2) p'^2/(p^2 (p'^2 - p^2)),
    is integrated in closed form to infinity."""
    phis = (np.arange(n_phi) + 0.5) * (2.0 * math.pi / n_phi)
    wphi = 2.0 * math.pi / n_phi
    cphi = np.cos(phis)
    xc, wc_ref = _gl(n_c)  # reference nodes on [-1, 1] for cos theta
    ls0 = float(ls_fn(1.0, 1.0, np.zeros((1, 1)))[0, 0]) if vacuum else 0.0
    total = 0.0
    Ks, wK = _gl_interval(0.0, 2.0 * kF, n_k)
    for K, wk in zip(Ks, wK):
        pp_max = math.sqrt(max(kF * kF - K * K / 4.0, 0.0))
        pmin = pp_max
        pfull = K / 2.0 + kF
        pbr = kF - K / 2.0  # for p' below this the whole hole angular range is allowed
        segs = []
        if 0.0 < pbr < pp_max:
            segs.append(_gl_interval(0.0, pbr, n_pp))
            segs.append(_graded(pbr, pp_max, n_pp, power=3, at="hi"))
        else:
            segs.append(_graded(0.0, pp_max, n_pp, power=3, at="hi"))
        # particle relative momenta: graded at pmin up to pfull, plain above
        pieces = [_graded(pmin, pfull, n_p, power=3, at="lo")]
        if not vacuum and pcut is not None and pcut > pfull:
            pieces.append(_gl_interval(pfull, pcut, n_p))
        ps = np.concatenate([x for x, _ in pieces])
        wps = np.concatenate([w for _, w in pieces])
        cm = np.minimum(1.0, (K * K / 4.0 + ps * ps - kF * kF) / (K * ps))
        keep = cm > 0.0
        ps, wps, cm = ps[keep], wps[keep], cm[keep]
        cs = cm[:, None] * xc[None, :]                  # (p, c)
        wcs = cm[:, None] * wc_ref[None, :]
        ss = np.sqrt(np.maximum(0.0, 1.0 - cs * cs))
        for pps, wpp in segs:
            for pp, wp in zip(pps, wpp):
                cmax = (kF * kF - K * K / 4.0 - pp * pp) / (K * pp) if K * pp > 0 else 1.0
                cmax = min(1.0, cmax)
                if cmax <= 0.0:
                    continue
                cps, wcp = _gl_interval(0.0, cmax, n_cp)
                sps = np.sqrt(np.maximum(0.0, 1.0 - cps * cps))
                # dot[c', p, c, phi]
                dot = (ps[None, :, None, None] * pp
                       * (cs[None, :, :, None] * cps[:, None, None, None]
                          + ss[None, :, :, None] * sps[:, None, None, None]
                          * cphi[None, None, None, :]))
                ls = ls_fn(ps[None, :, None, None], pp, dot)
                val = ls.sum(axis=3) * wphi                      # (c', p, c)
                val = (val * wcs[None, :, :]).sum(axis=2)        # (c', p)
                acc = (val * (wps * ps * ps / (hbar2_m * (pp * pp - ps * ps)))[None, :]).sum(axis=1)
                if vacuum:
                    # int_{|p| < pfull} d^3p / p^2 = 4 pi pfull, and
                    # int_{pfull}^inf 4 pi p'^2 / (p'^2 - p^2) dp
                    #   = -2 pi p' ln((pfull + p') / (pfull - p'))
                    acc = acc + ls0 / hbar2_m * (4.0 * math.pi * pfull
                                                 - 2.0 * math.pi * pp
                                                 * math.log((pfull + pp) / (pfull - pp)))
                inner = 2.0 * float(acc @ wcp)
                total += wk * K * K * wp * pp * pp * inner
    return 0.25 * (2.0 * math.pi) ** -9 * 4.0 * math.pi * 2.0 * math.pi * total


def second_order_pnm(density, C0=-1.0, Cy=-2.0, mpi=0.7, Lambda=2.0, reg_exp=4.0,
                     hbar2_m=41.47, hbarc=HBARC, pcut_factor=3.5, **npts):
    """Second-order energy per particle in neutron matter [MeV], Eq. (2)."""
    kF = fermi_momentum(density)

    def ls(p, pp, dot):
        return _ls_pnm(p, pp, dot, C0, Cy, mpi, Lambda, reg_exp, hbarc)

    pcut = kF + pcut_factor * Lambda
    return _second_order_core(kF, hbar2_m, ls, pcut=pcut, **npts) / density


def lee_yang_x2(kF, C0=-0.1, hbar2_m=41.47, hbarc=HBARC, **npts):
    """Medium-subtracted second order for an unregulated contact V0 = C0 hbarc,
    divided by (3/5) E_F (kF a)^2 with a = m V0 / (4 pi hbar^2).
    The Huang-Yang/Lee-Yang value is 4 (11 - 2 ln 2) / (21 pi^2)."""
    V0 = C0 * hbarc

    def ls(p, pp, dot):
        return np.full(np.shape(dot), 4.0 * V0 * V0)

    density = kF ** 3 / (3.0 * math.pi ** 2)
    x2 = _second_order_core(kF, hbar2_m, ls, vacuum=True, **npts) / density
    EF = 0.5 * hbar2_m * kF * kF
    a = V0 / (4.0 * math.pi * hbar2_m)
    return x2 / (0.6 * EF * (kF * a) ** 2)


LEE_YANG_COEF = 4.0 * (11.0 - 2.0 * math.log(2.0)) / (21.0 * math.pi ** 2)
