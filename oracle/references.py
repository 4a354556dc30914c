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
* ``hf_self_energy``: the HF self-energy of eq:spe as a 1-D integral over the
  momentum transfer (solid angle of the partner's Fermi sphere in closed form).
* ``second_order``: Eq. (2) in neutron or asymmetric nuclear matter with the
  free or the HF spectrum (eq:Dijkabc with each line's isospin): a second,
  independent 5-D quadrature (general Pauli limits per isospin pair, the
  relative azimuth integrated in closed form).
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


# --------------------------------------------------------------------------
# Second order, neutron or nuclear matter, free or Hartree-Fock spectrum
# --------------------------------------------------------------------------

def hf_self_energy(k, density, x=0.0, q=2, tau=0, C0=-1.0, Cy=-2.0, mpi=0.7, Lambda=2.0,
                   reg_exp=4.0, hbarc=HBARC, ng=64):
    """Sigma_tau(k) [MeV] of eq:spe for the spin(-isospin)-independent
    interaction, written as a 1-D integral over u = |k - k'| = 2p:

       Sigma_tau(k) = sum_tau' (2pi)^-3 int du u^2 Omega_tau'(u) [2 Vd(u/2) - delta Ve(u/2)],

    where Omega(u) is the solid angle of the directions of u for which the
    partner k' = k - u lies inside the Fermi sphere of tau' (4 pi while
    u < kF - k, else 2 pi (1 - (k^2 + u^2 - kF^2) / (2 k u)), zero beyond
    u = k + kF), Vd(p) = V(p, p) (zero momentum transfer, both partner
    spins) and Ve(p) = V(p, -p) (transfer 2p, equal spin and isospin only).
    Array k allowed."""
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    kfs = [fermi_momentum(density)] if q == 2 else [fermi_momentum((1.0 - x) * density),
                                                    fermi_momentum(x * density)]
    tg, wg = _gl(ng)
    out = np.zeros_like(k)

    def g(u, same):
        p = 0.5 * u
        f2 = np.exp(-2.0 * (p / Lambda) ** reg_exp)
        vd = hbarc * (C0 + Cy / (mpi * mpi)) * f2
        ve = hbarc * (C0 + Cy / (4.0 * p * p + mpi * mpi)) * f2
        return 2.0 * vd - (ve if same else 0.0)

    for tp, kf in enumerate(kfs):
        if kf <= 0.0:
            continue
        same = tp == tau
        lo = np.abs(kf - k)
        # full sphere part: 0 <= u < kF - k (only when k < kF)
        full = np.where(k < kf, lo, 0.0)
        u1 = 0.5 * full[:, None] * (tg[None, :] + 1.0)
        w1 = 0.5 * full[:, None] * wg[None, :]
        acc = (w1 * u1 * u1 * 4.0 * math.pi * g(u1, same)).sum(axis=1)
        # partial part: |k - kF| < u < k + kF
        a, b = lo, k + kf
        u2 = 0.5 * (b - a)[:, None] * tg[None, :] + 0.5 * (b + a)[:, None]
        w2 = 0.5 * (b - a)[:, None] * wg[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            c0 = (k[:, None] ** 2 + u2 * u2 - kf * kf) / (2.0 * k[:, None] * u2)
        c0 = np.clip(np.nan_to_num(c0, nan=1.0), -1.0, 1.0)
        acc += (w2 * u2 * u2 * 2.0 * math.pi * (1.0 - c0) * g(u2, same)).sum(axis=1)
        out += acc / (2.0 * math.pi) ** 3
    return out


def _smooth_nodes(a, b, n):
    """Gauss-Legendre on [a, b] through s = t^2 (3 - 2t): nodes clustered at
    both ends (for the logarithmic endpoint behaviour of 1/D)."""
    t, w = _gl_interval(0.0, 1.0, n)
    s = t * t * (3.0 - 2.0 * t)
    return a + (b - a) * s, (b - a) * 6.0 * t * (1.0 - t) * w


def _segments(bps, lo, hi):
    pts = sorted({lo, hi, *[v for v in bps if lo < v < hi]})
    return list(zip(pts[:-1], pts[1:]))


def second_order(density, x=0.0, q=2, spectrum="free", C0=-1.0, Cy=-2.0, mpi=0.7,
                 Lambda=2.0, reg_exp=4.0, hbar2_m=41.47, hbarc=HBARC, pcut_factor=3.5,
                 n_k=16, n_pp=10, n_cp=10, n_p=12, n_c=10, hf_grid=0.004):
    """Second-order energy per particle [MeV], Eq. (2), with the free spectrum
    or the HF spectrum eps_tau(k) = hbar^2 k^2 / 2m + Sigma_tau(k) (eq:spe,
    eq:Dijkabc with each line's own isospin), in neutron (q = 2) or nuclear
    (q = 4, proton fraction x) matter.

    Coordinates K = k_i + k_j (along z), p' = (k_i - k_j) / 2, p = (k_a - k_b) / 2;
    the hole pair has |K/2 + p'| < kF_ti, |K/2 - p'| < kF_tj, the particle pair
    |K/2 + p| >= kF_ta, |K/2 - p| >= kF_tb, which bound cos(theta') and
    cos(theta) (the angles to K) for each (K, p', p).  The spin-summed squared
    matrix elements (equal isospins: 4 Vd^2 + 4 Ve^2 - 4 Vd Ve; unequal: 4 Vd^2
    with the particles keeping the holes' isospins, 4 Ve^2 with them swapped)
    are integrated over the relative azimuth in closed form, since only the
    Yukawa denominators depend on it:
       int dphi / (a -+ b cos phi) = 2 pi / sqrt(a^2 - b^2),
       int dphi / (a -+ b cos phi)^2 = 2 pi a / (a^2 - b^2)^(3/2),
       1 / ((a_d - b c)(a_e + b c)) = [1 / (a_d - b c) + 1 / (a_e + b c)] / (a_d + a_e).
    The remaining 5-D integral is Gauss-Legendre on pieces between the points
    where a Pauli limit changes form, graded at both ends of every piece."""
    kfs = [fermi_momentum(density)] if q == 2 else [fermi_momentum((1.0 - x) * density),
                                                    fermi_momentum(x * density)]
    if q == 2 and x != 0.0:
        raise ValueError("neutron matter needs x = 0")
    kmax_all = max(kfs)
    pcut = kmax_all + pcut_factor * Lambda
    eps_fns = []
    for t in range(len(kfs)):
        if spectrum == "hf":
            kk = np.arange(0.0, 2.0 * kmax_all + pcut + 4 * hf_grid, hf_grid)
            sig = hf_self_energy(kk, density, x, q, t, C0, Cy, mpi, Lambda, reg_exp, hbarc)
            from scipy.interpolate import CubicSpline
            spl = CubicSpline(kk, sig)
            eps_fns.append(lambda k, s=spl: 0.5 * hbar2_m * k * k + s(k))
        elif spectrum == "free":
            eps_fns.append(lambda k: 0.5 * hbar2_m * k * k)
        else:
            raise ValueError(spectrum)

    # (hole isospins, particle isospins, label-sum kind)
    combos = []
    for ti in range(len(kfs)):
        for tj in range(len(kfs)):
            if ti == tj:
                combos.append((ti, tj, ti, tj, "same"))
            else:
                combos.append((ti, tj, ti, tj, "direct"))
                combos.append((ti, tj, tj, ti, "exchange"))

    def ang_lim(kfa, kfb, K, r, hole):
        """cos-theta interval from the two Pauli conditions (arrays over r)."""
        with np.errstate(divide="ignore", invalid="ignore"):
            A = (kfa * kfa - K * K / 4.0 - r * r) / (K * r)
            B = (kfb * kfb - K * K / 4.0 - r * r) / (K * r)
        if hole:   # |K/2 + r| < kfa  and  |K/2 - r| < kfb
            return np.maximum(-1.0, -B), np.minimum(1.0, A)
        return np.maximum(-1.0, A), np.minimum(1.0, -B)   # outside both

    tc, wcr = _gl_interval(0.0, 1.0, n_c)
    sc = tc * tc * (3.0 - 2.0 * tc)
    wsc = 6.0 * tc * (1.0 - tc) * wcr
    tcp, wcpr = _gl_interval(0.0, 1.0, n_cp)
    scp = tcp * tcp * (3.0 - 2.0 * tcp)
    wscp = 6.0 * tcp * (1.0 - tcp) * wcpr
    m2 = mpi * mpi
    total = 0.0
    for ti, tj, ta, tb, kind in combos:
        ki, kj, ka, kb = kfs[ti], kfs[tj], kfs[ta], kfs[tb]
        if ki <= 0.0 or kj <= 0.0:
            continue
        ei, ej, ea, eb = eps_fns[ti], eps_fns[tj], eps_fns[ta], eps_fns[tb]
        for K0, K1 in _segments([abs(ki - kj)], 0.0, ki + kj):
            Ks, wK = _gl_interval(K0, K1, n_k)
            for K, wk in zip(Ks, wK):
                # hole relative momenta
                hb = [abs(ki - K / 2), ki + K / 2, abs(kj - K / 2), kj + K / 2]
                e2 = 0.5 * (ki * ki + kj * kj) - K * K / 4.0
                if e2 > 0:
                    hb.append(math.sqrt(e2))
                pps, wpps = [], []
                for a, b in _segments(hb, 0.0, 0.5 * (ki + kj)):
                    lo, hi = ang_lim(ki, kj, K, np.array([0.5 * (a + b)]), True)
                    if hi[0] <= lo[0]:
                        continue
                    r, w = _smooth_nodes(a, b, n_pp)
                    pps.append(r)
                    wpps.append(w)
                if not pps:
                    continue
                pp = np.concatenate(pps)
                wpp = np.concatenate(wpps)
                lo, hi = ang_lim(ki, kj, K, pp, True)
                ok = hi > lo
                pp, wpp, lo, hi = pp[ok], wpp[ok], lo[ok], hi[ok]
                cp = lo[:, None] + (hi - lo)[:, None] * scp[None, :]        # (P', C')
                wcp = (hi - lo)[:, None] * wscp[None, :]
                # particle relative momenta
                pb_ = [abs(ka - K / 2), ka + K / 2, abs(kb - K / 2), kb + K / 2]
                e2 = 0.5 * (ka * ka + kb * kb) - K * K / 4.0
                if e2 > 0:
                    pb_.append(math.sqrt(e2))
                ps, wps = [], []
                for a, b in _segments(pb_, 0.0, pcut):
                    lo2, hi2 = ang_lim(ka, kb, K, np.array([0.5 * (a + b)]), False)
                    if hi2[0] <= lo2[0]:
                        continue
                    r, w = _smooth_nodes(a, b, n_p)
                    ps.append(r)
                    wps.append(w)
                p = np.concatenate(ps)
                wp = np.concatenate(wps)
                lo2, hi2 = ang_lim(ka, kb, K, p, False)
                ok = hi2 > lo2
                p, wp, lo2, hi2 = p[ok], wp[ok], lo2[ok], hi2[ok]
                c = lo2[:, None] + (hi2 - lo2)[:, None] * sc[None, :]       # (P, C)
                wc = (hi2 - lo2)[:, None] * wsc[None, :]
                # energies: holes depend on (p', c'), particles on (p, c)
                kh1 = np.sqrt(np.maximum(0.0, K * K / 4 + pp[:, None] ** 2 + K * pp[:, None] * cp))
                kh2 = np.sqrt(np.maximum(0.0, K * K / 4 + pp[:, None] ** 2 - K * pp[:, None] * cp))
                kp1 = np.sqrt(np.maximum(0.0, K * K / 4 + p[:, None] ** 2 + K * p[:, None] * c))
                kp2 = np.sqrt(np.maximum(0.0, K * K / 4 + p[:, None] ** 2 - K * p[:, None] * c))
                eh = ei(kh1) + ej(kh2)                                       # (P', C')
                ep = ea(kp1) + eb(kp2)                                       # (P, C)
                D = eh[:, :, None, None] - ep[None, None, :, :]              # (P', C', P, C)
                # azimuth-integrated label sums
                P4 = pp[:, None, None, None]
                Q4 = p[None, None, :, None]
                ccp = cp[:, :, None, None] * c[None, None, :, :]
                ssp = (np.sqrt(np.maximum(0.0, 1 - cp * cp))[:, :, None, None]
                       * np.sqrt(np.maximum(0.0, 1 - c * c))[None, None, :, :])
                base = P4 * P4 + Q4 * Q4 + m2
                ad = base - 2.0 * P4 * Q4 * ccp
                ae = base + 2.0 * P4 * Q4 * ccp
                bb = 2.0 * P4 * Q4 * ssp
                rd = np.sqrt(ad * ad - bb * bb)
                re = np.sqrt(ae * ae - bb * bb)
                i1d, i1e = 2.0 * math.pi / rd, 2.0 * math.pi / re
                i2d, i2e = 2.0 * math.pi * ad / rd ** 3, 2.0 * math.pi * ae / re ** 3
                F2 = (hbarc * np.exp(-(P4 / Lambda) ** reg_exp - (Q4 / Lambda) ** reg_exp)) ** 2
                vdd = F2 * (2 * math.pi * C0 * C0 + 2 * C0 * Cy * i1d + Cy * Cy * i2d)
                vee = F2 * (2 * math.pi * C0 * C0 + 2 * C0 * Cy * i1e + Cy * Cy * i2e)
                if kind == "same":
                    vde = F2 * (2 * math.pi * C0 * C0 + C0 * Cy * (i1d + i1e)
                                + Cy * Cy * (i1d + i1e) / (ad + ae))
                    ls = 4.0 * vdd + 4.0 * vee - 4.0 * vde
                elif kind == "direct":
                    ls = 4.0 * vdd
                else:
                    ls = 4.0 * vee
                wt = ((wpp * pp * pp)[:, None, None, None] * wcp[:, :, None, None]
                      * (wp * p * p)[None, None, :, None] * wc[None, None, :, :])
                total += wk * K * K * float((wt * ls / D).sum())
    # 1/4 (2pi)^-9, 4 pi (K direction), 2 pi (azimuth of p' about K)
    return 0.25 * (2.0 * math.pi) ** -9 * 4.0 * math.pi * 2.0 * math.pi * total / density
