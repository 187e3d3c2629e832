"""Apparent-permeability class table (Sec. 2.1, Eq. 3, 4, 18, 19, 38).

The oracle module oracle.kapp is pinned to closed forms derived from the
paper's equations with the ideal-gas density, and to the qualitative claims
the paper prints for its parameter studies (Sec. 3.1).  The product's native
class table (glbm_class_table, C++) is then checked against the oracle.
"""
import math

import numpy as np
import pytest

from oracle import kapp
import shale_inputs as si

ETA = 18.231e-6          # Pa s, Tab. 4
TORT = 2.0               # Tab. 4 / Tab. 7


def vbar(T):
    return math.sqrt(8 * kapp.R_GAS * T / (math.pi * kapp.M_CH4))


# ----------------------------------------------------------- closed forms --
@pytest.mark.parametrize("r,P,T,eps", [(20e-9, 5e6, 400, 0.1), (2e-9, 21e6, 350, 0.04), (1e-7, 1e5, 300, 0.3)])
def test_iom_ratio_closed_form(r, P, T, eps):
    """With rho_g = P M / (R T), Eq. (18) reduces to K_app = K_0 + eta D_K / P and
    K_app / K_0 = 1 + (32/3) eta vbar / (P d), independent of eps / tortuosity."""
    d = 2 * r
    k0 = eps / TORT * d * d / 32
    k = kapp.kapp_iom(r, P, T, eps, TORT, ETA)
    assert abs(k / k0 - (1 + 32.0 / 3.0 * ETA * vbar(T) / (P * d))) < 1e-13 * (k / k0)


def test_om_surface_term_closed_form():
    """Eq. (19) - Eq. (18) = (eta R T / P)(1 - eps) q_sat b D_s / (1 + b P): independent of the radius."""
    P, T, eps, q, b, ds = 5e6, 400.0, 0.3, 4000.0, 0.25e-6, 1e-8
    want = ETA * kapp.R_GAS * T / P * (1 - eps) * q * b * ds / (1 + b * P)
    for r in (2e-9, 5e-9, 50e-9):
        ks = kapp.kapp_om(r, P, T, eps, TORT, ETA, q, b, ds) - kapp.kapp_iom(r, P, T, eps, TORT, ETA)
        assert abs(ks - want) / want < 1e-9


def test_shale128_values():
    """The 128^2 case at its median radii: IOM K_0 = (0.1/2)(40 nm)^2 / 32 = 2.5e-18 m^2."""
    k0 = kapp.intrinsic_permeability(0.1, TORT, 40e-9)
    assert abs(k0 - 2.5e-18) < 1e-30
    k = kapp.kapp_iom(20e-9, 5e6, 400.0, 0.1, TORT, ETA)
    assert abs(k - (2.5e-18 + ETA * 4.0 / 3.0 * 0.05 * 10e-9 * vbar(400.0) / 5e6)) < 1e-30


def test_knudsen_and_langmuir_units():
    """D_K in m^2/s equals (4/3) K_c vbar; q_sat of Eq. (38) in mol/m^3."""
    dk = kapp.knudsen_diffusivity(0.1, TORT, 40e-9, 400.0)
    assert abs(dk - 4 / 3 * 5e-10 * vbar(400.0)) < 1e-22
    q = kapp.qsat_from_langmuir_volume(0.004, 0.3, 0.15)
    assert abs(q - 0.004 * 1650 / (0.7 * 0.15) * 0.7158 / 0.016043) < 1e-9


# ------------------------------------------------------- paper's claims --
def test_iom_continuum_limit_near_100nm():
    """Sec. 3.1.1: K_app approaches K_0 when the pore size approaches 100 nm."""
    for T in (300.0, 350.0, 400.0):
        r = 100e-9
        ratio = kapp.kapp_iom(r, 21e6, T, 0.04, TORT, ETA) / kapp.intrinsic_permeability(0.04, TORT, 2 * r)
        assert 1.0 < ratio < 1.1


def test_iom_knudsen_falls_with_pressure():
    """Sec. 3.1.1 (Fig. 6): K_0 does not change with pressure; the Knudsen part falls as 1/P."""
    r, T, eps = 2e-9, 350.0, 0.04
    k0 = kapp.intrinsic_permeability(eps, TORT, 2 * r)
    kn = [kapp.kapp_iom(r, P, T, eps, TORT, ETA) - k0 for P in (5e6, 10e6, 20e6)]
    assert abs(kn[0] / kn[1] - 2) < 1e-12 and abs(kn[1] / kn[2] - 2) < 1e-12


def test_om_surface_diffusion_dominates_small_pores():
    """Sec. 3.1.2 (Fig. 9): with D_s = 5e-7, q = 4000, b = 0.25 / MPa at reservoir pressure,
    K_app / K_0 of organic matter exceeds 10 for r < 2 nm."""
    for T in (300.0, 350.0, 400.0):
        for r in (1e-9, 1.5e-9, 2e-9):
            k = kapp.kapp_om(r, 21e6, T, 0.04, TORT, ETA, 4000.0, 0.25e-6, 5e-7)
            assert k / kapp.intrinsic_permeability(0.04, TORT, 2 * r) > 10


def test_om_surface_term_decreases_with_pressure():
    """Sec. 3.1.2 (Fig. 10): the surface-diffusion contribution decreases with pressure."""
    vals = []
    for P in (1e6, 5e6, 10e6, 20e6):
        vals.append(kapp.kapp_om(2e-9, P, 350.0, 0.04, TORT, ETA, 4000.0, 0.25e-6, 5e-7)
                    - kapp.kapp_iom(2e-9, P, 350.0, 0.04, TORT, ETA))
    assert all(a > b for a, b in zip(vals, vals[1:]))


def test_om_langmuir_dependence():
    """Sec. 3.1.2 (Fig. 11): K_app linear in q_sat and increasing with b."""
    r, P, T = 11e-9, 21e6, 350.0
    ks = [kapp.kapp_om(r, P, T, 0.04, TORT, ETA, q, 0.25e-6, 5e-7) for q in (1000, 2000, 3000, 4000)]
    d = np.diff(ks)
    assert np.abs(d - d[0]).max() < 1e-12 * abs(d[0])
    kb = [kapp.kapp_om(r, P, T, 0.04, TORT, ETA, 4000, b, 5e-7) for b in (0.125e-6, 0.25e-6, 0.5e-6, 1e-6)]
    assert all(a < b for a, b in zip(kb, kb[1:]))


# ---------------------------------------------- product vs oracle (host) --
@pytest.mark.parametrize("which", ["shale128", "shale4096", "batch", "shale3d"])
def test_native_class_table_matches_oracle(which):
    import paper_1601_00704_amd.glbm as g
    inst = {"shale128": si.shale128(), "shale4096": si.shale4096(64), "batch": si.batch_instance(17, side=64),
            "shale3d": si.shale3d(16)}[which]
    r_iom, r_om = inst.radii()
    eps, k = g.glbm_class_table(g.gas_params(inst), r_iom, r_om)
    e_o, k_o, _ = kapp.class_table(inst)
    assert np.array_equal(eps, e_o)
    fin = np.isfinite(k_o)
    assert np.array_equal(np.isfinite(k), fin)
    assert np.abs(k[fin] - k_o[fin]).max() / np.abs(k_o[fin]).max() < 1e-14
    assert np.all(np.abs(k[fin] - k_o[fin]) / k_o[fin] < 1e-14)


def test_native_class_table_rejects_bad_input():
    import paper_1601_00704_amd.glbm as g
    inst = si.shale128()
    p = g.gas_params(inst)
    p.pressure = -1.0
    with pytest.raises(g.GlbmError):
        g.glbm_class_table(p, *inst.radii())
    p = g.gas_params(inst)
    p.q_sat = 0.0
    p.langmuir_vl = 0.0
    with pytest.raises(g.GlbmError):
        g.glbm_class_table(p, *inst.radii())


def test_methane_reference_density_is_ideal_gas_at_standard_conditions():
    """Reading R14 of Eq. (38): rho_CH4 is methane at 273.15 K and 101.325 kPa as an
    ideal gas, P M / (R T) = 0.71576 kg/m^3; the constant keeps four digits."""
    rho = 101325.0 * kapp.M_CH4 / (kapp.R_GAS * 273.15)
    assert abs(rho - 0.715759) < 1e-6
    assert abs(kapp.RHO_CH4_STD - rho) / rho < 1e-4


def test_langmuir_capacity_range_over_the_batch_draws():
    """Eq. (38) over the batch's ranges (V_L 0.002-0.008 m^3/kg, TOC 0.05-0.30,
    eps_OM 0.3) gives a few hundred to tens of thousands of mol/m^3, bracketing the
    1000-8000 mol/m^3 the paper quotes next to Eq. (38) for its own data.  A unit slip
    (litres, MPa, or mass instead of volume) moves it by three orders of magnitude."""
    q = [kapp.qsat_from_langmuir_volume(vl, 0.3, toc) for vl in (0.002, 0.008) for toc in (0.05, 0.30)]
    assert 500 < min(q) < 1000 and 8000 < max(q) < 20000



@pytest.mark.parametrize("v_l,eps,toc", [(0.004, 0.3, 0.15), (0.002, 0.2, 0.05), (0.008, 0.45, 0.30),
                                         (0.0035, 0.1, 0.9)])
def test_langmuir_capacity_mole_balance(v_l, eps, toc):
    """Eq. (38) against the definitions the paper gives beside it, worked out as a mole
    balance over a bulk sample rather than through the formula: q_sat,b is the methane
    volume (at the reference state) adsorbed per kilogram of bulk sample, TOC the
    kerogen's volume fraction of the bulk, eps the kerogen's porosity, and q_sat,k the
    moles of methane per cubic metre of kerogen skeleton.  Moles come from the ideal-gas
    law at 273.15 K and 101.325 kPa (not from a density constant); the bulk density is
    the 1650 kg/m^3 quoted with Eq. (38).  The tolerance covers the four-digit
    methane density at the reference state.  A dropped (1 - eps), TOC on the wrong side
    or a mass in place of a volume fails by far more."""
    m_bulk = 3.7                          # kg of sample
    v_bulk = m_bulk / 1650.0              # m^3 of sample
    v_kerogen = toc * v_bulk              # m^3 of kerogen (pores included)
    v_skeleton = (1.0 - eps) * v_kerogen  # m^3 of kerogen skeleton
    v_gas = v_l * m_bulk                  # m^3 of methane at the reference state
    moles = 101325.0 * v_gas / (8.314462618 * 273.15)
    want = moles / v_skeleton
    got = kapp.qsat_from_langmuir_volume(v_l, eps, toc)
    assert abs(got - want) <= 1e-4 * want, (got, want)


def test_native_pressure_coefficients_match_oracle():
    """glbm_class_table_pressure (native) against the oracle's K(P) coefficients of
    Eq. (18)-(19), class by class, and K(P) at the instance pressure equals the constant
    class table of the same classes."""
    import paper_1601_00704_amd.glbm as g
    import shale_inputs as si
    inst = si.batch_instance(7)
    prm = g.gas_params(inst)
    r_iom, r_om = inst.radii()
    eps, kc, kk, ks, b = g.glbm_class_table_pressure(prm, r_iom, r_om)
    eps0, k0 = g.glbm_class_table(prm, r_iom, r_om)
    q_sat = kapp.qsat_from_langmuir_volume(inst.langmuir_vl, inst.eps_om, inst.toc)
    dx2 = inst.dx ** 2
    for lo, radii, ep, qs in ((1, r_iom, inst.eps_iom, 0.0), (128, r_om, inst.eps_om, q_sat)):
        A, B, C = kapp.pressure_coefficients(radii, inst.temperature, ep, inst.tortuosity, inst.viscosity, qs,
                                             1.0 / inst.langmuir_pl, inst.d_s)
        sl = slice(lo, lo + len(radii))
        assert np.allclose(kc[sl], A / dx2, rtol=1e-14, atol=0)
        assert np.allclose(kk[sl], B / dx2, rtol=1e-14, atol=0)
        assert np.allclose(ks[sl], C / dx2, rtol=1e-13, atol=0)
        assert np.all(eps[sl] == ep)
    P = inst.pressure
    kp = kc + (kk + ks / (1 + b * P)) / P
    m = np.isfinite(k0)
    assert np.allclose(kp[m], k0[m], rtol=1e-13, atol=0)
    assert np.all(np.isinf(kc[~m]))


def test_native_radius_bins_match_scipy_quantiles():
    """glbm_radius_bins (bisection on erfc) equals the equal-probability lognormal bins
    built from SciPy's normal quantile (the input generator's radius_bins)."""
    import paper_1601_00704_amd.glbm as g
    import shale_inputs as si
    for med, sig in ((20e-9, 0.5), (5e-9, 0.25), (1e-7, 1.0)):
        got = g.glbm_radius_bins(np.log(med), sig)
        want = si.radius_bins(med, sig)
        assert np.allclose(got, want, rtol=1e-13, atol=0)
    with pytest.raises(g.GlbmError):
        g.glbm_radius_bins(0.0, 0.0)
