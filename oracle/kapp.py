"""Apparent permeability of one pore class from the DGM + GMS relations.

TEST INFRASTRUCTURE ONLY (oracle): the product computes its class table in
its own native code; this module is the independent reference it is checked
against.

Written in the order and notation of the paper's Sec. 2.1:
    K_c  = (eps / tau_t) d_p / 4,  K_0 = K_c d_p / 8           Eq. (4)
    D_K  = (4/3) K_c sqrt(8 R T / (pi M))                       Eq. (3)
    K_app (IOM) = (eta M / rho_g) (1/(R T)) (D_K + K_0 P / eta)  Eq. (18)
    K_app (OM)  = Eq. (18) + (eta M / rho_g) (1 - eps) q_sat b D_s / (1 + b P)   Eq. (19)
    q_sat,k = q_sat,b rho_b / ((1 - eps) TOC) * rho_CH4 / M_CH4   Eq. (38)

Readings (the paper leaves them open):
    rho_g is the ideal-gas density P M / (R T);
    d_p = 2 r (r the pore radius), tau_t the tortuosity;
    rho_b = 1650 kg/m^3 (kerogen density quoted with Eq. 38);
    rho_CH4 = 0.7158 kg/m^3, methane at 273.15 K and 101.325 kPa (ideal gas),
    the reference state of a Langmuir volume in m^3/kg.
"""
from __future__ import annotations

import math

import numpy as np

R_GAS = 8.314462618       # J/(mol K)
M_CH4 = 0.016043          # kg/mol
RHO_KEROGEN = 1650.0      # kg/m^3
RHO_CH4_STD = 0.7158      # kg/m^3
DARCY_M2 = 9.869233e-13   # 1 darcy in m^2


def knudsen_coefficient(eps, tort, d_p):
    """K_c of Eq. (4)."""
    return eps / tort * d_p / 4.0


def intrinsic_permeability(eps, tort, d_p):
    """K_0 of Eq. (4): K_c = (8 / d_p) K_0."""
    return knudsen_coefficient(eps, tort, d_p) * d_p / 8.0


def knudsen_diffusivity(eps, tort, d_p, T, M=M_CH4):
    """D_K of Eq. (3)."""
    return 4.0 / 3.0 * knudsen_coefficient(eps, tort, d_p) * np.sqrt(8.0 * R_GAS * T / (math.pi * M))


def gas_density(P, T, M=M_CH4):
    return P * M / (R_GAS * T)


def kapp_iom(r, P, T, eps, tort, eta, M=M_CH4):
    """Eq. (18): K_app = (eta M / rho_g) (1 / (R T)) (D_K + K_0 P / eta)."""
    d_p = 2.0 * np.asarray(r, dtype=np.float64)
    dk = knudsen_diffusivity(eps, tort, d_p, T, M)
    k0 = intrinsic_permeability(eps, tort, d_p)
    rho_g = gas_density(P, T, M)
    return eta * M / rho_g * (1.0 / (R_GAS * T)) * (dk + k0 * P / eta)


def kapp_om(r, P, T, eps, tort, eta, q_sat, b, d_s, M=M_CH4):
    """Eq. (19): Eq. (18) plus (eta M / rho_g) (1 - eps) q_sat b D_s / (1 + b P)."""
    d_p = 2.0 * np.asarray(r, dtype=np.float64)
    dk = knudsen_diffusivity(eps, tort, d_p, T, M)
    k0 = intrinsic_permeability(eps, tort, d_p)
    rho_g = gas_density(P, T, M)
    return eta * M / rho_g * ((1.0 / (R_GAS * T)) * (dk + k0 * P / eta)
                              + (1.0 - eps) * q_sat * b * d_s / (1.0 + b * P))


def qsat_from_langmuir_volume(v_l, eps, toc):
    """Eq. (38): mol of methane per m^3 of kerogen skeleton from a volume per bulk mass."""
    return v_l * RHO_KEROGEN / ((1.0 - eps) * toc) * RHO_CH4_STD / M_CH4


def class_table(inst):
    """(eps, K_lattice, F_eps) for the 256 classes of an instance (class 255: wall, unused).

    Class 0 is open pore (eps = 1, K = +inf); 1..127 IOM radius bins and
    128..254 OM radius bins at the instance's pressure and temperature.
    K_lattice = K_app / dx^2.
    """
    from shale_inputs import radius_bins, N_BINS
    eps = np.ones(256)
    k = np.full(256, math.inf)
    fe = np.zeros(256)
    r_iom = radius_bins(inst.r_iom_median, inst.sigma_ln_r)
    r_om = radius_bins(inst.r_om_median, inst.sigma_ln_r)
    b = 1.0 / inst.langmuir_pl
    q_sat = inst.q_sat
    if q_sat is None:
        q_sat = qsat_from_langmuir_volume(inst.langmuir_vl, inst.eps_om, inst.toc)
    k_iom = kapp_iom(r_iom, inst.pressure, inst.temperature, inst.eps_iom, inst.tortuosity,
                     inst.viscosity)
    k_om = kapp_om(r_om, inst.pressure, inst.temperature, inst.eps_om, inst.tortuosity,
                   inst.viscosity, q_sat, b, inst.d_s)
    eps[1:1 + N_BINS] = inst.eps_iom
    k[1:1 + N_BINS] = k_iom / inst.dx ** 2
    eps[128:128 + N_BINS] = inst.eps_om
    k[128:128 + N_BINS] = k_om / inst.dx ** 2
    return eps, k, fe


def pressure_coefficients(r, T, eps, tort, eta, q_sat=0.0, b=0.0, d_s=0.0, M=M_CH4):
    """(A, B, C) of K_app(P) = A + B / P + C / (P (1 + b P)) in m^2 (P in Pa).

    With the ideal-gas density rho_g = P M / (R T), the prefactor eta M / (rho_g R T)
    of Eq. (18)-(19) is eta / P, so Eq. (18) is K_0 + eta D_K / P (A = K_0, B = eta D_K)
    and the surface term of Eq. (19) is eta R T (1 - eps) q_sat b D_s / (P (1 + b P))
    (C = eta R T (1 - eps) q_sat b D_s; zero for inorganic matter, q_sat = 0).
    """
    d_p = 2.0 * np.asarray(r, dtype=np.float64)
    a = intrinsic_permeability(eps, tort, d_p)
    bb = eta * knudsen_diffusivity(eps, tort, d_p, T, M)
    c = eta * R_GAS * T * (1.0 - eps) * q_sat * b * d_s
    return a, bb, c
