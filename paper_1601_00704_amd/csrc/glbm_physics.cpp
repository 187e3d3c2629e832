// Class table of a three-phase shale map: porosity and apparent permeability
// per class from the dusty-gas and generalized Maxwell-Stefan relations of
// arXiv:1601.00704, Sec. 2.1.
//
// For a pore of diameter d = 2r, porosity eps and tortuosity tau_t (Eq. 4):
//   K_c = (eps / tau_t) d / 4,   K_0 = K_c d / 8 = (eps / tau_t) d^2 / 32
// Knudsen diffusivity (Eq. 3):  D_K = (4/3) K_c sqrt(8 R T / (pi M))
// With the ideal-gas density rho_g = P M / (R T) the prefactor of Eq. (18)-(19)
// is eta M / rho_g = eta R T / P, so
//   inorganic (Eq. 18):  K_app = K_0 + eta D_K / P
//   organic   (Eq. 19):  K_app = K_0 + eta D_K / P + (eta R T / P) (1 - eps) q_sat b D_s / (1 + b P)
// q_sat from a Langmuir volume per bulk rock mass (Eq. 38):
//   q_sat = V_L rho_b / ((1 - eps) TOC) * rho_CH4 / M_CH4
// with rho_b = 1650 kg/m^3 (kerogen) and rho_CH4 = 0.7158 kg/m^3 (methane at
// 273.15 K and 101.325 kPa, the reference state of a volume in m^3/kg).
#include "glbm.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>

namespace {
constexpr double kR = 8.314462618;      // J / (mol K)
constexpr double kPi = 3.14159265358979323846;
constexpr double kRhoKerogen = 1650.0;  // kg / m^3
constexpr double kRhoMethaneStd = 0.7158;  // kg / m^3

bool positive(double v) { return v > 0.0 && std::isfinite(v); }
}  // namespace

extern "C" int glbm_class_table(const glbm_gas_params* p, int32_t n_iom, const double* r_iom, int32_t n_om,
                                const double* r_om, double* eps_out, double* k_out)
{
    if (!p || !eps_out || !k_out) return GLBM_EINVAL;
    if (n_iom < 0 || n_iom > 127 || n_om < 0 || n_om > 127) return GLBM_EINVAL;
    if ((n_iom && !r_iom) || (n_om && !r_om)) return GLBM_EINVAL;
    if (!positive(p->pressure) || !positive(p->temperature) || !positive(p->viscosity) ||
        !positive(p->molar_mass) || !positive(p->tortuosity) || !positive(p->dx))
        return GLBM_EINVAL;
    if (!(p->eps_iom > 0 && p->eps_iom <= 1) || !(p->eps_om > 0 && p->eps_om <= 1)) return GLBM_EINVAL;
    if (!(p->langmuir_b >= 0) || !(p->d_s >= 0)) return GLBM_EINVAL;
    double q_sat = p->q_sat;
    if (!(q_sat > 0)) {
        if (!positive(p->langmuir_vl) || !positive(p->toc) || p->eps_om >= 1.0) return GLBM_EINVAL;
        q_sat = p->langmuir_vl * kRhoKerogen / ((1.0 - p->eps_om) * p->toc) * kRhoMethaneStd / p->molar_mass;
    }
    const double P = p->pressure, T = p->temperature, eta = p->viscosity;
    const double vbar = std::sqrt(8.0 * kR * T / (kPi * p->molar_mass));
    const double dx2 = p->dx * p->dx;
    for (int k = 0; k < 256; ++k) {
        eps_out[k] = 1.0;
        k_out[k] = INFINITY;
    }
    auto matrix = [&](double eps, double r, bool organic) {
        const double d = 2.0 * r;
        const double kc = eps / p->tortuosity * d / 4.0;
        const double k0 = kc * d / 8.0;
        const double dk = 4.0 / 3.0 * kc * vbar;
        double kapp = k0 + eta * dk / P;
        if (organic) kapp += eta * kR * T / P * (1.0 - eps) * q_sat * p->langmuir_b * p->d_s / (1.0 + p->langmuir_b * P);
        return kapp;
    };
    for (int k = 0; k < n_iom; ++k) {
        if (!positive(r_iom[k])) return GLBM_EINVAL;
        eps_out[1 + k] = p->eps_iom;
        k_out[1 + k] = matrix(p->eps_iom, r_iom[k], false) / dx2;
    }
    for (int k = 0; k < n_om; ++k) {
        if (!positive(r_om[k])) return GLBM_EINVAL;
        eps_out[128 + k] = p->eps_om;
        k_out[128 + k] = matrix(p->eps_om, r_om[k], true) / dx2;
    }
    return GLBM_OK;
}

extern "C" int glbm_class_table_pressure(const glbm_gas_params* p, int32_t n_iom, const double* r_iom, int32_t n_om,
                                         const double* r_om, double* eps_out, double* kc_out, double* kkn_out,
                                         double* ksf_out, double* b_out)
{
    if (!p || !eps_out || !kc_out || !kkn_out || !ksf_out || !b_out) return GLBM_EINVAL;
    if (n_iom < 0 || n_iom > 127 || n_om < 0 || n_om > 127) return GLBM_EINVAL;
    if ((n_iom && !r_iom) || (n_om && !r_om)) return GLBM_EINVAL;
    if (!positive(p->temperature) || !positive(p->viscosity) || !positive(p->molar_mass) ||
        !positive(p->tortuosity) || !positive(p->dx))
        return GLBM_EINVAL;
    if (!(p->eps_iom > 0 && p->eps_iom <= 1) || !(p->eps_om > 0 && p->eps_om <= 1)) return GLBM_EINVAL;
    if (!(p->langmuir_b >= 0) || !(p->d_s >= 0)) return GLBM_EINVAL;
    double q_sat = p->q_sat;
    if (!(q_sat > 0)) {
        if (!positive(p->langmuir_vl) || !positive(p->toc) || p->eps_om >= 1.0) return GLBM_EINVAL;
        q_sat = p->langmuir_vl * kRhoKerogen / ((1.0 - p->eps_om) * p->toc) * kRhoMethaneStd / p->molar_mass;
    }
    const double T = p->temperature, eta = p->viscosity;
    const double vbar = std::sqrt(8.0 * kR * T / (kPi * p->molar_mass));
    const double dx2 = p->dx * p->dx;
    for (int k = 0; k < 256; ++k) {
        eps_out[k] = 1.0;
        kc_out[k] = INFINITY;
        kkn_out[k] = ksf_out[k] = b_out[k] = 0.0;
    }
    auto fill = [&](int k, double eps, double r, bool organic) {
        const double d = 2.0 * r;
        const double kc = eps / p->tortuosity * d / 4.0;   // Eq. (4)
        eps_out[k] = eps;
        kc_out[k] = kc * d / 8.0 / dx2;                      // K_0
        kkn_out[k] = eta * (4.0 / 3.0 * kc * vbar) / dx2;    // eta D_K, Eq. (3)
        ksf_out[k] = organic ? eta * kR * T * (1.0 - eps) * q_sat * p->langmuir_b * p->d_s / dx2 : 0.0;
        b_out[k] = organic ? p->langmuir_b : 0.0;
    };
    for (int k = 0; k < n_iom; ++k) {
        if (!positive(r_iom[k])) return GLBM_EINVAL;
        fill(1 + k, p->eps_iom, r_iom[k], false);
    }
    for (int k = 0; k < n_om; ++k) {
        if (!positive(r_om[k])) return GLBM_EINVAL;
        fill(128 + k, p->eps_om, r_om[k], true);
    }
    return GLBM_OK;
}

namespace {
// Standard normal quantile: the z with Phi(z) = p, Phi(z) = erfc(-z / sqrt 2) / 2,
// by bisection to the resolution of a double (Phi is monotone).
double normal_quantile(double p)
{
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (0.5 * std::erfc(-mid / std::sqrt(2.0)) < p) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}
}  // namespace

extern "C" int glbm_radius_bins(double mu_ln, double sigma_ln, int32_t n, double* r_out)
{
    if (!r_out || n < 1 || n > 127 || !std::isfinite(mu_ln) || !positive(sigma_ln)) return GLBM_EINVAL;
    for (int k = 0; k < n; ++k) r_out[k] = std::exp(mu_ln + sigma_ln * normal_quantile((k + 0.5) / n));
    return GLBM_OK;
}
