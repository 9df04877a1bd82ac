// thermo_host.hpp -- host-side thermodynamics used by the runtime (Sec. 3.1).
#pragma once

namespace lbm {

double critical_temperature(int eos, double a, double b, double R);
double alpha_of(int eos, double acentric, double T_reduced);

struct HostEos {
    int eos;
    double a, b, R, T, aa;
    HostEos(int eos, double a, double b, double R, double acentric, double T_reduced);
    double P(double rho) const;
    double dP(double rho) const;
    double rho_max() const;
};

// Maxwell equal-area coexistence; returns 0 or -1 (no van der Waals loop)
int coexistence(const HostEos &e, double *rho_v, double *rho_l, double *p_sat);
// kappa giving interface width W = (rho_l - rho_v)/max|rho'| for the flat profile
int kappa_for_width(const HostEos &e, double width, double *kappa);
// surface tension of the flat interface of the second-gradient fluid with capillary
// coefficient kappa: sigma = integral kappa rho'^2 dx = integral sqrt(2 kappa dOmega) drho
int surface_tension(const HostEos &e, double kappa, double *sigma);

}  // namespace lbm
