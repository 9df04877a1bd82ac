// thermo_host.cpp -- host-side thermodynamics of the problem statement (Sec. 3.1):
// critical temperature from the printed a(Tc, Pc), b(Tc, Pc) relations, alpha(T),
// the equation of state, the Maxwell equal-area coexistence (eq Maxwell_equal_area)
// and the capillary coefficient giving a flat interface of width W (eq interface_W)
// from the second-gradient profile (kappa/2) rho'^2 = Omega(rho) - Omega_sat.
//
// Quadrature: composite 16-point Gauss-Legendre in s = ln(rho); roots by bisection.
#include <math.h>

#include <vector>

#include "thermo_host.hpp"

namespace lbm {

double critical_temperature(int eos, double a, double b, double R) {
    switch (eos) {
    case 0: return 8.0 * a / (27.0 * b * R);           // vdW: a = 27 R^2 Tc^2/(64 Pc), b = R Tc/(8 Pc)
    case 1: return 0.0778 * a / (0.45724 * b * R);     // PR
    case 2: return 0.08664 * a / (0.42748 * b * R);    // RKS
    case 3: return 0.18727 * a / (0.4963 * b * R);     // CS
    default: return 1.0 / 3.0;                         // ideal gas, Shan-Chen: no temperature scale
    }
}

// Shan-Chen critical couplings (sound-speed appendix): P = rho/3 + (G/6) psi^2 has
// dP = d2P = 0 at exp(-rho) = 1/2, G = -4 for psi = 1 - exp(-rho) and at rho = 1,
// G = -e^2 for psi = exp(-1/rho)
static double sc_critical_coupling(int eos) { return eos == 5 ? -4.0 : -exp(2.0); }

double alpha_of(int eos, double acentric, double T_reduced) {
    double m;
    if (eos == 1) m = 0.37464 + 1.54226 * acentric - 0.26992 * acentric * acentric;
    else if (eos == 2) m = 0.480 + 1.574 * acentric - 0.176 * acentric * acentric;
    else return 1.0;
    double s = 1.0 + m * (1.0 - sqrt(T_reduced));
    return s * s;
}

HostEos::HostEos(int eos_, double a_, double b_, double R_, double acentric, double T_reduced)
    : eos(eos_), a(a_), b(b_), R(R_) {
    T = T_reduced * critical_temperature(eos, a, b, R);
    aa = (eos == 5 || eos == 6) ? sc_critical_coupling(eos) / T_reduced : a * alpha_of(eos, acentric, T_reduced);
}

double HostEos::P(double r) const {
    double RT = R * T;
    switch (eos) {
    case 0: return r * RT / (1.0 - b * r) - aa * r * r;
    case 1: return r * RT / (1.0 - b * r) - aa * r * r / (1.0 + 2.0 * b * r - b * b * r * r);
    case 2: return r * RT / (1.0 - b * r) - aa * r * r / (1.0 + b * r);
    case 3: {
        double e = 0.25 * b * r, m = 1.0 - e;
        return r * RT * (1.0 + e + e * e - e * e * e) / (m * m * m) - aa * r * r;
    }
    case 5: {
        double s = 1.0 - exp(-r);
        return r / 3.0 + aa / 6.0 * s * s;
    }
    case 6: return r / 3.0 + aa / 6.0 * exp(-2.0 / r);
    default: return r / 3.0;
    }
}

double HostEos::dP(double r) const {
    // dP/drho term by term: repulsive part rho RT/(1 - b rho) (or the CS form) and attraction
    double RT = R * T;
    switch (eos) {
    case 0: return RT / ((1.0 - b * r) * (1.0 - b * r)) - 2.0 * aa * r;
    case 1: {
        double q = 1.0 + 2.0 * b * r - b * b * r * r, dq = 2.0 * b - 2.0 * b * b * r;
        return RT / ((1.0 - b * r) * (1.0 - b * r)) - aa * (2.0 * r * q - r * r * dq) / (q * q);
    }
    case 2: {
        double q = 1.0 + b * r;
        return RT / ((1.0 - b * r) * (1.0 - b * r)) - aa * (2.0 * r * q - r * r * b) / (q * q);
    }
    case 3: {
        // Z(e) = (1 + e + e^2 - e^3)/(1 - e)^3 with e = b rho/4; d(rho Z)/drho = Z + e Z'(e)
        double e = 0.25 * b * r, m = 1.0 - e;
        double num = 1.0 + e + e * e - e * e * e, dnum = 1.0 + 2.0 * e - 3.0 * e * e;
        double Z = num / (m * m * m), dZ = dnum / (m * m * m) + 3.0 * num / (m * m * m * m);
        return RT * (Z + e * dZ) - 2.0 * aa * r;
    }
    case 5: return 1.0 / 3.0 + aa / 3.0 * (1.0 - exp(-r)) * exp(-r);        // psi psi', psi' = exp(-rho)
    case 6: return 1.0 / 3.0 + aa / 3.0 * exp(-2.0 / r) / (r * r);          // psi' = exp(-1/rho)/rho^2
    default: return 1.0 / 3.0;
    }
}

double HostEos::rho_max() const {
    if (eos == 0 || eos == 1 || eos == 2) return 1.0 / b;
    if (eos == 3) return 4.0 / b;
    if (eos == 5 || eos == 6) return 50.0;   // no repulsive pole: upper end of the density search
    return INFINITY;
}

namespace {

struct Gauss {
    double x[16], w[16];
    Gauss() {
        const int n = 16;
        for (int i = 0; i < n; ++i) {
            double z = cos(M_PI * (i + 0.75) / (n + 0.5));
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                double dp = n * (z * p1 - p0) / (z * z - 1.0);
                double dz = p1 / dp;
                z -= dz;
                if (fabs(dz) < 1e-16) break;
            }
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = n * (z * p1 - p0) / (z * z - 1.0);
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

const Gauss &gauss() {
    static Gauss g;
    return g;
}

// integral over [lo, hi] of (P(rho) - p)/rho^2 d rho, in s = ln rho, `panels` panels
double integral_P_minus(const HostEos &e, double p, double lo, double hi, int panels = 96) {
    const Gauss &G = gauss();
    double s0 = log(lo), s1 = log(hi), hw = 0.5 * (s1 - s0) / panels, acc = 0.0;
    for (int k = 0; k < panels; ++k) {
        double mid = s0 + (2 * k + 1) * hw, sub = 0.0;
        for (int q = 0; q < 16; ++q) {
            double s = mid + hw * G.x[q], r = exp(s);
            sub += G.w[q] * (e.P(r) - p) / r;
        }
        acc += sub * hw;
    }
    return acc;
}

template <class F> double bisect(F f, double lo, double hi, int iters = 400) {
    double flo = f(lo);
    for (int it = 0; it < iters; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        double fm = f(mid);
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
    }
    return 0.5 * (lo + hi);
}

}  // namespace

int coexistence(const HostEos &e, double *rv_out, double *rl_out, double *psat_out) {
    if (e.eos == 4) return -1;
    double top = e.rho_max() * (1.0 - 1e-9), bot = top * 1e-9;
    // spinodals: sign changes of dP/drho on a logarithmic scan
    std::vector<double> roots;
    const int M = 6000;
    double prev_r = bot, prev_d = e.dP(bot);
    for (int k = 1; k <= M; ++k) {
        double r = bot * pow(top / bot, double(k) / M), d = e.dP(r);
        if ((d < 0) != (prev_d < 0)) roots.push_back(bisect([&](double q) { return e.dP(q); }, prev_r, r));
        prev_r = r;
        prev_d = d;
    }
    if (roots.size() != 2) return -1;
    double sv = roots[0], sl = roots[1];
    double ptop = e.P(sv), pbot = e.P(sl) > 0 ? e.P(sl) : 0.0;
    double rmax = e.rho_max() * (1.0 - 1e-15);
    auto branch = [&](double p, double lo, double hi) { return bisect([&](double r) { return e.P(r) - p; }, lo, hi); };
    auto area = [&](double p) {
        double rv = branch(p, 1e-300, sv), rl = branch(p, sl, rmax);
        return -integral_P_minus(e, p, rv, rl);   // integral of (p - P)/rho^2
    };
    double span = ptop - pbot;
    double lo = pbot > 0 ? pbot + 1e-14 * span : ptop * 1e-30, hi = ptop - 1e-13 * span;
    if ((area(lo) < 0) == (area(hi) < 0)) return -1;
    double psat = bisect(area, lo, hi, 200);
    *rv_out = branch(psat, 1e-300, sv);
    *rl_out = branch(psat, sl, rmax);
    *psat_out = psat;
    return 0;
}

int surface_tension(const HostEos &e, double kappa, double *sigma) {
    double rv, rl, ps;
    if (coexistence(e, &rv, &rl, &ps)) return -1;
    // along the flat equilibrium profile kappa rho'^2 / 2 = Omega(rho) - Omega_sat, so
    // sigma = integral_{rho_v}^{rho_l} sqrt(2 kappa (Omega - Omega_sat)) drho; the inner
    // integral runs on from the previous node, the outer by Gauss panels in rho
    const Gauss &G = gauss();
    const int panels = 64;
    const double hw = 0.5 * (rl - rv) / panels;
    double acc = 0.0;
    for (int k = 0; k < panels; ++k) {
        const double mid = rv + (2 * k + 1) * hw;
        double sub = 0.0;
        for (int q = 0; q < 16; ++q) {
            const double r = mid + hw * G.x[q];
            const double dom = r * integral_P_minus(e, ps, rv, r, 24);
            sub += G.w[q] * sqrt(dom > 0.0 ? 2.0 * kappa * dom : 0.0);
        }
        acc += sub * hw;
    }
    *sigma = acc;
    return 0;
}

int kappa_for_width(const HostEos &e, double width, double *kappa) {
    double rv, rl, ps;
    if (coexistence(e, &rv, &rl, &ps)) return -1;
    // Omega(rho) - Omega_sat = rho * integral_{rho_v}^{rho} (P - P_sat)/s^2 ds, maximised by golden section
    auto om = [&](double r) { return r * integral_P_minus(e, ps, rv, r, 48); };
    const double g = 0.5 * (sqrt(5.0) - 1.0);
    double a = rv, b = rl, c = b - g * (b - a), d = a + g * (b - a), fc = om(c), fd = om(d);
    for (int it = 0; it < 200 && (b - a) > 1e-13 * rl; ++it) {
        if (fc > fd) { b = d; d = c; fd = fc; c = b - g * (b - a); fc = om(c); }
        else { a = c; c = d; fc = fd; d = a + g * (b - a); fd = om(d); }
    }
    double mx = om(0.5 * (a + b));
    *kappa = 2.0 * mx * (width / (rl - rv)) * (width / (rl - rv));
    return 0;
}

}  // namespace lbm
