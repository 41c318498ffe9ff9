// mcrt_tables.cpp -- FP64 host tables of libmcrt, built once per model:
// bin-integrated Planck functions, source spectral and luminosity CDFs, the
// emissivity rows j_k = kappa_k B_k(T_m) of Sec. 2.1.3 (as cumulative
// distributions), and the ln Adot(ln T) table of the LTE balance of Eq. 3
// over the model's bins.
//
// The Planck integral int_a^b x^3/(e^x - 1) dx is evaluated by composite
// 16-point Gauss-Legendre quadrature on panels at most one unit wide (the
// integrand is analytic within 2 pi of the real axis, so each panel is exact
// to rounding).
#include <math.h>

#include <vector>

#include "mcrt_tables.h"

namespace mcrt {

namespace {
constexpr double kH = 6.62607015e-27;   // erg s
constexpr double kK = 1.380649e-16;     // erg / K
constexpr double kC = 2.99792458e10;    // cm / s
constexpr double kPi = 3.14159265358979323846;

struct GaussLegendre16 {
    double x[16], w[16];
    GaussLegendre16() {
        const int n = 16;
        // Newton iteration on P_16 from the usual cosine guesses; a fixed number
        // of steps (quadratic convergence reaches rounding in a handful), then
        // the weight 2 / ((1 - z^2) P'_16(z)^2) at the final node
        auto legendre = [n](double z, double* dp) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            *dp = n * (z * p0 - p1) / (z * z - 1.0);
            return p0;
        };
        for (int i = 0; i < n; ++i) {
            double z = cos(kPi * (i + 0.75) / (n + 0.5));
            for (int it = 0; it < 12; ++it) {
                double dp;
                const double p = legendre(z, &dp);
                z -= p / dp;
            }
            double dp;
            legendre(z, &dp);
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

const GaussLegendre16& gl16() {
    static const GaussLegendre16 g;
    return g;
}

inline double planck_integrand(double x) {
    if (x <= 0.0) return 0.0;
    if (x > 745.0) return 0.0;
    if (x < 1e-8) return x * x * (1.0 - 0.5 * x);
    if (x > 700.0) return x * x * x * exp(-x);  // expm1 overflows past 709.78
    return x * x * x / expm1(x);
}
}  // namespace

double planck_x_integral(double a, double b) {
    if (!(b > a)) return 0.0;
    if (a < 0.0) a = 0.0;
    if (a >= 745.0) return 0.0;
    if (b > 745.0) b = 745.0;
    const GaussLegendre16& g = gl16();
    const int panels = (int)ceil((b - a) / 1.0);
    const double h = (b - a) / panels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double c = a + (p + 0.5) * h;
        double s = 0.0;
        for (int i = 0; i < 16; ++i) s += g.w[i] * planck_integrand(c + 0.5 * h * g.x[i]);
        sum += 0.5 * h * s;
    }
    return sum;
}

// integral of B_nu(T) over [nu_lo, nu_hi]
double planck_bin(double nu_lo, double nu_hi, double T) {
    if (!(T > 0.0)) return 0.0;
    const double kT = kK * T;
    const double pref = 2.0 * kT * kT * kT * kT / (kH * kH * kH * kC * kC);
    return pref * planck_x_integral(kH * nu_lo / kT, kH * nu_hi / kT);
}

void blackbody_bins(const std::vector<double>& nu, double T, std::vector<double>& out) {
    const size_t nb = nu.size() - 1;
    out.resize(nb);
    for (size_t k = 0; k < nb; ++k) out[k] = planck_bin(nu[k], nu[k + 1], T);
}

bool cumulative(const std::vector<double>& v, std::vector<double>& cdf) {
    cdf.resize(v.size());
    double s = 0.0;
    for (size_t k = 0; k < v.size(); ++k) {
        s += v[k];
        cdf[k] = s;
    }
    if (!(s > 0.0)) {
        for (size_t k = 0; k < v.size(); ++k) cdf[k] = (double)(k + 1) / v.size();
        return false;
    }
    for (size_t k = 0; k < v.size(); ++k) cdf[k] /= s;
    cdf.back() = 1.0;
    return true;
}

double row_temperature(int m) {
    return exp(log(kTLo) + m * (log(kTHi) - log(kTLo)) / (kRows - 1));
}

void emission_rows(const std::vector<double>& nu, const std::vector<double>& kappa,
                   std::vector<double>& ecdf) {
    const size_t nb = kappa.size();
    ecdf.assign((size_t)kRows * nb, 0.0);
    std::vector<double> b, row(nb), c;
    for (int m = 0; m < kRows; ++m) {
        blackbody_bins(nu, row_temperature(m), b);
        for (size_t k = 0; k < nb; ++k) row[k] = kappa[k] * b[k];
        cumulative(row, c);
        for (size_t k = 0; k < nb; ++k) ecdf[(size_t)m * nb + k] = c[k];
    }
}

// Adot(T) = 4 pi sum_k kappa_k B_k(T) and dlnAdot/dlnT, where
// T dB_k/dT = pref [4 I_k + a f(a) - b f(b)], f(x) = x^3/(e^x - 1), x = h nu/kT.
void adot_of_T(const std::vector<double>& nu, const std::vector<double>& kappa, double T,
               double* adot, double* dlnA_dlnT) {
    const double kT = kK * T;
    const double pref = 2.0 * kT * kT * kT * kT / (kH * kH * kH * kC * kC);
    double s = 0.0, ds = 0.0;
    for (size_t k = 0; k < kappa.size(); ++k) {
        if (kappa[k] == 0.0) continue;
        const double a = kH * nu[k] / kT, b = kH * nu[k + 1] / kT;
        const double I = planck_x_integral(a, b);
        s += kappa[k] * I;
        ds += kappa[k] * (4.0 * I + a * planck_integrand(a) - b * planck_integrand(b));
    }
    *adot = 4.0 * kPi * pref * s;
    *dlnA_dlnT = s > 0.0 ? ds / s : 4.0;
}

// F(y) = 1 + 2 sum_{n>=1} (-1)^n exp(-n^2 y), the probability that diffusion
// from the centre of a sphere has reached its surface by the scaled time y,
// its complement G = 1 - F without cancellation, and dF/dy; for y < 2 the
// same functions after Jacobi's transformation,
// F = 2 sqrt(pi / y) sum_{m>=0} exp(-a_m^2 / (4 y)), a_m = (2m + 1) pi.
static void escape_cdf(double y, double* F, double* G, double* dF) {
    double f = 0.0, d = 0.0;
    if (y < 2.0) {
        for (int m = 0; m < 60; ++m) {
            const double a = (2.0 * m + 1.0) * kPi, q = a * a / (4.0 * y);
            const double t = exp(-q);
            f += t;
            d += t * (q / y - 0.5 / y);
            if (t < 1e-300) break;
        }
        const double c = 2.0 * sqrt(kPi / y);
        *F = c * f;
        *G = 1.0 - *F;
        *dF = c * d;
        return;
    }
    double sg = -1.0;
    for (int n = 1; n < 60; ++n) {
        const double t = exp(-(double)n * n * y);
        f += sg * t;
        d -= sg * (double)n * n * t;
        sg = -sg;
        if (t < 1e-300) break;
    }
    *F = 1.0 + 2.0 * f;
    *G = -2.0 * f;
    *dF = 2.0 * d;
}

void mrw_escape_table(std::vector<double>& tab) {
    tab.assign((size_t)kMrwYRows * 2, 0.0);
    const double h = (kMrwW1 - kMrwW0) / (kMrwYRows - 1);
    for (int i = 0; i < kMrwYRows; ++i) {
        const double w = kMrwW0 + i * h;
        // u and 1 - u without cancellation
        const double u = w < 0.0 ? exp(w) / (1.0 + exp(w)) : 1.0 / (1.0 + exp(-w));
        const double v = w < 0.0 ? 1.0 / (1.0 + exp(w)) : exp(-w) / (1.0 + exp(-w));
        // F(y) = u by bisection to the last bit, in the variable that keeps
        // both tails resolved: F < 1/2 compares F with u, F > 1/2 compares
        // 1 - F with v
        double lo = 1e-3, hi = 120.0;
        for (int it = 0; it < 400; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            double F, G, dF;
            escape_cdf(mid, &F, &G, &dF);
            const bool below = u <= 0.5 ? F < u : G > v;
            if (below) lo = mid;
            else hi = mid;
        }
        const double y = 0.5 * (lo + hi);
        double F, G, dF;
        escape_cdf(y, &F, &G, &dF);
        tab[2 * (size_t)i] = y;
        tab[2 * (size_t)i + 1] = dF > 0.0 ? u * v / dF : 0.0;  // dy/dw = (du/dw) / F'(y)
    }
}

void planck_ln_table(const std::vector<double>& nu, std::vector<double>& tab) {
    const size_t nb = nu.size() - 1;
    tab.assign((size_t)kRayTRows * nb * 2, 0.0);
    const double dl = (log(kTHi) - log(kTLo)) / (kRayTRows - 1);
    for (int i = 0; i < kRayTRows; ++i) {
        const double T = exp(log(kTLo) + i * dl);
        const double kT = kK * T;
        const double pref = 2.0 * kT * kT * kT * kT / (kH * kH * kH * kC * kC);
        for (size_t k = 0; k < nb; ++k) {
            const double a = kH * nu[k] / kT, b = kH * nu[k + 1] / kT;
            const double I = planck_x_integral(a, b);
            double* e = &tab[2 * ((size_t)i * nb + k)];
            if (!(pref * I > 1e-300)) {
                e[0] = kLnBFloor;
                e[1] = 0.0;
            } else {
                // B = pref(T) I(a(T), b(T)) with pref ~ T^4 and a, b ~ 1/T
                e[0] = log(pref * I);
                e[1] = (4.0 * I + a * planck_integrand(a) - b * planck_integrand(b)) / I;
            }
        }
    }
}

void tsolve_table(const std::vector<double>& nu, const std::vector<double>& kappa,
                  std::vector<double>& lnA, std::vector<double>& slope, double* dy) {
    lnA.resize(kTSolveRows);
    slope.resize(kTSolveRows);
    *dy = (log(kTHi) - log(kTLo)) / (kTSolveRows - 1);
    for (int i = 0; i < kTSolveRows; ++i) {
        const double T = exp(log(kTLo) + i * *dy);
        double a, s;
        adot_of_T(nu, kappa, T, &a, &s);
        lnA[i] = log(a);
        slope[i] = s;
    }
}

}  // namespace mcrt

namespace mcrt {
namespace {

// x^4 e^x / (e^x - 1)^2, the integrand of dB_nu/dT in x = h nu / kT
inline double dplanck_integrand(double x) {
    if (x <= 0.0 || x > 745.0) return 0.0;
    if (x < 1e-8) return x * x;
    const double e = exp(-x), d = -expm1(-x);
    return x * x * x * x * e / (d * d);
}

double dplanck_x_integral(double a, double b) {
    if (!(b > a)) return 0.0;
    if (a < 0.0) a = 0.0;
    if (a >= 745.0) return 0.0;
    if (b > 745.0) b = 745.0;
    const GaussLegendre16& g = gl16();
    const int panels = (int)ceil((b - a) / 1.0);
    const double h = (b - a) / panels;
    double sum = 0.0;
    for (int p = 0; p < panels; ++p) {
        const double c = a + (p + 0.5) * h;
        double s = 0.0;
        for (int i = 0; i < 16; ++i) s += g.w[i] * dplanck_integrand(c + 0.5 * h * g.x[i]);
        sum += 0.5 * h * s;
    }
    return sum;
}

// Planck-mean absorption and Rosseland-mean extinction at T over the bins
void mean_opacities(const std::vector<double>& nu, const std::vector<double>& kappa,
                    const std::vector<double>& chi, double T, double* kp, double* chir) {
    const double kT = kK * T;
    double nb = 0.0, db = 0.0, nr = 0.0, dr = 0.0;
    for (size_t k = 0; k < kappa.size(); ++k) {
        const double a = kH * nu[k] / kT, b = kH * nu[k + 1] / kT;
        const double B = planck_x_integral(a, b), dB = dplanck_x_integral(a, b);
        nb += kappa[k] * B;
        db += B;
        nr += dB;
        dr += dB / chi[k];
    }
    *kp = db > 0.0 ? nb / db : 0.0;
    *chir = dr > 0.0 ? nr / dr : INFINITY;
}

}  // namespace

// kMrwRows rows, log-spaced in T over [kTLo, kTHi]: kappa_P, d kappa_P / d ln T,
// chi_R, d chi_R / d ln T (central differences at +-1e-4 in ln T), for cubic
// Hermite interpolation in ln T
void mrw_table(const std::vector<double>& nu, const std::vector<double>& kappa,
               const std::vector<double>& chi, std::vector<double>& tab) {
    tab.resize((size_t)kMrwRows * 4);
    const double h = (log(kTHi) - log(kTLo)) / (kMrwRows - 1), e = 1e-4;
    for (int i = 0; i < kMrwRows; ++i) {
        const double lt = log(kTLo) + i * h;
        double kp, cr, kp1, cr1, kp0, cr0;
        mean_opacities(nu, kappa, chi, exp(lt), &kp, &cr);
        mean_opacities(nu, kappa, chi, exp(lt + e), &kp1, &cr1);
        mean_opacities(nu, kappa, chi, exp(lt - e), &kp0, &cr0);
        tab[4 * (size_t)i + 0] = kp;
        tab[4 * (size_t)i + 1] = (kp1 - kp0) / (2.0 * e);
        tab[4 * (size_t)i + 2] = cr;
        tab[4 * (size_t)i + 3] = (cr1 - cr0) / (2.0 * e);
    }
}

}  // namespace mcrt
