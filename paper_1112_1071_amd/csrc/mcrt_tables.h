// mcrt_tables.h -- FP64 host tables of libmcrt (see mcrt_tables.cpp).
#pragma once

#include <vector>

#include "mcrt_internal.h"

namespace mcrt {

double planck_x_integral(double a, double b);
double planck_bin(double nu_lo, double nu_hi, double T);
void blackbody_bins(const std::vector<double>& nu, double T, std::vector<double>& out);
bool cumulative(const std::vector<double>& v, std::vector<double>& cdf);
double row_temperature(int m);
void emission_rows(const std::vector<double>& nu, const std::vector<double>& kappa,
                   std::vector<double>& ecdf);
void adot_of_T(const std::vector<double>& nu, const std::vector<double>& kappa, double T,
               double* adot, double* dlnA_dlnT);
void tsolve_table(const std::vector<double>& nu, const std::vector<double>& kappa,
                  std::vector<double>& lnA, std::vector<double>& slope, double* dy);
// raytracing: ln B_k(T) and d ln B_k / d ln T per bin on kRayTRows rows of ln T
// over [kTLo, kTHi], interleaved per (row, bin); underflowing bins hold kLnBFloor
void planck_ln_table(const std::vector<double>& nu, std::vector<double>& tab);
// modified random walk: the inverse of the first-passage distribution F of
// diffusion from the centre of a sphere, y(w) and dy/dw at kMrwYRows points of
// w = ln(u / (1 - u)) over [kMrwW0, kMrwW1], interleaved
void mrw_escape_table(std::vector<double>& tab);
// modified random walk: Planck-mean kappa and Rosseland-mean chi against ln T
void mrw_table(const std::vector<double>& nu, const std::vector<double>& kappa,
               const std::vector<double>& chi, std::vector<double>& tab);

}  // namespace mcrt
