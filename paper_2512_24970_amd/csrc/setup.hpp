// Host-side planning of the IRBSOG evaluation: SOG split (Section 2.1),
// k-space sampling tables (eq. 28), kernel coefficient blocks.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"

namespace rbsog {

struct SogSplit {
    double b = 0, s = 0, x_c = 0;
    int M = 0;
    std::vector<double> w;  // w[0..M], w[0] adjusted
};

// b = 2^(1/(2J)) for the smallest J whose eq. (5) bound is <= eps.
double sog_base(double eps, int* J);
// Smallest positive x with value and slope continuity (eqs. 8-10), s = 1.
double sog_root(double b, int M);
// Full split for the cutoff r_c = r_shell.
bool sog_split(double eps, double r_shell, SogSplit* out, std::string* err);
// Kernel coefficients: explicit narrow Gaussians + Taylor block for the wide ones.
bool sog_kernel_coef(const SogSplit& sp, int J, double r_shell, bool mixed, SogCoef* c, std::string* err);

// Importance-sampling tables of P(k) = k^2 F^(k) / S (eq. 28) as a mixture
// over (m, d) of products of 1D lattice distributions.
struct KTables {
    int nm = 0;
    std::vector<int32_t> off, len;      // [nm*3]
    std::vector<double> g0cdf, g2cdf;   // concatenated per (m, d)
    std::vector<double> comp_cdf;       // [nm*3]
    double S = 0;
};
void build_ktables(const SogSplit& sp, const double box[3], KTables* t);

// Every k != 0 whose narrowest Gaussian factor exp(-s^2 k^2/2) is >= e^-45,
// with the coefficient F^(k)/V of eq. (23).
void enumerate_modes(const SogSplit& sp, const double box[3], std::vector<int32_t>* m, std::vector<double>* coef);

// F^(k) of eq. (21).
double far_hat(const SogSplit& sp, double k);
// FP32 table of the SOG near-field kernels for the mixed form, in s = r^2
// (Section 2.4 evaluates the near field by table lookup with the table
// indexed by bits of r^2): each binade [2^(e0+b), 2^(e0+b+1)), b < nbin, is
// cut into 64 intervals, so the interval of s is given by its exponent and
// its six leading mantissa bits.  Per interval, cubic Hermite polynomials in
// t = s - s_j (ascending powers) of
//   CF(s) = s^(-3/2) - sum_m (w_m / sigma_m^2) exp(-s / (2 sigma_m^2))
//   CU(s) = s^(-1/2) - sum_m w_m exp(-s / (2 sigma_m^2))
// (pair force k_e q_i q_j CF(r^2) r_ij and energy k_e q_i q_j CU(r^2); eqs.
// 8, 14-15), coef[interval][8] = CF c0..c3, CU c0..c3.  nbin covers r_shell^2;
// no table (nbin = 0) above kMaxNearBins binades.
constexpr int kNearSub = 64;
constexpr int kMaxNearBins = 12;
struct NearTable {
    int e0 = 0, nbin = 0;
    std::vector<float> coef;
};
void build_near_table(const SogSplit& sp, double r_shell, NearTable* t);

// Terms of F^ for the device: F^(k) = sum_m c[m] exp(-s2[m] k^2 / 2) with
// c_m = (2 pi)^{3/2} w_m sigma_m^3 and s2_m = sigma_m^2, m = 0..M.
void sog_kspace_terms(const SogSplit& sp, std::vector<double>* c, std::vector<double>* s2);

}  // namespace rbsog
