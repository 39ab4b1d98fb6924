// Host-side planning: SOG split, sampling tables, kernel coefficients.
#include "setup.hpp"

#include <algorithm>
#include <cmath>

namespace rbsog {

namespace {

// Eq. (5): |1 - r BSA(r)| <~ 2 sqrt(2) exp(-pi^2 / (2 ln b)).
double bsa_error_bound(double b) { return 2.0 * std::sqrt(2.0) * std::exp(-kPi * kPi / (2.0 * std::log(b))); }

// BSA weight of Gaussian m in units s = 1 (eq. 7).
double weight_s1(double b, int m) { return std::sqrt(2.0) * std::log(b) / (std::sqrt(kPi) * std::pow(b, (double)m)); }

// Slope condition after the value condition fixed w_0:
// 1/x^2 - 1 + x sum_{m=1..M} v_m exp(-x^2/(2 b^{2m})) (1 - b^{-2m}).
double slope_gap(double b, int M, double x)
{
    double sum = 0.0;
    for (int m = 1; m <= M; ++m) {
        const double b2m = std::pow(b, 2.0 * m);
        sum += weight_s1(b, m) * std::exp(-x * x / (2.0 * b2m)) * (1.0 - 1.0 / b2m);
    }
    return 1.0 / (x * x) - 1.0 + x * sum;
}

}  // namespace

double sog_base(double eps, int* J)
{
    for (int j = 1; j < 64; ++j) {
        const double b = std::pow(2.0, 1.0 / (2.0 * j));
        if (bsa_error_bound(b) <= eps) {
            if (J) *J = j;
            return b;
        }
    }
    if (J) *J = 64;
    return std::pow(2.0, 1.0 / 128.0);
}

double sog_root(double b, int M)
{
    // bracket the first sign change on a 1e-3 grid from x = 0.5, then bisect
    double xa = 0.5;
    double ha = slope_gap(b, M, xa);
    for (double xb = xa + 1e-3; xb < 50.0; xb += 1e-3) {
        const double hb = slope_gap(b, M, xb);
        if ((ha > 0.0) != (hb > 0.0)) {
            double lo = xa, hi = xb;
            const bool lo_pos = ha > 0.0;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (!(mid > lo && mid < hi)) break;
                if ((slope_gap(b, M, mid) > 0.0) == lo_pos)
                    lo = mid;
                else
                    hi = mid;
            }
            return 0.5 * (lo + hi);
        }
        xa = xb;
        ha = hb;
    }
    return -1.0;
}

bool sog_split(double eps, double r_shell, SogSplit* out, std::string* err)
{
    if (!(eps > 0.0)) eps = 1e-5;
    int J = 0;
    const double b = sog_base(eps, &J);
    const double x_inf = sog_root(b, 400);
    if (x_inf <= 0.0) {
        *err = "SOG: no cutoff root";
        return false;
    }
    // series length: sum_{m>M} w_m * r_c <= 1e-3 eps
    int M = -1;
    for (int m = 1; m <= kMaxSog; ++m) {
        const double tail = std::sqrt(2.0) * std::log(b) / std::sqrt(kPi) * x_inf * std::pow(b, -(double)(m + 1)) /
                            (1.0 - 1.0 / b);
        if (tail <= 1e-3 * eps) {
            M = m;
            break;
        }
    }
    if (M < 0) {
        *err = "SOG: series too long";
        return false;
    }
    const double xc = sog_root(b, M);
    if (xc <= 0.0) {
        *err = "SOG: no cutoff root";
        return false;
    }
    const double s = r_shell / xc;
    double rest = 0.0;
    for (int m = 1; m <= M; ++m) rest += weight_s1(b, m) * std::exp(-xc * xc / (2.0 * std::pow(b, 2.0 * m)));
    const double w0 = std::exp(xc * xc / 2.0) * (1.0 / xc - rest);
    out->b = b;
    out->s = s;
    out->x_c = xc;
    out->M = M;
    out->w.assign(M + 1, 0.0);
    out->w[0] = w0 / s;
    for (int m = 1; m <= M; ++m) out->w[m] = weight_s1(b, m) / s;
    return true;
}

bool sog_kernel_coef(const SogSplit& sp, int J, double r_shell, bool mixed, SogCoef* c, std::string* err)
{
    *c = SogCoef{};
    if (J < 1 || J > 2) {
        *err = "SOG: base b must be 2^(1/2) or 2^(1/4) (sog_eps >= ~1e-12)";
        return false;
    }
    // explicit Gaussians while sigma_m < 1.5 r_shell; the rest as a series in r^2
    int n_exp = 0;
    while (n_exp <= sp.M && sp.s * std::pow(sp.b, (double)n_exp) < 1.5 * r_shell) ++n_exp;
    if (n_exp < J) n_exp = std::min(J, sp.M + 1);
    if (n_exp > kMaxExplicit) {
        *err = "SOG: too many explicit Gaussians";
        return false;
    }
    c->n_exp = n_exp;
    c->chain = J;
    for (int m = 0; m < n_exp; ++m) {
        const double sg = sp.s * std::pow(sp.b, (double)m);
        c->a[m] = 1.0 / (2.0 * sg * sg);
        c->fw[m] = sp.w[m] / (sg * sg);
        c->ew[m] = sp.w[m];
    }
    if (n_exp > sp.M) {
        c->n_poly = 0;
        return true;
    }
    // Taylor terms: |x|^n/n! with x = r_shell^2 a_{n_exp} below 1e-17 (FP64) or 1e-9 (FP32)
    const double sg0 = sp.s * std::pow(sp.b, (double)n_exp);
    const double xmax = r_shell * r_shell / (2.0 * sg0 * sg0);
    const double tol = mixed ? 1e-9 : 1e-17;
    int T = 1;
    double term = 1.0;
    while (T < kMaxPoly) {
        term *= xmax / T;
        if (term < tol) break;
        ++T;
    }
    c->n_poly = T;
    for (int n = 0; n < T; ++n) {
        double fsum = 0.0, esum = 0.0;
        for (int m = sp.M; m >= n_exp; --m) {  // small terms first
            const double sg = sp.s * std::pow(sp.b, (double)m);
            const double a = 1.0 / (2.0 * sg * sg);
            double f = 1.0;
            for (int k = 1; k <= n; ++k) f *= -a / k;
            fsum += sp.w[m] / (sg * sg) * f;
            esum += sp.w[m] * f;
        }
        c->pc[n] = fsum;
        c->pd[n] = esum;
    }
    return true;
}

void build_ktables(const SogSplit& sp, const double box[3], KTables* t)
{
    const int nm = sp.M + 1;
    t->nm = nm;
    t->off.assign(nm * 3, 0);
    t->len.assign(nm * 3, 0);
    int64_t total = 0;
    for (int m = 0; m < nm; ++m) {
        const double sigma = sp.s * std::pow(sp.b, (double)m);
        for (int d = 0; d < 3; ++d) {
            const double kd = 2.0 * kPi / box[d];
            const int nmax = (int)std::floor(std::sqrt(1380.0) / (sigma * kd));
            t->off[m * 3 + d] = (int32_t)total;
            t->len[m * 3 + d] = nmax + 1;
            total += nmax + 1;
        }
    }
    t->g0cdf.assign(total, 0.0);
    t->g2cdf.assign(total, 0.0);
    std::vector<double> G0(nm * 3), G2(nm * 3);
    for (int m = 0; m < nm; ++m) {
        const double sigma = sp.s * std::pow(sp.b, (double)m);
        for (int d = 0; d < 3; ++d) {
            const double kd = 2.0 * kPi / box[d];
            double* c0 = t->g0cdf.data() + t->off[m * 3 + d];
            double* c2 = t->g2cdf.data() + t->off[m * 3 + d];
            const int L = t->len[m * 3 + d];
            double run0 = 0.0, run2 = 0.0;
            for (int n = 0; n < L; ++n) {
                const double k = (double)n * kd;
                const double a = sigma * k;
                const double g = std::exp(-0.5 * a * a);
                run0 += (n == 0 ? 1.0 : 2.0) * g;
                run2 += (n == 0 ? 0.0 : 2.0 * k * k * g);
                c0[n] = run0;
                c2[n] = run2;
            }
            for (int n = 0; n < L; ++n) {
                c0[n] = c0[n] / run0;
                c2[n] = run2 > 0.0 ? c2[n] / run2 : 0.0;
            }
            G0[m * 3 + d] = run0;
            G2[m * 3 + d] = run2;
        }
    }
    t->comp_cdf.assign(nm * 3, 0.0);
    double run = 0.0;
    for (int m = 0; m < nm; ++m) {
        const double sigma = sp.s * std::pow(sp.b, (double)m);
        const double cm = std::pow(2.0 * kPi, 1.5) * sp.w[m] * sigma * sigma * sigma;
        for (int d = 0; d < 3; ++d) {
            double z = cm * G2[m * 3 + d];
            for (int e = 0; e < 3; ++e)
                if (e != d) z *= G0[m * 3 + e];
            run += z;
            t->comp_cdf[m * 3 + d] = run;
        }
    }
    for (auto& v : t->comp_cdf) v /= run;
    t->S = run;
}

double far_hat(const SogSplit& sp, double k)
{
    double acc = 0.0;
    for (int m = 0; m <= sp.M; ++m) {
        const double sg = sp.s * std::pow(sp.b, (double)m);
        acc += std::pow(2.0 * kPi, 1.5) * sp.w[m] * sg * sg * sg * std::exp(-sg * sg * k * k / 2.0);
    }
    return acc;
}

void build_near_table(const SogSplit& sp, double r_shell, NearTable* t)
{
    t->e0 = 0;
    t->nbin = 0;
    t->coef.clear();
    const double rs2 = r_shell * r_shell;
    int nb = 1;
    while (std::ldexp(1.0, t->e0 + nb) <= rs2) ++nb;
    if (nb > kMaxNearBins) return;
    t->nbin = nb;
    std::vector<double> a(sp.M + 1), fw(sp.M + 1);
    for (int m = 0; m <= sp.M; ++m) {
        const double sg = sp.s * std::pow(sp.b, (double)m);
        a[m] = 1.0 / (2.0 * sg * sg);
        fw[m] = sp.w[m] / (sg * sg);
    }
    // value and s-derivative of CF and CU
    auto eval = [&](double s, double* cf, double* dcf, double* cu, double* dcu) {
        double gf = 0.0, dgf = 0.0, gu = 0.0, dgu = 0.0;
        for (int m = 0; m <= sp.M; ++m) {
            const double e = std::exp(-a[m] * s);
            gf += fw[m] * e;
            dgf -= fw[m] * a[m] * e;
            gu += sp.w[m] * e;
            dgu -= sp.w[m] * a[m] * e;
        }
        const double is = 1.0 / s, rs = std::sqrt(is);
        *cf = is * rs - gf;
        *dcf = -1.5 * is * is * rs - dgf;
        *cu = rs - gu;
        *dcu = -0.5 * is * rs - dgu;
    };
    t->coef.assign((size_t)nb * kNearSub * 8, 0.0f);
    for (int b = 0; b < nb; ++b)
        for (int j = 0; j < kNearSub; ++j) {
            const double s0 = std::ldexp(1.0 + (double)j / kNearSub, t->e0 + b);
            const double s1 = std::ldexp(1.0 + (double)(j + 1) / kNearSub, t->e0 + b);
            const double h = s1 - s0;
            double f0[2], d0[2], f1[2], d1[2];
            eval(s0, &f0[0], &d0[0], &f0[1], &d0[1]);
            eval(s1, &f1[0], &d1[0], &f1[1], &d1[1]);
            float* o = t->coef.data() + ((size_t)b * kNearSub + j) * 8;
            for (int q = 0; q < 2; ++q) {
                // cubic Hermite: value and slope at both ends
                const double c2 = (3.0 * (f1[q] - f0[q]) / h - 2.0 * d0[q] - d1[q]) / h;
                const double c3 = (2.0 * (f0[q] - f1[q]) / h + d0[q] + d1[q]) / (h * h);
                o[4 * q + 0] = (float)f0[q];
                o[4 * q + 1] = (float)d0[q];
                o[4 * q + 2] = (float)c2;
                o[4 * q + 3] = (float)c3;
            }
        }
}

void sog_kspace_terms(const SogSplit& sp, std::vector<double>* c, std::vector<double>* s2)
{
    c->assign(sp.M + 1, 0.0);
    s2->assign(sp.M + 1, 0.0);
    for (int m = 0; m <= sp.M; ++m) {
        const double sg = sp.s * std::pow(sp.b, (double)m);
        (*c)[m] = std::pow(2.0 * kPi, 1.5) * sp.w[m] * sg * sg * sg;
        (*s2)[m] = sg * sg;
    }
}

void enumerate_modes(const SogSplit& sp, const double box[3], std::vector<int32_t>* m, std::vector<double>* coef)
{
    m->clear();
    coef->clear();
    int nmax[3];
    for (int a = 0; a < 3; ++a) nmax[a] = (int)std::floor(std::sqrt(90.0) / (sp.s * 2.0 * kPi / box[a]));
    const double V = box[0] * box[1] * box[2];
    for (int x = -nmax[0]; x <= nmax[0]; ++x)
        for (int y = -nmax[1]; y <= nmax[1]; ++y)
            for (int z = -nmax[2]; z <= nmax[2]; ++z) {
                if (x == 0 && y == 0 && z == 0) continue;
                const double kx = 2.0 * kPi * x / box[0], ky = 2.0 * kPi * y / box[1], kz = 2.0 * kPi * z / box[2];
                const double k2 = kx * kx + ky * ky + kz * kz;
                if (0.5 * sp.s * sp.s * k2 > 45.0) continue;
                m->push_back(x);
                m->push_back(y);
                m->push_back(z);
                coef->push_back(far_hat(sp, std::sqrt(k2)) / V);
            }
}

}  // namespace rbsog
