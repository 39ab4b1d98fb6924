/*
 * oracle.c -- plain double-precision CPU reference of the IRBSOG force
 * evaluation (arXiv:2512.24970).  TEST INFRASTRUCTURE ONLY: loaded by the test
 * suite, the smoke check and the benchmark's CPU-baseline leg, never by the
 * GPU library.  Slow and direct on purpose: brute-force neighbour search,
 * every Gaussian of the sum-of-Gaussians series evaluated with libm exp, libm
 * sin/cos for every Fourier phase, sums in the order the formulas are written.
 *
 * Where the paper is silent the readings are:
 *   - every Coulomb term carries k_e (coulomb_k);
 *   - b = 2^(1/(2j)) with j the smallest integer meeting the eq. (5) bound;
 *   - the SOG cutoff r_c is r_shell, and s = r_shell / x_c;
 *   - series length M: the smallest M whose neglected weights, times r_c, are
 *     below 1e-3 of the eq. (5) target;
 *   - shell batches are drawn without replacement (Floyd) from the stored
 *     candidate list, N_shell = candidate count, f_ij masked at the current
 *     distance; a fresh batch every force evaluation;
 *   - Fourier modes are drawn i.i.d. from P(k) of eq. (28) by an exact
 *     separable-mixture sampler instead of Metropolis-Hastings;
 *   - randomness comes from Philox4x32-10 with counter (index, eval,
 *     tag | replica << 8, block) and key = the 64-bit seed.
 *
 * Parity status: see the comment of each function in oracle.h.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
/* 1 eV/(Angstrom*amu) in Angstrom/ps^2 (CODATA 2018 e and atomic mass unit). */
#define ORC_ACC 9648.533212331

static int g_threads = 0;

void orc_set_threads(int n) { g_threads = n; }

int orc_get_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

#ifdef _OPENMP
#define ORC_NT (orc_get_threads())
#endif

/* ======================================================================
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies, the key
 * advanced by the Weyl constants between rounds.
 * ==================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* A word stream: counter (index, eval, tag | replica << 8, block), key = seed. */
typedef struct {
    uint32_t ctr[4];
    uint32_t key[2];
    uint32_t buf[4];
    int pos;
} orc_stream;

static void stream_init(orc_stream* s, uint64_t seed, uint32_t index, uint32_t eval,
                        uint32_t tag, uint32_t replica)
{
    s->key[0] = (uint32_t)(seed & 0xFFFFFFFFu);
    s->key[1] = (uint32_t)(seed >> 32);
    s->ctr[0] = index;
    s->ctr[1] = eval;
    s->ctr[2] = (tag & 0xFFu) | (replica << 8);
    s->ctr[3] = 0;
    s->pos = 4;
}

static uint32_t stream_next(orc_stream* s)
{
    if (s->pos == 4) {
        orc_philox4x32_10(s->ctr, s->key, s->buf);
        s->ctr[3] += 1u;
        s->pos = 0;
    }
    return s->buf[s->pos++];
}

void orc_stream_words(uint64_t seed, uint32_t index, uint32_t eval, uint32_t tag,
                      uint32_t replica, int n, uint32_t* out)
{
    orc_stream s;
    stream_init(&s, seed, index, eval, tag, replica);
    for (int i = 0; i < n; ++i) out[i] = stream_next(&s);
}

/* 53-bit uniform in [0,1) from two consecutive words: 27 high bits of the
 * first, 26 high bits of the second. */
static double stream_uniform(orc_stream* s)
{
    uint32_t a = stream_next(s) >> 5;
    uint32_t b = stream_next(s) >> 6;
    return ((double)a * 67108864.0 + (double)b) * (1.0 / 9007199254740992.0);
}

/* Lemire, "Fast random integer generation in an interval" (ACM TOMACS 2019):
 * x*range >> 32, rejecting low parts below 2^32 mod range. */
static uint32_t stream_bounded(orc_stream* s, uint32_t range)
{
    uint32_t x = stream_next(s);
    uint64_t m = (uint64_t)x * (uint64_t)range;
    uint32_t l = (uint32_t)m;
    if (l < range) {
        uint32_t t = (uint32_t)(0u - range) % range;
        while (l < t) {
            x = stream_next(s);
            m = (uint64_t)x * (uint64_t)range;
            l = (uint32_t)m;
        }
    }
    return (uint32_t)(m >> 32);
}

uint32_t orc_bounded_from_words(const uint32_t* words, int n_words, uint32_t range,
                                int* consumed)
{
    int k = 0;
    uint32_t x = words[k++];
    uint64_t m = (uint64_t)x * (uint64_t)range;
    uint32_t l = (uint32_t)m;
    if (l < range) {
        uint32_t t = (uint32_t)(0u - range) % range;
        while (l < t && k < n_words) {
            x = words[k++];
            m = (uint64_t)x * (uint64_t)range;
            l = (uint32_t)m;
        }
    }
    if (consumed) *consumed = k;
    return (uint32_t)(m >> 32);
}

/* ======================================================================
 * SOG decomposition (Section 2.1, eqs. 4-10).
 * ==================================================================== */

/* Eq. (5) bound as a function of b. */
static double bsa_bound(double b) { return 2.0 * sqrt(2.0) * exp(-ORC_PI * ORC_PI / (2.0 * log(b))); }

double orc_sog_b_from_eps(double eps)
{
    for (int j = 1; j < 64; ++j) {
        double b = pow(2.0, 1.0 / (2.0 * j));
        if (bsa_bound(b) <= eps) return b;
    }
    return pow(2.0, 1.0 / 128.0);
}

/* Unadjusted BSA weight in units s = 1: sqrt(2) ln b / (sqrt(pi) b^m)  (eq. 7). */
static double bsa_weight(double b, int m) { return sqrt(2.0) * log(b) / (sqrt(ORC_PI) * pow(b, (double)m)); }

/* With w_0 eliminated by the value condition x F(x) = 1, the slope condition
 * F'(x) = -1/x^2 reads h(x) = 0 with
 *   h(x) = 1/x^2 - 1 + x sum_{m>=1} v_m e^{-x^2/(2 b^{2m})} (1 - b^{-2m}). */
static double c1_residual(double b, int M, double x)
{
    double acc = 0.0;
    for (int m = 1; m <= M; ++m) {
        double b2m = pow(b, 2.0 * m);
        acc += bsa_weight(b, m) * exp(-x * x / (2.0 * b2m)) * (1.0 - 1.0 / b2m);
    }
    return 1.0 / (x * x) - 1.0 + x * acc;
}

double orc_sog_xc(double b, int M)
{
    /* scan for the first sign change, then bisect */
    const double step = 1e-3;
    double x0 = 0.5, h0 = c1_residual(b, M, x0);
    for (double x1 = x0 + step; x1 < 50.0; x1 += step) {
        double h1 = c1_residual(b, M, x1);
        if ((h0 > 0.0) != (h1 > 0.0)) {
            double lo = x0, hi = x1, hlo = h0;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double hm = c1_residual(b, M, mid);
                if ((hm > 0.0) == (hlo > 0.0)) {
                    lo = mid;
                    hlo = hm;
                } else {
                    hi = mid;
                }
            }
            return 0.5 * (lo + hi);
        }
        x0 = x1;
        h0 = h1;
    }
    return -1.0;
}

int orc_sog_setup(orc_params* p)
{
    double eps = p->sog_eps > 0.0 ? p->sog_eps : 1e-5;
    double b = orc_sog_b_from_eps(eps);
    /* series length: neglected weights sum_{m>M} w_m times r_c below 1e-3 eps */
    double xc_inf = orc_sog_xc(b, 400);
    if (xc_inf <= 0.0) return -1;
    int M = -1;
    for (int m = 1; m <= ORC_MAXM; ++m) {
        double tail = sqrt(2.0) * log(b) / sqrt(ORC_PI) * xc_inf * pow(b, -(double)(m + 1)) / (1.0 - 1.0 / b);
        if (tail <= 1e-3 * eps) {
            M = m;
            break;
        }
    }
    if (M < 0) return -2;
    double xc = orc_sog_xc(b, M);
    if (xc <= 0.0) return -3;
    double s = p->r_shell / xc;
    /* w_0 from the value condition x F(x) = 1 at x_c (units s = 1). */
    double tail = 0.0;
    for (int m = 1; m <= M; ++m) tail += bsa_weight(b, m) * exp(-xc * xc / (2.0 * pow(b, 2.0 * m)));
    double w0 = exp(xc * xc / 2.0) * (1.0 / xc - tail);
    memset(p->w, 0, sizeof(p->w));
    p->w[0] = w0 / s;
    for (int m = 1; m <= M; ++m) p->w[m] = bsa_weight(b, m) / s;
    p->b = b;
    p->s = s;
    p->M = M;
    p->x_c = xc;
    return 0;
}

static double sigma_m(const orc_params* p, int m) { return p->s * pow(p->b, (double)m); }

/* Eq. (7). */
double orc_far(const orc_params* p, double r)
{
    double acc = 0.0;
    for (int m = 0; m <= p->M; ++m) {
        double sg = sigma_m(p, m);
        acc += p->w[m] * exp(-r * r / (2.0 * sg * sg));
    }
    return acc;
}

/* Eq. (8) with r_c = r_shell. */
double orc_near(const orc_params* p, double r)
{
    if (r >= p->r_shell) return 0.0;
    return 1.0 / r - orc_far(p, r);
}

/* Eq. (21). */
double orc_far_hat(const orc_params* p, double k)
{
    double acc = 0.0;
    for (int m = 0; m <= p->M; ++m) {
        double sg = sigma_m(p, m);
        acc += pow(2.0 * ORC_PI, 1.5) * p->w[m] * sg * sg * sg * exp(-sg * sg * k * k / 2.0);
    }
    return acc;
}

double orc_far_hat_g(const orc_params* p, double k)
{
    double acc = 0.0;
    for (int m = 0; m <= p->M; ++m) {
        double sg = sigma_m(p, m);
        acc += pow(2.0 * ORC_PI, 1.5) * p->w[m] * sg * sg * sg * sg * sg * exp(-sg * sg * k * k / 2.0);
    }
    return acc;
}

/* Adds (k_e/2) e (delta_ab - g k_a k_b) to W[6] (xx, yy, zz, xy, xz, yz):
 * the strain derivative of one mode's energy (k_e/2) coef |rho|^2, with the
 * mode's k shrinking as the box grows (dk_a/de_ab = -k_b). */
static void mode_virial(double ke_half_e, double g, const double k[3], double W[6])
{
    W[0] += ke_half_e * (1.0 - g * k[0] * k[0]);
    W[1] += ke_half_e * (1.0 - g * k[1] * k[1]);
    W[2] += ke_half_e * (1.0 - g * k[2] * k[2]);
    W[3] -= ke_half_e * g * k[0] * k[1];
    W[4] -= ke_half_e * g * k[0] * k[2];
    W[5] -= ke_half_e * g * k[1] * k[2];
}

/* ======================================================================
 * Importance sampling of eq. (28): P(k) = k^2 F^(k) / S.
 *
 * k^2 F^(k) = sum_m c_m (kx^2 + ky^2 + kz^2) gx(kx) gy(ky) gz(kz) with
 * c_m = (2 pi)^{3/2} w_m sigma_m^3 and g(k) = exp(-sigma_m^2 k^2 / 2), so
 * P is a mixture over (m, d) of products of 1D lattice distributions:
 * axis d has weights k_d^2 g(k_d), the two other axes g(k).  Drawing the
 * component by its mass and then each axis independently is an exact i.i.d.
 * draw from P.  The k = 0 vector has zero mass (its k_d^2 factor).
 *
 * 1D tables run over n >= 0 (k_n = 2 pi n / L_d), n > 0 weighted twice for
 * +-n, truncated where sigma^2 k^2 / 2 > 690.  cdf[n] = (running sum in
 * ascending n) / total; a draw u picks the first n with u < cdf[n].
 * ==================================================================== */
typedef struct {
    int nm;          /* number of Gaussians M+1 */
    int* off;        /* [nm*3] offset of table (m,d) */
    int* len;        /* [nm*3] n_max+1 */
    double* g0cdf;   /* concatenated */
    double* g2cdf;
    double* comp_cdf; /* [nm*3] */
    double S;
} orc_ktab;

static void ktab_free(orc_ktab* t)
{
    free(t->off);
    free(t->len);
    free(t->g0cdf);
    free(t->g2cdf);
    free(t->comp_cdf);
    memset(t, 0, sizeof(*t));
}

static int ktab_build(const orc_params* p, orc_ktab* t)
{
    memset(t, 0, sizeof(*t));
    int nm = p->M + 1;
    t->nm = nm;
    t->off = (int*)malloc(sizeof(int) * nm * 3);
    t->len = (int*)malloc(sizeof(int) * nm * 3);
    double* G0 = (double*)malloc(sizeof(double) * nm * 3);
    double* G2 = (double*)malloc(sizeof(double) * nm * 3);
    long total = 0;
    for (int m = 0; m < nm; ++m) {
        for (int d = 0; d < 3; ++d) {
            double kd = 2.0 * ORC_PI / p->box[d];
            int nmax = (int)floor(sqrt(1380.0) / (sigma_m(p, m) * kd));
            t->off[m * 3 + d] = (int)total;
            t->len[m * 3 + d] = nmax + 1;
            total += nmax + 1;
        }
    }
    t->g0cdf = (double*)malloc(sizeof(double) * total);
    t->g2cdf = (double*)malloc(sizeof(double) * total);
    for (int m = 0; m < nm; ++m) {
        double sg = sigma_m(p, m);
        for (int d = 0; d < 3; ++d) {
            double kd = 2.0 * ORC_PI / p->box[d];
            int o = t->off[m * 3 + d], L = t->len[m * 3 + d];
            double c0 = 0.0, c2 = 0.0;
            for (int n = 0; n < L; ++n) {
                double k = (double)n * kd;
                double a = sg * k;
                double g = exp(-0.5 * a * a);
                double w0 = (n == 0 ? 1.0 : 2.0) * g;
                double w2 = (n == 0 ? 0.0 : 2.0 * k * k * g);
                c0 += w0;
                c2 += w2;
                t->g0cdf[o + n] = c0;
                t->g2cdf[o + n] = c2;
            }
            for (int n = 0; n < L; ++n) {
                t->g0cdf[o + n] = t->g0cdf[o + n] / c0;
                t->g2cdf[o + n] = c2 > 0.0 ? t->g2cdf[o + n] / c2 : 0.0;
            }
            G0[m * 3 + d] = c0;
            G2[m * 3 + d] = c2;
        }
    }
    t->comp_cdf = (double*)malloc(sizeof(double) * nm * 3);
    double cum = 0.0;
    for (int m = 0; m < nm; ++m) {
        double sg = sigma_m(p, m);
        double cm = pow(2.0 * ORC_PI, 1.5) * p->w[m] * sg * sg * sg;
        for (int d = 0; d < 3; ++d) {
            double z = cm * G2[m * 3 + d];
            for (int e = 0; e < 3; ++e)
                if (e != d) z *= G0[m * 3 + e];
            cum += z;
            t->comp_cdf[m * 3 + d] = cum;
        }
    }
    for (int c = 0; c < nm * 3; ++c) t->comp_cdf[c] /= cum;
    t->S = cum;
    free(G0);
    free(G2);
    return 0;
}

static int cdf_pick(const double* cdf, int len, double u)
{
    for (int i = 0; i < len; ++i)
        if (u < cdf[i]) return i;
    return len - 1;
}

double orc_kspace_S(const orc_params* p)
{
    orc_ktab t;
    ktab_build(p, &t);
    double S = t.S;
    ktab_free(&t);
    return S;
}

static void kmodes_from_tab(const orc_params* p, const orc_ktab* t, uint64_t eval, int32_t* m_out)
{
    for (int pidx = 0; pidx < p->p_f; ++pidx) {
        orc_stream s;
        stream_init(&s, p->seed, (uint32_t)pidx, (uint32_t)eval, ORC_TAG_KMODE, p->replica);
        double uc = stream_uniform(&s);
        double ua[3];
        for (int a = 0; a < 3; ++a) ua[a] = stream_uniform(&s);
        uint32_t signs = stream_next(&s);
        int c = cdf_pick(t->comp_cdf, t->nm * 3, uc);
        int m = c / 3, d = c % 3;
        for (int a = 0; a < 3; ++a) {
            int o = t->off[m * 3 + a], L = t->len[m * 3 + a];
            const double* cdf = (a == d) ? t->g2cdf + o : t->g0cdf + o;
            int n = cdf_pick(cdf, L, ua[a]);
            if (n > 0 && ((signs >> a) & 1u)) n = -n;
            m_out[pidx * 3 + a] = n;
        }
    }
}

int orc_kmodes(const orc_params* p, uint64_t eval, int32_t* m_out, double* S_out)
{
    orc_ktab t;
    ktab_build(p, &t);
    kmodes_from_tab(p, &t, eval, m_out);
    if (S_out) *S_out = t.S;
    ktab_free(&t);
    return 0;
}

/* ======================================================================
 * System state.
 * ==================================================================== */
struct orc_ctx {
    orc_params p;
    int32_t n;
    int32_t* type;
    double* pos;  /* [n][3] */
    double* vel;  /* [n][3] */
    double* frc;  /* [n][3] last force */
    uint64_t eval;
    uint64_t n_builds; /* list builds so far */
    double nh_x, nh_v; /* Nose-Hoover variable xi and its velocity */
    double* epot;      /* [n] per-atom potential energy of the last evaluation */
    double* wat;       /* [n][6] per-atom virial of the last evaluation */
    /* lists */
    int32_t* core_off;
    int32_t* core;
    int32_t* cand_off;
    int32_t* cand;
    double* ref;  /* [n][3] positions at the last list build */
    int nc[3];    /* cell grid that orders shell candidates */
    double cscale[3];
    orc_ktab kt;
    int have_kt;
};

/* Minimum-image displacement, with the operations in this order and no fused
 * multiply-add: d = ri - rj; d -= L * rint(d * (1/L)). */
static void min_image(const orc_params* p, const double* ri, const double* rj, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double L = p->box[a];
        double inv = 1.0 / L;
        double x = ri[a] - rj[a];
        double k = rint(x * inv);
        double Lk = L * k;
        d[a] = x - Lk;
    }
}

static double norm2(const double d[3])
{
    double xy = d[0] * d[0] + d[1] * d[1];
    return xy + d[2] * d[2];
}

static void wrap(const orc_params* p, double* x)
{
    for (int a = 0; a < 3; ++a) {
        double L = p->box[a];
        double inv = 1.0 / L;
        double f = floor(x[a] * inv);
        double v = x[a] - L * f;
        if (v >= L) v -= L;
        if (v < 0.0) v += L;
        x[a] = v;
    }
}

orc_ctx* orc_create(const orc_params* p, int32_t n, const int32_t* type,
                    const double* pos, const double* vel)
{
    orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    c->p = *p;
    c->n = n;
    c->type = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    c->pos = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    c->vel = (double*)calloc(3 * (n > 0 ? n : 1), sizeof(double));
    c->frc = (double*)calloc(3 * (n > 0 ? n : 1), sizeof(double));
    if (n > 0) {
        memcpy(c->type, type, sizeof(int32_t) * n);
        memcpy(c->pos, pos, sizeof(double) * 3 * n);
        if (vel) memcpy(c->vel, vel, sizeof(double) * 3 * n);
    }
    for (int i = 0; i < n; ++i) wrap(&c->p, c->pos + 3 * i);
    /* ordering grid: twice floor(L / (r_shell + skin)) cells per axis, so
       cells of side >= (r_shell + skin) / 2; one cell along an axis where
       floor(L / (r_shell + skin)) is below 3 */
    for (int a = 0; a < 3; ++a) {
        int nc = (int)floor(c->p.box[a] / (c->p.r_shell + c->p.skin + 1e-9));
        nc = nc < 3 ? 1 : 2 * nc;
        c->nc[a] = nc;
        c->cscale[a] = (double)nc / c->p.box[a];
    }
    return c;
}

/* Cell of a wrapped position on the ordering grid: floor(x n_c / L) per
   axis, x fastest. */
static int cell_of(const orc_ctx* c, const double* x)
{
    int cc[3];
    for (int a = 0; a < 3; ++a) {
        int v = (int)(x[a] * c->cscale[a]);
        cc[a] = v < 0 ? 0 : (v >= c->nc[a] ? c->nc[a] - 1 : v);
    }
    return (cc[2] * c->nc[1] + cc[1]) * c->nc[0] + cc[0];
}

typedef struct {
    int cell, j;
} cand_key;

static int cand_cmp(const void* a, const void* b)
{
    const cand_key* x = (const cand_key*)a;
    const cand_key* y = (const cand_key*)b;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return x->j < y->j ? -1 : (x->j > y->j ? 1 : 0);
}

void orc_destroy(orc_ctx* c)
{
    if (!c) return;
    free(c->type);
    free(c->pos);
    free(c->vel);
    free(c->frc);
    free(c->core_off);
    free(c->core);
    free(c->cand_off);
    free(c->cand);
    free(c->ref);
    free(c->epot);
    free(c->wat);
    if (c->have_kt) ktab_free(&c->kt);
    free(c);
}

/* Core radius of the species pair (a, b): its own if set, else r_core. */
static double core_radius(const orc_params* p, int a, int b)
{
    double r = p->r_core_pair[a * ORC_MAXS + b];
    return r > 0.0 ? r : p->r_core;
}

/* Core and candidate lists of atom i by a scan over every other atom.
 * Candidates are ordered by (cell of the candidate, atom index), the order
 * that shell ranks refer to. */
static void scan_atom(const orc_ctx* c, int i, int32_t* core, int* nc, int32_t* cand, int* nk, int count_only)
{
    const orc_params* p = &c->p;
    double hi = p->r_shell + p->skin;
    double hi2 = hi * hi;
    int a = 0, k = 0;
    for (int j = 0; j < c->n; ++j) {
        if (j == i) continue;
        double rcp = core_radius(p, c->type[i], c->type[j]);
        double rc = rcp + p->skin;
        double rc2 = rc * rc;
        double lo = rcp - p->skin;
        double lo2 = lo > 0.0 ? lo * lo : 0.0;
        double d[3];
        min_image(p, c->pos + 3 * i, c->pos + 3 * j, d);
        double r2 = norm2(d);
        if (r2 < rc2) {
            if (!count_only) core[a] = j;
            ++a;
        }
        if (r2 >= lo2 && r2 < hi2) {
            if (!count_only) cand[k] = j;
            ++k;
        }
    }
    *nc = a;
    *nk = k;
    if (!count_only && k > 1) {
        cand_key* key = (cand_key*)malloc(sizeof(cand_key) * k);
        for (int t = 0; t < k; ++t) {
            key[t].cell = cell_of(c, c->pos + 3 * cand[t]);
            key[t].j = cand[t];
        }
        qsort(key, k, sizeof(cand_key), cand_cmp);
        for (int t = 0; t < k; ++t) cand[t] = key[t].j;
        free(key);
    }
}

int orc_build_lists(orc_ctx* c)
{
    int n = c->n;
    free(c->core_off);
    free(c->core);
    free(c->cand_off);
    free(c->cand);
    c->core_off = (int32_t*)calloc(n + 1, sizeof(int32_t));
    c->cand_off = (int32_t*)calloc(n + 1, sizeof(int32_t));
    int32_t* nc = (int32_t*)calloc(n > 0 ? n : 1, sizeof(int32_t));
    int32_t* nk = (int32_t*)calloc(n > 0 ? n : 1, sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 16) num_threads(ORC_NT)
    for (int i = 0; i < n; ++i) {
        int a, k;
        scan_atom(c, i, NULL, &a, NULL, &k, 1);
        nc[i] = a;
        nk[i] = k;
    }
    for (int i = 0; i < n; ++i) {
        c->core_off[i + 1] = c->core_off[i] + nc[i];
        c->cand_off[i + 1] = c->cand_off[i] + nk[i];
    }
    c->core = (int32_t*)malloc(sizeof(int32_t) * (c->core_off[n] + 1));
    c->cand = (int32_t*)malloc(sizeof(int32_t) * (c->cand_off[n] + 1));
#pragma omp parallel for schedule(dynamic, 16) num_threads(ORC_NT)
    for (int i = 0; i < n; ++i) {
        int a, k;
        scan_atom(c, i, c->core + c->core_off[i], &a, c->cand + c->cand_off[i], &k, 0);
    }
    free(nc);
    free(nk);
    free(c->ref);
    c->ref = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    if (n > 0) memcpy(c->ref, c->pos, sizeof(double) * 3 * n);
    c->n_builds += 1;
    return 0;
}

int64_t orc_n_builds(const orc_ctx* c) { return (int64_t)c->n_builds; }

int orc_list_counts(const orc_ctx* c, int32_t* n_core, int32_t* n_cand)
{
    if (!c->core_off) return -1;
    for (int i = 0; i < c->n; ++i) {
        n_core[i] = c->core_off[i + 1] - c->core_off[i];
        n_cand[i] = c->cand_off[i + 1] - c->cand_off[i];
    }
    return 0;
}

int orc_list_atom(const orc_ctx* c, int32_t i, int32_t* core, int32_t* cand)
{
    if (!c->core_off || i < 0 || i >= c->n) return -1;
    memcpy(core, c->core + c->core_off[i], sizeof(int32_t) * (c->core_off[i + 1] - c->core_off[i]));
    memcpy(cand, c->cand + c->cand_off[i], sizeof(int32_t) * (c->cand_off[i + 1] - c->cand_off[i]));
    return 0;
}

/* Shell batch (eq. 25): P_R distinct ranks out of n candidates by Floyd's
 * algorithm (Bentley & Floyd, CACM 30(9), 1987): for j = n-P_R .. n-1 draw
 * t uniform in [0, j]; take t unless already taken, else take j.  Ranks are
 * returned ascending.  n <= P_R (or P_R <= 0) takes every rank.  The stream
 * is (atom, ctr1, tag): ctr1 = eval with TAG_SHELL for a fresh batch per
 * evaluation, ctr1 = build number with TAG_SHELL_BUILD for a batch kept
 * from one list build to the next. */
static int shell_ranks(const orc_params* p, uint32_t atom_index, int n, uint32_t ctr1, uint32_t tag,
                       int32_t* ranks)
{
    if (p->p_r <= 0 || n <= p->p_r) {
        for (int t = 0; t < n; ++t) ranks[t] = t;
        return n;
    }
    unsigned char* taken = (unsigned char*)calloc(n, 1);
    orc_stream s;
    stream_init(&s, p->seed, atom_index, ctr1, tag, p->replica);
    for (int j = n - p->p_r; j < n; ++j) {
        uint32_t t = stream_bounded(&s, (uint32_t)(j + 1));
        if (taken[t])
            taken[j] = 1;
        else
            taken[t] = 1;
    }
    int k = 0;
    for (int t = 0; t < n; ++t)
        if (taken[t]) ranks[k++] = t;
    free(taken);
    return k;
}

/* Stream of the shell batch used at evaluation `eval`: per evaluation, or,
 * with shell_stored, the one of the last list build (number n_builds - 1; 0
 * before any build, the number the first build will take). */
static void shell_stream(const orc_ctx* c, uint64_t eval, uint32_t* ctr1, uint32_t* tag)
{
    if (c->p.shell_stored) {
        *ctr1 = (uint32_t)(c->n_builds > 0 ? c->n_builds - 1 : 0);
        *tag = ORC_TAG_SHELL_BUILD;
    } else {
        *ctr1 = (uint32_t)eval;
        *tag = ORC_TAG_SHELL;
    }
}

int orc_scan_lists_atom(const orc_ctx* c, int32_t i, int32_t* core, int32_t* cand, int32_t* n_core, int32_t* n_cand)
{
    if (i < 0 || i >= c->n) return -1;
    int nc, nk;
    scan_atom(c, i, core, &nc, cand, &nk, core == NULL || cand == NULL);
    *n_core = nc;
    *n_cand = nk;
    return 0;
}

int orc_shell_ranks_count(const orc_ctx* c, int32_t i, int32_t n, uint64_t eval, int32_t* ranks)
{
    if (i < 0 || i >= c->n || n < 0) return -1;
    uint32_t ctr1, tag;
    shell_stream(c, eval, &ctr1, &tag);
    return shell_ranks(&c->p, (uint32_t)i, n, ctr1, tag, ranks);
}

int orc_shell_ranks(const orc_ctx* c, int32_t i, uint64_t eval, int32_t* ranks)
{
    if (!c->cand_off || i < 0 || i >= c->n) return -1;
    int n = c->cand_off[i + 1] - c->cand_off[i];
    uint32_t ctr1, tag;
    shell_stream(c, eval, &ctr1, &tag);
    return shell_ranks(&c->p, (uint32_t)i, n, ctr1, tag, ranks);
}

/* Pair force scalar f (F_i += f * r_ij) of eq. (15) with k_e on the Coulomb
 * part, and the pair energy q_i q_j k_e N(r) + B_BMH(r) (eqs. 8, 14). */
static double pair_scalar(const orc_params* p, int ti, int tj, double r2, double* u)
{
    double r = sqrt(r2);
    double qq = p->coulomb_k * p->q[ti] * p->q[tj];
    int t = ti * ORC_MAXS + tj;
    double A = p->A[t], sg = p->sig[t], rh = p->rho[t], C = p->C[t], D = p->D[t];
    double gsum = 0.0, fsum = 0.0;
    for (int m = 0; m <= p->M; ++m) {
        double sm = sigma_m(p, m);
        double e = exp(-r2 / (2.0 * sm * sm));
        gsum += p->w[m] / (sm * sm) * e;
        fsum += p->w[m] * e;
    }
    double rep = A * exp((sg - r) / rh);
    double r6 = r2 * r2 * r2;
    double r8 = r6 * r2;
    double f = qq * (1.0 / (r2 * r) - gsum) + rep / (rh * r) - 6.0 * C / r8 - 8.0 * D / (r8 * r2);
    if (u) *u = qq * (1.0 / r - fsum) + rep - C / r6 - D / r8;
    return f;
}

double orc_pair_force(const orc_params* p, int32_t ti, int32_t tj, const double d[3], double f[3])
{
    double r2 = norm2(d);
    double u = 0.0;
    double fs = pair_scalar(p, ti, tj, r2, &u);
    for (int a = 0; a < 3; ++a) f[a] = fs * d[a];
    return u;
}

/* Short-range force on atom i from its lists: core sum (eq. 24) plus the
 * reweighted shell batch (eq. 25).  No momentum correction. */
/* 1/2 r_ij (x) F_ij of one pair, F_ij = f r_ij the force on i from j. */
static void pair_virial(double f, const double d[3], double W[6])
{
    W[0] += 0.5 * f * d[0] * d[0];
    W[1] += 0.5 * f * d[1] * d[1];
    W[2] += 0.5 * f * d[2] * d[2];
    W[3] += 0.5 * f * d[0] * d[1];
    W[4] += 0.5 * f * d[0] * d[2];
    W[5] += 0.5 * f * d[1] * d[2];
}

static void short_atom(const orc_params* p, const orc_ctx* c, int i, const int32_t* core, int nc,
                       const int32_t* cand, int nk, uint64_t eval, double f_out[3], double* uc, double* us,
                       double w_out[6])
{
    double Wc[6] = {0, 0, 0, 0, 0, 0}, Ws[6] = {0, 0, 0, 0, 0, 0};
    double rs2 = p->r_shell * p->r_shell;
    double F[3] = {0.0, 0.0, 0.0};
    double Uc = 0.0, Us = 0.0;
    int ti = c->type[i];
    for (int a = 0; a < nc; ++a) {
        int j = core[a];
        double d[3];
        min_image(p, c->pos + 3 * i, c->pos + 3 * j, d);
        double r2 = norm2(d);
        double rcp = core_radius(p, ti, c->type[j]);
        if (!(r2 < rcp * rcp)) continue;
        double u;
        double f = pair_scalar(p, ti, c->type[j], r2, &u);
        for (int x = 0; x < 3; ++x) F[x] += f * d[x];
        Uc += 0.5 * u;
        pair_virial(f, d, Wc);
    }
    int32_t* ranks = (int32_t*)malloc(sizeof(int32_t) * (nk > 0 ? nk : 1));
    uint32_t ctr1, tag;
    shell_stream(c, eval, &ctr1, &tag);
    int nr = shell_ranks(p, (uint32_t)i, nk, ctr1, tag, ranks);
    double wgt = (p->p_r <= 0 || nk <= p->p_r) ? 1.0 : (double)nk / (double)p->p_r;
    double Fs[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < nr; ++a) {
        int j = cand[ranks[a]];
        double d[3];
        min_image(p, c->pos + 3 * i, c->pos + 3 * j, d);
        double r2 = norm2(d);
        double rcp = core_radius(p, ti, c->type[j]);
        if (!(r2 >= rcp * rcp && r2 < rs2)) continue;
        double u;
        double f = pair_scalar(p, ti, c->type[j], r2, &u);
        for (int x = 0; x < 3; ++x) Fs[x] += f * d[x];
        Us += 0.5 * u;
        pair_virial(f, d, Ws);
    }
    free(ranks);
    for (int x = 0; x < 3; ++x) f_out[x] = F[x] + wgt * Fs[x];
    *uc = Uc;
    *us = wgt * Us;
    if (w_out)
        for (int a = 0; a < 6; ++a) w_out[a] = Wc[a] + wgt * Ws[a];
}

/* Short-range force, and per atom its core energy, shell energy and virial. */
static void short_parts(orc_ctx* c, uint64_t eval, double* force, double* uc, double* us, double* wv)
{
    if (!c->core_off) orc_build_lists(c);
    const orc_params* p = &c->p;
    int n = c->n;
#pragma omp parallel for schedule(dynamic, 16) num_threads(ORC_NT)
    for (int i = 0; i < n; ++i) {
        short_atom(p, c, i, c->core + c->core_off[i], c->core_off[i + 1] - c->core_off[i],
                   c->cand + c->cand_off[i], c->cand_off[i + 1] - c->cand_off[i], eval, force + 3 * i, uc + i,
                   us + i, wv + 6 * i);
    }
}

int orc_forces_short(orc_ctx* c, uint64_t eval, double* force, double* u_core, double* u_shell,
                     double* virial)
{
    int n = c->n;
    double* uc = (double*)calloc(n > 0 ? n : 1, sizeof(double));
    double* us = (double*)calloc(n > 0 ? n : 1, sizeof(double));
    double* wv = (double*)calloc(6 * (n > 0 ? n : 1), sizeof(double));
    short_parts(c, eval, force, uc, us, wv);
    double Uc = 0.0, Us = 0.0;
    for (int i = 0; i < n; ++i) {
        Uc += uc[i];
        Us += us[i];
    }
    if (virial) {
        for (int a = 0; a < 6; ++a) virial[a] = 0.0;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 6; ++a) virial[a] += wv[6 * i + a];
    }
    free(uc);
    free(us);
    free(wv);
    if (u_core) *u_core = Uc;
    if (u_shell) *u_shell = Us;
    return 0;
}

int orc_rdf_counts(const orc_ctx* c, double r_max, int32_t n_bins, uint64_t* counts)
{
    if (n_bins < 1 || !(r_max > 0.0)) return -1;
    const orc_params* p = &c->p;
    const int S = p->n_species;
    const double D = r_max / (double)n_bins;
    const double top = ((double)n_bins * D) * ((double)n_bins * D);
    memset(counts, 0, sizeof(uint64_t) * (size_t)S * S * n_bins);
    for (int i = 0; i < c->n; ++i)
        for (int j = 0; j < c->n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(p, c->pos + 3 * i, c->pos + 3 * j, d);
            double r2 = norm2(d);
            if (!(r2 < top)) continue;
            int k = n_bins - 1;  /* the last bin whose lower edge is at or below r^2 */
            while (((double)k * D) * ((double)k * D) > r2) --k;
            counts[((size_t)c->type[i] * S + c->type[j]) * n_bins + k] += 1;
        }
    return 0;
}

int orc_forces_short_atoms(const orc_ctx* c, uint64_t eval, int32_t n_sel, const int32_t* sel, double* force)
{
    const orc_params* p = &c->p;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(ORC_NT)
    for (int a = 0; a < n_sel; ++a) {
        int i = sel[a];
        if (i < 0 || i >= c->n) {
            bad = 1;
            continue;
        }
        int nc, nk;
        scan_atom(c, i, NULL, &nc, NULL, &nk, 1);
        int32_t* core = (int32_t*)malloc(sizeof(int32_t) * (nc + 1));
        int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (nk + 1));
        scan_atom(c, i, core, &nc, cand, &nk, 0);
        double uc, us;
        short_atom(p, c, i, core, nc, cand, nk, eval, force + 3 * a, &uc, &us, NULL);
        free(core);
        free(cand);
    }
    return bad ? -1 : 0;
}

/* Eq. (22): rho(k) = sum_i q_i exp(i k.r_i), k = 2 pi m / L. */
void orc_rho(const orc_ctx* c, int32_t n_modes, const int32_t* m, double* rho)
{
    const orc_params* p = &c->p;
#pragma omp parallel for schedule(static) num_threads(ORC_NT)
    for (int q = 0; q < n_modes; ++q) {
        double k[3];
        for (int a = 0; a < 3; ++a) k[a] = 2.0 * ORC_PI * (double)m[3 * q + a] / p->box[a];
        double re = 0.0, im = 0.0;
        for (int i = 0; i < c->n; ++i) {
            const double* r = c->pos + 3 * i;
            double th = k[0] * r[0] + k[1] * r[1] + k[2] * r[2];
            double qi = p->q[c->type[i]];
            re += qi * cos(th);
            im += qi * sin(th);
        }
        rho[2 * q] = re;
        rho[2 * q + 1] = im;
    }
}

/* Per-atom sum over modes of coef_q * k_q * Im(exp(-i k.r_i) rho_q), times
 * -k_e q_i coef_scale.  coef for sampled modes is 1/|k|^2 (eq. 29), for the
 * full sum F^(k) (eq. 23); the caller folds the remaining constants into
 * coef_scale.  Here coef is 1/|k|^2. */
void orc_kforce_atoms(const orc_ctx* c, int32_t n_modes, const int32_t* m, const double* rho,
                      double coef_scale, int32_t n_sel, const int32_t* sel, double* force)
{
    const orc_params* p = &c->p;
#pragma omp parallel for schedule(static) num_threads(ORC_NT)
    for (int a = 0; a < n_sel; ++a) {
        int i = sel ? sel[a] : a;
        const double* r = c->pos + 3 * i;
        double F[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < n_modes; ++q) {
            double k[3];
            for (int x = 0; x < 3; ++x) k[x] = 2.0 * ORC_PI * (double)m[3 * q + x] / p->box[x];
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            double th = k[0] * r[0] + k[1] * r[1] + k[2] * r[2];
            /* Im(exp(-i th) (re + i im)) = cos(th) im - sin(th) re */
            double imv = cos(th) * rho[2 * q + 1] - sin(th) * rho[2 * q];
            for (int x = 0; x < 3; ++x) F[x] += k[x] / k2 * imv;
        }
        double qi = p->q[c->type[i]];
        for (int x = 0; x < 3; ++x) force[3 * a + x] = -p->coulomb_k * qi * coef_scale * F[x];
    }
}

static double box_volume(const orc_params* p) { return p->box[0] * p->box[1] * p->box[2]; }

/* Per-atom split of the k-space energy and virial: mode p's energy
 * (k_e/2) coef_p |rho_p|^2 is shared among atoms as (k_e/2) coef_p q_i
 * Re(e^{-ik.r_i} rho_p) (these sum to it), its virial alike with the
 * factor (delta_ab - g_p k_a k_b).  Adds into epot[n] and wat[n][6]. */
static void kspace_atom_parts(const orc_ctx* c, long cnt, const int32_t* m, const double* rho, const double* coef,
                              const double* g, double* epot, double* wat)
{
    const orc_params* p = &c->p;
#pragma omp parallel for schedule(static) num_threads(ORC_NT)
    for (int i = 0; i < c->n; ++i) {
        const double* r = c->pos + 3 * i;
        double qh = 0.5 * p->coulomb_k * p->q[c->type[i]];
        double e = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
        for (long t = 0; t < cnt; ++t) {
            double k[3];
            for (int a = 0; a < 3; ++a) k[a] = 2.0 * ORC_PI * (double)m[3 * t + a] / p->box[a];
            double th = k[0] * r[0] + k[1] * r[1] + k[2] * r[2];
            /* Re(e^{-i th} rho) = cos(th) Re rho + sin(th) Im rho */
            double re = cos(th) * rho[2 * t] + sin(th) * rho[2 * t + 1];
            double x = qh * coef[t] * re;
            e += x;
            mode_virial(x, g[t], k, w);
        }
        epot[i] += e;
        for (int a = 0; a < 6; ++a) wat[6 * i + a] += w[a];
    }
}

/* Full k-sum of eq. (23) over every k != 0 whose narrowest-Gaussian factor
 * exp(-s^2 k^2 / 2) is at least e^-45. */
static int kspace_full(orc_ctx* c, double* force, double* u_k, double* virial, double* epot, double* wat)
{
    const orc_params* p = &c->p;
    int nmax[3];
    for (int a = 0; a < 3; ++a) nmax[a] = (int)floor(sqrt(90.0) / (p->s * 2.0 * ORC_PI / p->box[a]));
    long cnt = 0;
    for (int x = -nmax[0]; x <= nmax[0]; ++x)
        for (int y = -nmax[1]; y <= nmax[1]; ++y)
            for (int z = -nmax[2]; z <= nmax[2]; ++z) {
                if (x == 0 && y == 0 && z == 0) continue;
                double kx = 2.0 * ORC_PI * x / p->box[0], ky = 2.0 * ORC_PI * y / p->box[1],
                       kz = 2.0 * ORC_PI * z / p->box[2];
                double k2 = kx * kx + ky * ky + kz * kz;
                if (0.5 * p->s * p->s * k2 > 45.0) continue;
                ++cnt;
            }
    int32_t* m = (int32_t*)calloc(3 * (cnt + 1), sizeof(int32_t));
    double* fh = (double*)malloc(sizeof(double) * (cnt + 1));
    long q = 0;
    for (int x = -nmax[0]; x <= nmax[0]; ++x)
        for (int y = -nmax[1]; y <= nmax[1]; ++y)
            for (int z = -nmax[2]; z <= nmax[2]; ++z) {
                if (x == 0 && y == 0 && z == 0) continue;
                double kx = 2.0 * ORC_PI * x / p->box[0], ky = 2.0 * ORC_PI * y / p->box[1],
                       kz = 2.0 * ORC_PI * z / p->box[2];
                double k2 = kx * kx + ky * ky + kz * kz;
                if (0.5 * p->s * p->s * k2 > 45.0) continue;
                m[3 * q] = x;
                m[3 * q + 1] = y;
                m[3 * q + 2] = z;
                fh[q] = orc_far_hat(p, sqrt(k2));
                ++q;
            }
    double* rho = (double*)malloc(sizeof(double) * 2 * (cnt + 1));
    orc_rho(c, (int32_t)cnt, m, rho);
    double V = box_volume(p);
    double U = 0.0;
    for (long t = 0; t < cnt; ++t) U += fh[t] * (rho[2 * t] * rho[2 * t] + rho[2 * t + 1] * rho[2 * t + 1]) / (2.0 * V);
    *u_k = p->coulomb_k * U;
    if (virial) {
        /* W_ab = sum_k (k_e |rho|^2 / 2V) (F^ delta_ab - G k_a k_b) */
        for (int a = 0; a < 6; ++a) virial[a] = 0.0;
        for (long t = 0; t < cnt; ++t) {
            double k[3];
            for (int a = 0; a < 3; ++a) k[a] = 2.0 * ORC_PI * (double)m[3 * t + a] / p->box[a];
            double kk = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
            double e = fh[t] * (rho[2 * t] * rho[2 * t] + rho[2 * t + 1] * rho[2 * t + 1]) / V;
            mode_virial(0.5 * p->coulomb_k * e, orc_far_hat_g(p, kk) / fh[t], k, virial);
        }
    }
    if (epot) {
        double* coef = (double*)malloc(sizeof(double) * (cnt + 1));
        double* g = (double*)malloc(sizeof(double) * (cnt + 1));
        for (long t = 0; t < cnt; ++t) {
            double k2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double k = 2.0 * ORC_PI * (double)m[3 * t + a] / p->box[a];
                k2 += k * k;
            }
            coef[t] = fh[t] / V;
            g[t] = orc_far_hat_g(p, sqrt(k2)) / fh[t];
        }
        kspace_atom_parts(c, cnt, m, rho, coef, g, epot, wat);
        free(coef);
        free(g);
    }
    /* eq. (23): F_i = -sum_k (q_i k / V) F^(k) Im(e^{-ik.r_i} rho(k)) */
#pragma omp parallel for schedule(static) num_threads(ORC_NT)
    for (int i = 0; i < c->n; ++i) {
        const double* r = c->pos + 3 * i;
        double F[3] = {0.0, 0.0, 0.0};
        for (long t = 0; t < cnt; ++t) {
            double k[3];
            for (int a = 0; a < 3; ++a) k[a] = 2.0 * ORC_PI * (double)m[3 * t + a] / p->box[a];
            double th = k[0] * r[0] + k[1] * r[1] + k[2] * r[2];
            double imv = cos(th) * rho[2 * t + 1] - sin(th) * rho[2 * t];
            for (int a = 0; a < 3; ++a) F[a] += k[a] / V * fh[t] * imv;
        }
        double qi = p->q[c->type[i]];
        for (int a = 0; a < 3; ++a) force[3 * i + a] = -p->coulomb_k * qi * F[a];
    }
    free(m);
    free(fh);
    free(rho);
    return 0;
}

static int kspace_parts(orc_ctx* c, uint64_t eval, double* force, double* u_k, double* virial, double* epot,
                        double* wat);

int orc_forces_kspace(orc_ctx* c, uint64_t eval, double* force, double* u_k, double* virial)
{
    return kspace_parts(c, eval, force, u_k, virial, NULL, NULL);
}

static int kspace_parts(orc_ctx* c, uint64_t eval, double* force, double* u_k, double* virial, double* epot,
                        double* wat)
{
    const orc_params* p = &c->p;
    if (p->p_f <= 0) return kspace_full(c, force, u_k, virial, epot, wat);
    if (!c->have_kt) {
        ktab_build(p, &c->kt);
        c->have_kt = 1;
    }
    int P = p->p_f;
    int32_t* m = (int32_t*)malloc(sizeof(int32_t) * 3 * P);
    kmodes_from_tab(p, &c->kt, eval, m);
    double* rho = (double*)malloc(sizeof(double) * 2 * P);
    orc_rho(c, P, m, rho);
    double V = box_volume(p), S = c->kt.S;
    /* eq. (29): F_i = -(S q_i / (P_F V)) sum_p k_p Im(e^{-ik_p.r_i} rho_p) / |k_p|^2 */
    orc_kforce_atoms(c, P, m, rho, S / ((double)P * V), c->n, NULL, force);
    /* U* = sum_k F^ |rho|^2 / (2V) estimated as S/(2 V P_F) sum_p |rho_p|^2 / |k_p|^2 */
    double U = 0.0;
    for (int q = 0; q < P; ++q) {
        double k2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double k = 2.0 * ORC_PI * (double)m[3 * q + a] / p->box[a];
            k2 += k * k;
        }
        U += (rho[2 * q] * rho[2 * q] + rho[2 * q + 1] * rho[2 * q + 1]) / k2;
    }
    *u_k = p->coulomb_k * S / (2.0 * V * (double)P) * U;
    if (virial) {
        /* importance-sampled estimator of the full-sum virial: each mode's
         * term divided by P_F P(k) = P_F k^2 F^(k) / S */
        for (int a = 0; a < 6; ++a) virial[a] = 0.0;
        for (int q = 0; q < P; ++q) {
            double k[3];
            for (int a = 0; a < 3; ++a) k[a] = 2.0 * ORC_PI * (double)m[3 * q + a] / p->box[a];
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            double kk = sqrt(k2);
            double e = S / ((double)P * V * k2) * (rho[2 * q] * rho[2 * q] + rho[2 * q + 1] * rho[2 * q + 1]);
            mode_virial(0.5 * p->coulomb_k * e, orc_far_hat_g(p, kk) / orc_far_hat(p, kk), k, virial);
        }
    }
    if (epot) {
        double* coef = (double*)malloc(sizeof(double) * P);
        double* g = (double*)malloc(sizeof(double) * P);
        for (int q = 0; q < P; ++q) {
            double k2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double k = 2.0 * ORC_PI * (double)m[3 * q + a] / p->box[a];
                k2 += k * k;
            }
            coef[q] = S / ((double)P * V * k2);
            g[q] = orc_far_hat_g(p, sqrt(k2)) / orc_far_hat(p, sqrt(k2));
        }
        kspace_atom_parts(c, P, m, rho, coef, g, epot, wat);
        free(coef);
        free(g);
    }
    free(m);
    free(rho);
    return 0;
}

static double self_energy(const orc_ctx* c)
{
    const orc_params* p = &c->p;
    double W = 0.0;
    for (int m = 0; m <= p->M; ++m) W += p->w[m];
    double Q2 = 0.0;
    for (int i = 0; i < c->n; ++i) Q2 += p->q[c->type[i]] * p->q[c->type[i]];
    return 0.5 * p->coulomb_k * Q2 * W;
}

static double kinetic(const orc_ctx* c)
{
    double K = 0.0;
    for (int i = 0; i < c->n; ++i) {
        double m = c->p.mass[c->type[i]];
        const double* v = c->vel + 3 * i;
        K += 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
    return K / ORC_ACC;
}

/* Per-atom energy and virial shares of the last evaluation (kept when the
 * evaluation is asked for them): the core and shell half-pair sums of the
 * atom's own lists (the shell part with its batch weight), the atom's share
 * of each k-space mode, minus its self term k_e q_i^2 sum_m w_m / 2. */
static void forces_eval(orc_ctx* c, uint64_t eval, double* force, orc_energy* e, int parts)
{
    int n = c->n;
    int n1 = n > 0 ? n : 1;
    double* fk = (double*)calloc(3 * n1, sizeof(double));
    double* ucs = (double*)calloc(n1, sizeof(double));
    double* uss = (double*)calloc(n1, sizeof(double));
    double* wv = (double*)calloc(6 * n1, sizeof(double));
    double uc = 0.0, us = 0.0, uk = 0.0, ws[6] = {0, 0, 0, 0, 0, 0}, wk[6] = {0, 0, 0, 0, 0, 0};
    short_parts(c, eval, force, ucs, uss, wv);
    for (int i = 0; i < n; ++i) {
        uc += ucs[i];
        us += uss[i];
    }
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 6; ++a) ws[a] += wv[6 * i + a];
    if (parts) {
        if (!c->epot) {
            c->epot = (double*)malloc(sizeof(double) * n1);
            c->wat = (double*)malloc(sizeof(double) * 6 * n1);
        }
        const orc_params* p = &c->p;
        double wsum = 0.0;
        for (int m = 0; m <= p->M; ++m) wsum += p->w[m];
        for (int i = 0; i < n; ++i) {
            double qi = p->q[c->type[i]];
            c->epot[i] = ucs[i] + uss[i] - 0.5 * p->coulomb_k * qi * qi * wsum;
        }
        memcpy(c->wat, wv, sizeof(double) * 6 * n);
    }
    free(ucs);
    free(uss);
    free(wv);
    /* eq. (26)-(27): subtract the mean short-range force */
    double corr[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) corr[a] += force[3 * i + a];
    for (int a = 0; a < 3; ++a) corr[a] = n > 0 ? corr[a] / n : 0.0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) force[3 * i + a] -= corr[a];
    if (n > 0) kspace_parts(c, eval, fk, &uk, wk, parts ? c->epot : NULL, parts ? c->wat : NULL);
    for (int i = 0; i < 3 * n; ++i) force[i] += fk[i];
    free(fk);
    memcpy(c->frc, force, sizeof(double) * 3 * n);
    c->eval = eval;
    if (e) {
        e->u_core = uc;
        e->u_shell = us;
        e->u_kspace = uk;
        e->u_self = self_energy(c);
        e->u_total = uc + us + uk - e->u_self;
        e->kinetic = kinetic(c);
        for (int a = 0; a < 3; ++a) e->p_corr[a] = corr[a];
        for (int a = 0; a < 6; ++a) e->virial[a] = ws[a] + wk[a];
    }
}

/* Eq. (50) and eq. (51) at the current velocities, from the per-atom shares
 * of the last evaluation.  The pair term of eq. (51), half the sum over pairs
 * of (F_ij . (v_i + v_j)) r_ij, equals sum_i W_i v_i with W_i half the sum of
 * r_ij (x) F_ij over the atom's partners; the k-space modes enter through
 * their per-atom virial shares the same way. */
static void transport_terms(const orc_ctx* c, orc_energy* e)
{
    const orc_params* p = &c->p;
    double S[6] = {0, 0, 0, 0, 0, 0}, J[3] = {0, 0, 0};
    for (int i = 0; i < c->n; ++i) {
        double m = p->mass[c->type[i]] / ORC_ACC;
        const double* v = c->vel + 3 * i;
        const double* w = c->wat + 6 * i;
        S[0] += m * v[0] * v[0];
        S[1] += m * v[1] * v[1];
        S[2] += m * v[2] * v[2];
        S[3] += m * v[0] * v[1];
        S[4] += m * v[0] * v[2];
        S[5] += m * v[1] * v[2];
        double ei = 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + c->epot[i];
        J[0] += ei * v[0] + w[0] * v[0] + w[3] * v[1] + w[4] * v[2];
        J[1] += ei * v[1] + w[3] * v[0] + w[1] * v[1] + w[5] * v[2];
        J[2] += ei * v[2] + w[4] * v[0] + w[5] * v[1] + w[2] * v[2];
    }
    double V = box_volume(p);
    for (int a = 0; a < 6; ++a) e->stress[a] = S[a] + e->virial[a];
    for (int a = 0; a < 3; ++a) e->heat_flux[a] = J[a] / V;
}

int orc_forces(orc_ctx* c, uint64_t eval, double* force, orc_energy* e)
{
    forces_eval(c, eval, force, e, e != NULL);
    if (e) transport_terms(c, e);
    return 0;
}

#define ORC_KB 8.617333262e-5 /* eV/K */

/* Nose-Hoover half step (Trotter splitting of the NVT equations of motion
 * with one thermostat variable; Martyna, Tuckerman & Klein, Mol. Phys. 87,
 * 1117 (1996), chain of length one): with G = (2K - g k_B T0)/Q,
 * v_xi += G dt/4; v *= exp(-v_xi dt/2) (K scaled alike); xi += v_xi dt/2;
 * v_xi += G dt/4 with the new K.  g = 3N - 3, Q = g k_B T0 tau^2. */
static void nh_half(orc_ctx* c, double gkt, double Q, double dt)
{
    double K = kinetic(c);
    c->nh_v += 0.25 * dt * (2.0 * K - gkt) / Q;
    double s = exp(-0.5 * dt * c->nh_v);
    for (int i = 0; i < 3 * c->n; ++i) c->vel[i] *= s;
    K *= s * s;
    c->nh_x += 0.5 * dt * c->nh_v;
    c->nh_v += 0.25 * dt * (2.0 * K - gkt) / Q;
}

/* Three standard normals for the Langevin step of atom i at step `step`:
 * Box-Muller on four 53-bit uniforms of the stream (i, step, TAG_LANGEVIN):
 * r = sqrt(-2 ln(1 - u1)), z0 = r cos(2 pi u2), z1 = r sin(2 pi u2), then
 * z2 = sqrt(-2 ln(1 - u3)) cos(2 pi u4). */
static void langevin_normals(const orc_params* p, uint32_t i, uint32_t step, double z[3])
{
    orc_stream s;
    stream_init(&s, p->seed, i, step, ORC_TAG_LANGEVIN, p->replica);
    double u1 = stream_uniform(&s), u2 = stream_uniform(&s);
    double u3 = stream_uniform(&s), u4 = stream_uniform(&s);
    double r = sqrt(-2.0 * log(1.0 - u1));
    z[0] = r * cos(2.0 * ORC_PI * u2);
    z[1] = r * sin(2.0 * ORC_PI * u2);
    z[2] = sqrt(-2.0 * log(1.0 - u3)) * cos(2.0 * ORC_PI * u4);
}

/* Velocity Verlet: v += dt/2 F/m; r += dt v (wrapped); lists rebuilt when the
 * step number is a multiple of rebuild_every or when some atom has moved more
 * than skin/2 since the last build; F at eval index = step number;
 * v += dt/2 F/m.  Thermostats (t_target > 0 and tau_t > 0):
 *  Berendsen: v *= sqrt(1 + (dt/tau)(T0/T - 1)) at the start of each step,
 *    T from the current kinetic energy and 3N - 3 degrees of freedom;
 *  Nose-Hoover: a half step of nh_half before the first kick and after the
 *    second;
 *  Langevin (BAOAB; Leimkuhler & Matthews, AMRX 2013): the drift becomes
 *    r += dt/2 v; v = c1 v + c2 z; r += dt/2 v with c1 = exp(-dt/tau),
 *    c2 = sqrt((1 - c1^2) k_B T0 / m), z standard normals. */
int orc_vv_steps(orc_ctx* c, int32_t n_steps, orc_energy* e_last)
{
    int n = c->n;
    const orc_params* p = &c->p;
    if (!c->core_off) orc_build_lists(c);
    double* f = (double*)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    orc_energy e;
    memset(&e, 0, sizeof(e));
    int thermo = p->t_target > 0.0 && p->tau_t > 0.0 && n > 1;
    int kind = thermo ? p->thermostat : -1;
    double gkt = (3.0 * n - 3.0) * ORC_KB * p->t_target;
    double Q = gkt * p->tau_t * p->tau_t;
    double c1 = exp(-p->dt / p->tau_t);
    for (int k = 0; k < n_steps; ++k) {
        uint64_t step = c->eval + 1;
        double lam = 1.0;
        if (kind == ORC_THERMO_BERENDSEN) {
            double ke = kinetic(c);
            if (ke > 0.0) {
                double T = 2.0 * ke / ((3.0 * n - 3.0) * ORC_KB);
                double l2 = 1.0 + p->dt / p->tau_t * (p->t_target / T - 1.0);
                lam = l2 > 0.0 ? sqrt(l2) : 0.0;
            }
        } else if (kind == ORC_THERMO_NOSE_HOOVER) {
            nh_half(c, gkt, Q, p->dt);
        }
        for (int i = 0; i < n; ++i) {
            double a = 0.5 * p->dt * ORC_ACC / p->mass[c->type[i]];
            double* v = c->vel + 3 * i;
            double* x = c->pos + 3 * i;
            if (kind == ORC_THERMO_LANGEVIN) {
                double z[3];
                langevin_normals(p, (uint32_t)i, (uint32_t)step, z);
                double c2 = sqrt((1.0 - c1 * c1) * ORC_KB * p->t_target * ORC_ACC / p->mass[c->type[i]]);
                for (int d = 0; d < 3; ++d) {
                    v[d] = v[d] + a * c->frc[3 * i + d];
                    x[d] += 0.5 * p->dt * v[d];
                    v[d] = c1 * v[d] + c2 * z[d];
                    x[d] += 0.5 * p->dt * v[d];
                }
            } else {
                for (int d = 0; d < 3; ++d) {
                    v[d] = lam * v[d] + a * c->frc[3 * i + d];
                    x[d] += p->dt * v[d];
                }
            }
            wrap(p, x);
        }
        int every = p->rebuild_every > 0 ? p->rebuild_every : 1;
        int moved = 0;
        double half2 = 0.25 * p->skin * p->skin;
        for (int i = 0; i < n && !moved; ++i) {
            double d[3];
            min_image(p, c->pos + 3 * i, c->ref + 3 * i, d);
            if (norm2(d) > half2) moved = 1;
        }
        if (step % (uint64_t)every == 0 || moved) orc_build_lists(c);
        forces_eval(c, step, f, &e, k == n_steps - 1);
        for (int i = 0; i < n; ++i) {
            double a = 0.5 * p->dt * ORC_ACC / p->mass[c->type[i]];
            for (int x = 0; x < 3; ++x) c->vel[3 * i + x] += a * f[3 * i + x];
        }
        if (kind == ORC_THERMO_NOSE_HOOVER) nh_half(c, gkt, Q, p->dt);
    }
    e.kinetic = kinetic(c);
    e.u_total = e.u_core + e.u_shell + e.u_kspace - e.u_self;
    e.e_thermostat = kind == ORC_THERMO_NOSE_HOOVER ? 0.5 * Q * c->nh_v * c->nh_v + gkt * c->nh_x : 0.0;
    if (n_steps > 0) transport_terms(c, &e);
    if (e_last) *e_last = e;
    free(f);
    return (int)c->eval;
}

void orc_get_state(const orc_ctx* c, double* pos, double* vel, double* force, uint64_t* eval)
{
    if (pos) memcpy(pos, c->pos, sizeof(double) * 3 * c->n);
    if (vel) memcpy(vel, c->vel, sizeof(double) * 3 * c->n);
    if (force) memcpy(force, c->frc, sizeof(double) * 3 * c->n);
    if (eval) *eval = c->eval;
}
