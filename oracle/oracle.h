/*
 * oracle.h -- plain double-precision CPU reference of the IRBSOG force
 * evaluation for Born-Mayer-Huggins (BMH) melts (Chen, Liang, Xu, Zhang,
 * "Random Batch Sum-of-Gaussians Method for Molecular Dynamics of
 * Born-Mayer-Huggins Systems", arXiv:2512.24970).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no source with the GPU library: every formula
 * here is written again from the paper (and from the published definitions of
 * Philox4x32-10, Lemire's bounded integers and Floyd's sampling).
 *
 * Units: eV, Angstrom, ps, amu, elementary charge.
 *
 * Parity status of each function is listed in its comment; "pinned" means a
 * CPU test checks it against something other than itself (a closed form, a
 * published value, a brute-force sum, a statistical identity).
 */
#ifndef RBSOG_ORACLE_H
#define RBSOG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXS 8      /* species */
#define ORC_MAXM 511    /* highest Gaussian index of the SOG series */

/* Philox stream tags (third counter word, low byte). */
#define ORC_TAG_SHELL 2u
#define ORC_TAG_KMODE 3u
#define ORC_TAG_SHELL_BUILD 5u  /* shell batch drawn once per list build */
#define ORC_TAG_LANGEVIN 6u     /* Langevin noise: counter word 1 = step number */

/* Thermostats (active when t_target > 0 and tau_t > 0). */
#define ORC_THERMO_BERENDSEN 0    /* v <- lambda v at the start of each step */
#define ORC_THERMO_NOSE_HOOVER 1  /* one Nose-Hoover variable, Trotter half steps around the step */
#define ORC_THERMO_LANGEVIN 2     /* BAOAB splitting, friction 1/tau_t */

typedef struct {
    int32_t n_species;
    int32_t p_r;            /* shell batch size; <= 0: every candidate, weight 1 */
    int32_t p_f;            /* Fourier batch size; <= 0: full k-sum of eq. (23) */
    int32_t M;              /* SOG series runs over m = 0..M (set by orc_sog_setup) */
    uint32_t replica;
    int32_t rebuild_every;
    uint64_t seed;
    double box[3];
    double r_core, r_shell, skin;
    double coulomb_k;       /* e^2/(4 pi eps0) in eV*Angstrom */
    double dt;              /* ps */
    double sog_eps;
    double b, s;            /* SOG base and bandwidth (set by orc_sog_setup) */
    double x_c;             /* r_shell / s */
    double w[ORC_MAXM + 1]; /* SOG weights, w[0] adjusted for C1 continuity */
    double q[ORC_MAXS];
    double mass[ORC_MAXS];
    double A[ORC_MAXS * ORC_MAXS];
    double sig[ORC_MAXS * ORC_MAXS];
    double rho[ORC_MAXS * ORC_MAXS];
    double C[ORC_MAXS * ORC_MAXS];
    double D[ORC_MAXS * ORC_MAXS];
    double t_target;        /* K; Berendsen thermostat when t_target > 0 and tau_t > 0 */
    double tau_t;           /* ps */
    int32_t shell_stored;   /* 0: fresh shell batch every force evaluation,
                               stream (atom, eval, TAG_SHELL); 1: one batch per
                               list build, kept until the next build, stream
                               (atom, build number, TAG_SHELL_BUILD) with builds
                               counted from 0 (Section 2.4: O(core + P_R) list
                               entries per atom).  Needs p_r > 0. */
    int32_t thermostat;     /* ORC_THERMO_* */
    double r_core_pair[ORC_MAXS * ORC_MAXS]; /* core radius per species pair (symmetric);
                                                0 means r_core.  Pairs inside it are summed
                                                in full (eq. 24), the rest of the shell is
                                                sampled (eq. 25). */
} orc_params;

typedef struct {
    double u_core, u_shell, u_kspace, u_self, u_total, kinetic;
    double p_corr[3];       /* momentum correction that was subtracted, eq. (26) */
    double e_thermostat;    /* Nose-Hoover: Q v_xi^2 / 2 + g k_B T0 xi (else 0) */
    double virial[6];       /* W_ab = -dU/de_ab (xx, yy, zz, xy, xz, yz), eV; pressure
                               tensor V P_ab = sum m v_a v_b + W_ab.  Excludes the
                               momentum correction (a uniform force of zero mean). */
    double stress[6];       /* S_ab of eq. (50): sum m v_a v_b + W_ab, eV (same order) */
    double heat_flux[3];    /* J of eq. (51), eV / (A^2 ps): (1/V) [sum e_i v_i + sum W_i v_i]
                               with e_i = m v_i^2 / 2 + the atom's share of the potential
                               energy and W_i its share of the virial */
} orc_energy;

/* ---- Philox4x32-10 (Salmon et al., SC'11).  Pinned: published test vectors. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* First `n` 32-bit words of the stream (index, eval, tag|replica<<8, block=0..). */
void orc_stream_words(uint64_t seed, uint32_t index, uint32_t eval, uint32_t tag,
                      uint32_t replica, int n, uint32_t* out);

/* Uniform integer in [0, range) by Lemire's multiply-shift with rejection,
 * drawn from the given words (at most n_words consumed).  Returns the value
 * and stores the number of consumed words.  Pinned: exhaustive identity. */
uint32_t orc_bounded_from_words(const uint32_t* words, int n_words, uint32_t range,
                                int* consumed);

/* ---- SOG decomposition, eqs. (4)-(10) ------------------------------------ */
/* b = 2^(1/(2j)) for the smallest j >= 1 whose eq. (5) bound is <= eps. */
double orc_sog_b_from_eps(double eps);
/* Smallest positive root x_c = r_c/s of the C1 conditions (value and slope)
 * for the series m = 0..M with base b, in units s = 1.  Pinned: C1 residuals. */
double orc_sog_xc(double b, int M);
/* Fill p->b, p->s, p->M, p->x_c, p->w from p->sog_eps and p->r_shell. */
int orc_sog_setup(orc_params* p);

/* F(r) (eq. 7) and N(r) (eq. 8) and -dN/dr / r for the configured series. */
double orc_far(const orc_params* p, double r);
double orc_near(const orc_params* p, double r);
/* Fourier transform of F (eq. 21). */
double orc_far_hat(const orc_params* p, double k);

/* ---- Fourier-space importance sampling, eq. (28) ------------------------- */
/* S = sum_{k != 0} k^2 F^(k) by the separable 1D lattice sums. */
double orc_kspace_S(const orc_params* p);
/* Draw P_F = p->p_f integer mode vectors m[P_F][3] for force evaluation `eval`. */
int orc_kmodes(const orc_params* p, uint64_t eval, int32_t* m_out, double* S_out);

/* ---- System ----------------------------------------------------------- */
typedef struct orc_ctx orc_ctx;

orc_ctx* orc_create(const orc_params* p, int32_t n, const int32_t* type,
                    const double* pos, const double* vel);
void orc_destroy(orc_ctx* c);
/* Brute-force core list (r < r_core(ti,tj) + skin) and shell candidates
 * (r_core(ti,tj) - skin <= r < r_shell + skin), r_core(ti,tj) the pair's
 * core radius.  Candidates are ordered by (cell,
 * atom index) on a grid of n_c = 2 floor(L / (r_shell + skin)) cells per
 * axis (one cell where floor(L / (r_shell + skin)) is below 3), cell =
 * floor(x n_c / L) with x fastest. */
int orc_build_lists(orc_ctx* c);
int orc_list_counts(const orc_ctx* c, int32_t* n_core, int32_t* n_cand);
int orc_list_atom(const orc_ctx* c, int32_t i, int32_t* core, int32_t* cand);
/* Shell batch of atom i for evaluation `eval`: ranks into the candidate list,
 * ascending.  Returns the number of ranks (min(P_R, n_i), or n_i if P_R <= 0).
 * With shell_stored the batch is the one drawn for the last list build and
 * `eval` is not used. */
int orc_shell_ranks(const orc_ctx* c, int32_t i, uint64_t eval, int32_t* ranks);
/* The lists of atom i alone, by the same scan over every other atom (no full
 * build, so usable at 10^6 atoms and more): with core or cand NULL only the
 * counts; otherwise core and cand must hold them.  -1 for a bad index. */
int orc_scan_lists_atom(const orc_ctx* c, int32_t i, int32_t* core, int32_t* cand, int32_t* n_core,
                        int32_t* n_cand);
/* The shell ranks of atom i for evaluation `eval` given its candidate count
 * n (no lists needed); as orc_shell_ranks otherwise. */
int orc_shell_ranks_count(const orc_ctx* c, int32_t i, int32_t n, uint64_t eval, int32_t* ranks);
/* List builds since the system was created (the first build is number 0). */
int64_t orc_n_builds(const orc_ctx* c);
/* Force on i from j (d = r_i - r_j, minimum image) of eq. (15) with k_e;
 * returns the pair energy q_i q_j k_e N(r) + B_BMH(r). */
double orc_pair_force(const orc_params* p, int32_t ti, int32_t tj, const double d[3], double f[3]);
/* Full IRBSOG force on every atom (eqs. 15, 24-27, 29).  force[N][3]. */
int orc_forces(orc_ctx* c, uint64_t eval, double* force, orc_energy* e);
/* Parts of the above: short range (before the momentum correction) and k-space. */
/* virial (may be NULL): W[6] of the short-range estimator, 1/2 sum_i sum_j
 * r_ij (x) F_ij over the core pairs plus N_shell/P_R times the same over the
 * batch (eqs. 24-25). */
int orc_forces_short(orc_ctx* c, uint64_t eval, double* force, double* u_core, double* u_shell,
                     double* virial);
/* virial (may be NULL): W[6] of the k-space part, sum over modes of
 * (k_e/2) e_k (delta_ab - g(k) k_a k_b) with e_k |rho|^2 times the mode's
 * coefficient (eq. 23 or 29) and g(k) = G(k)/F^(k), G = -F^'(k)/k. */
int orc_forces_kspace(orc_ctx* c, uint64_t eval, double* force, double* u_k, double* virial);
/* G(k) = -dF^/dk / k = sum_m (2 pi)^{3/2} w_m sigma_m^5 exp(-sigma_m^2 k^2 / 2). */
double orc_far_hat_g(const orc_params* p, double k);
/* Structure factors rho(k) (eq. 22) for the given integer modes. */
void orc_rho(const orc_ctx* c, int32_t n_modes, const int32_t* m, double* rho /*[n][2]*/);
/* Velocity-Verlet steps; lists are rebuilt when the step number is a multiple
 * of rebuild_every or when an atom has moved more than skin/2 since the last
 * build.  Returns the eval index of the last force evaluation. */
int orc_vv_steps(orc_ctx* c, int32_t n_steps, orc_energy* e_last);
void orc_get_state(const orc_ctx* c, double* pos, double* vel, double* force, uint64_t* eval);

/* Short-range force on selected atoms of a large system, each by an O(N) scan
 * (no stored lists).  Without the momentum correction. */
int orc_forces_short_atoms(const orc_ctx* c, uint64_t eval, int32_t n_sel,
                           const int32_t* sel, double* force);
/* k-space force on selected atoms given the structure factors of the modes. */
void orc_kforce_atoms(const orc_ctx* c, int32_t n_modes, const int32_t* m,
                      const double* rho, double coef_scale, int32_t n_sel,
                      const int32_t* sel, double* force);

/* Radial distribution counts at the current positions (the pair histogram
 * behind the RDF of Section 3.1): counts[(a S + b) n_bins + k] (S species)
 * = ordered pairs i != j of types (a, b) whose minimum-image r^2 satisfies
 * e_k <= r^2 < e_{k+1}, e_k = (k D)(k D) in FP64, D = r_max / n_bins.  All
 * pairs by brute force (O(N^2)).  Returns 0, or -1 for n_bins < 1 or
 * r_max <= 0. */
int orc_rdf_counts(const orc_ctx* c, double r_max, int32_t n_bins, uint64_t* counts);

/* Threads the oracle's parallel loops use (OpenMP), 0 = library default. */
void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
