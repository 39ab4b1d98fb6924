/*
 * rbsog.h -- C ABI of librbsog, the MI355X (gfx950) implementation of the
 * IRBSOG force evaluation for Born-Mayer-Huggins melts: random batch list
 * (RBL) short range plus random batch sum-of-Gaussians (RBSOG) long range,
 * and velocity-Verlet steps (Chen, Liang, Xu, Zhang, arXiv:2512.24970,
 * Section 2).
 *
 * Conventions
 *  - Units: eV, Angstrom, ps, amu, elementary charge, K.
 *  - Every call returns an rbsog_status (0 = OK, < 0 = error).  Nothing throws
 *    or aborts across the ABI; rbsog_last_error() holds the message of the
 *    last failed call of a context.
 *  - One context owns one HIP stream (the caller's, or the default stream)
 *    and the device memory of one system, or of a batch of independent
 *    systems (replicas) that every kernel launch covers at once.  A context
 *    is not thread safe.
 *  - Per-atom arrays passed in or out are in the caller's atom order ("user
 *    order", atom index = id) and row-major [N][3] for vectors.  For a batch
 *    the systems' rows follow each other in system order (system r starts at
 *    row n_atoms[0] + ... + n_atoms[r-1]) and N is the total.  Inside, the
 *    library keeps atoms sorted by cell; that order never leaks out.
 *  - Pointer arguments are owned by the caller and only read or written
 *    during the call (device outputs are written by work enqueued on the
 *    context's stream; the call returns once that work is enqueued unless it
 *    says it synchronises).
 *  - Invalid parameters are rejected before any device allocation.
 */
#ifndef RBSOG_H
#define RBSOG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RBSOG_MAX_SPECIES 8
#define RBSOG_MAX_SOG 512  /* capacity of the SOG weight array returned by rbsog_sog_params */

typedef struct rbsog_ctx rbsog_ctx;

typedef enum {
    RBSOG_OK = 0,
    RBSOG_E_ARG = -1,        /* invalid argument or parameter */
    RBSOG_E_STATE = -2,      /* call out of order (e.g. no system set) */
    RBSOG_E_HIP = -3,        /* a HIP runtime call failed */
    RBSOG_E_OOM = -4,        /* device allocation failed */
    RBSOG_E_LIST_STALE = -5, /* rbsog_compute_forces after rbsog_set_positions moved an atom more
                                than skin/2 from its position at the last list build */
    RBSOG_E_NONNEUTRAL = -6, /* total charge is not zero */
    RBSOG_E_BOX = -7,        /* box shorter than 2 (r_shell + skin) along some axis */
    RBSOG_E_NONFINITE = -8,  /* a non-finite input, or a non-finite force or position produced by a
                                step or an evaluation that synchronises; the context then refuses
                                every call that would use its state until a system is set again */
    RBSOG_E_CAPACITY = -9    /* a per-cell or per-atom capacity was exceeded */
} rbsog_status;

typedef enum { RBSOG_FP64 = 0, RBSOG_MIXED = 1 } rbsog_precision;

/* rbsog_params.flags bits.
 * RBSOG_FLAG_SHELL_STORED: the memory form of the random batch list
 *   (Section 2.4 bounds the per-atom list at O(core + P_R) entries).  The
 *   shell batch of each atom (eq. 25) is drawn when the lists are built and
 *   kept until the next build, instead of being drawn afresh at every force
 *   evaluation: Floyd's selection on the Philox stream (atom id, build
 *   number, tag 5, replica), builds numbered from 0 since the system was set
 *   (a build that overflowed and is redone keeps its number).  The library
 *   then keeps per atom the core list and P_R batch entries; candidate rows
 *   exist only during the build, one chunk of cells at a time (see
 *   rbsog_set_list_chunks).  Each evaluation still masks the batch to
 *   r_core <= r < r_shell at the current positions and weights it by
 *   N_shell/P_R (N_shell = candidate count at the build).  Needs p_r >= 1. */
#define RBSOG_FLAG_SHELL_STORED 1u
/* RBSOG_FLAG_INT_PHASE (FP32-mixed form only): the phase k.r of the
 * structure factors and the k-space force (eqs. 22, 29) is reduced in 32-bit
 * fixed point (Section 2.4 names fixed-point phases as an implementation
 * choice): each position is held as the fraction u = floor(2^32 x / L) of the
 * box, the phase m.u of an integer mode m wraps exactly modulo 2^32 (one
 * turn), and its signed value times 2^-32 is the FP32 turn given to the
 * hardware sine and cosine.  Without the flag the phase is formed in FP64
 * and its fractional turn rounded to FP32.  Both are within the mixed form's
 * error; the flag is equal across a batch. */
#define RBSOG_FLAG_INT_PHASE 2u

typedef struct {
    double q;    /* charge, e */
    double mass; /* amu */
} rbsog_species;

/* Born-Mayer-Huggins pair parameters of eq. (1):
 * U_B(r) = A exp((sigma - r)/rho) - C/r^6 - D/r^8. */
typedef struct {
    double A, sigma, rho, C, D;
} rbsog_pair;

typedef struct {
    int32_t n_atoms;
    int32_t n_species;                          /* 1..RBSOG_MAX_SPECIES */
    double box[3];                              /* orthorhombic, origin 0 */
    rbsog_species species[RBSOG_MAX_SPECIES];
    rbsog_pair pair[RBSOG_MAX_SPECIES * RBSOG_MAX_SPECIES]; /* [i*MAX + j], symmetric */
    double r_core;     /* RBL core radius (eq. 24) */
    double r_shell;    /* RBL shell radius (eq. 25); also the SOG cutoff r_c (eqs. 8-10) */
    double skin;       /* list skin; lists hold r < r_core+skin and
                          r_core-skin <= r < r_shell+skin */
    int32_t p_r;       /* shell batch size P_R; <= 0: every candidate, weight 1 */
    int32_t p_f;       /* Fourier batch size P_F; <= 0: full k-sum of eq. (23) */
    double sog_eps;    /* target of the eq. (5) bound; <= 0 means 1e-5 */
    double dt;         /* ps */
    int32_t rebuild_every; /* list rebuild period in steps (>= 1) */
    int32_t precision;     /* rbsog_precision */
    uint64_t seed;         /* Philox key */
    uint32_t replica;      /* Philox stream id of this system */
    uint32_t flags;        /* RBSOG_FLAG_* bits (others must be 0); equal across a batch */
    double coulomb_k;      /* e^2/(4 pi eps0) in eV*Angstrom; <= 0 means 14.399645478 */
    double t_target;       /* K; a thermostat acts when t_target > 0 and tau_t > 0, else NVE */
    double tau_t;          /* ps; coupling time of the thermostat (see `thermostat`) */
    int32_t thermostat;    /* RBSOG_THERMO_*; systems of a batch may differ */
    int32_t reserved;      /* 0 */
    double r_core_pair[RBSOG_MAX_SPECIES * RBSOG_MAX_SPECIES];
                           /* species-dependent core radii (Section 1 names the strategy, no rule):
                              [i*MAX + j] symmetric, 0 < r < r_shell, or 0 = r_core.  A pair inside
                              its own core radius is summed in full (eq. 24), outside it up to
                              r_shell it is a shell candidate (eq. 25); lists use the pair's
                              radius with the skin.  Equal across a batch. */
} rbsog_params;

/* Thermostats (rbsog_params.thermostat), with T from the kinetic energy and
 * g = 3N - 3 degrees of freedom.  The paper's runs are NVT (Section 3) and
 * its trajectory estimate (Theorem 2.3) is stated for Langevin dynamics;
 * it prints neither integrator, so these are the textbook forms.
 * BERENDSEN: v <- lambda v at the start of each step, lambda^2 =
 *   1 + (dt/tau_t)(t_target/T - 1); tau_t = dt rescales to t_target exactly.
 * NOSE_HOOVER: one thermostat variable xi with mass Q = g k_B t_target
 *   tau_t^2, advanced by Trotter half steps before the opening kick and
 *   after the closing kick (Martyna, Tuckerman, Klein 1996); the conserved
 *   extended energy is u_total + kinetic + e_thermostat.
 * LANGEVIN: BAOAB splitting (Leimkuhler, Matthews 2013), friction 1/tau_t:
 *   the drift becomes r += dt/2 v; v = c1 v + c2 z; r += dt/2 v with
 *   c1 = exp(-dt/tau_t), c2 = sqrt((1 - c1^2) k_B t_target / m) and z three
 *   standard normals per atom by Box-Muller from four 53-bit uniforms of the
 *   Philox stream (atom id, step number, tag 6, replica). */
#define RBSOG_THERMO_BERENDSEN 0
#define RBSOG_THERMO_NOSE_HOOVER 1
#define RBSOG_THERMO_LANGEVIN 2

typedef struct {
    double u_core;    /* core-list energy, sum over r < r_core of N + B_BMH (eqs. 13-14, 24) */
    double u_shell;   /* shell estimate, (N_shell/P_R) times the batch sum (eq. 25) */
    double u_kspace;  /* U*_F of eq. (18), estimated with the sampled modes */
    double u_self;    /* U_self of eq. (18) */
    double u_total;   /* u_core + u_shell + u_kspace - u_self */
    double kinetic;
    double p_corr[3]; /* momentum correction F_corr of eq. (26) that was subtracted */
    double max_disp;  /* largest displacement since the last list build */
    int64_t n_builds; /* list builds since the system was set */
    double e_thermostat; /* Nose-Hoover: Q v_xi^2 / 2 + g k_B t_target xi; else 0 */
    double virial[6];    /* W_ab = -dU/de_ab (xx, yy, zz, xy, xz, yz), eV, with positions and box
                            strained together: half the sum of r_ij (x) F_ij over core pairs plus
                            N_shell/P_R times the same over the shell batch (eqs. 24-25), and per
                            k-space mode (k_e/2) e_k (delta_ab - g(k) k_a k_b) with e_k the mode's
                            energy weight (eq. 23 or 29) and g = -F^'(k)/(k F^(k)) (eq. 21), so the
                            sampled form is unbiased for the full sum.  The momentum correction
                            (eq. 26) is not included.  Pressure tensor: P_ab V = sum_i m v_a v_b
                            + W_ab. */
    double stress[6];    /* S_ab of eq. (50), eV: sum_i m v_a v_b + W_ab, same order as virial,
                            with the velocities at the end of the call (after a step's closing
                            thermostat half step) */
    double heat_flux[3]; /* J of eq. (51), eV / (A^2 ps), at the same velocities:
                            (1/V) sum_i (e_i v_i + W_i v_i).  e_i = m v_i^2 / 2 plus the ion's
                            share of the potential energy: half of each core pair energy, the
                            shell batch's half pair energies times N_shell/P_R, the share
                            (k_e/2) q_i coef Re(e^{-ik.r_i} rho) of each k-space mode, less
                            k_e q_i^2 sum_m w_m / 2; W_i the ion's share of the virial, alike
                            (per mode times delta_ab - g k_a k_b).  For pairs, sum_i W_i v_i is
                            the pair term of eq. (51). */
} rbsog_energy;

/* Library version string. */
const char* rbsog_version(void);

/* SOG split of eqs. (4)-(10) for a target eps (eq. 5 bound) and cutoff
 * r_c = r_shell, computed on the host: base b, bandwidth s, x_c = r_c/s,
 * series length M (m = 0..M) and weights w[0..M] (w[0] adjusted for C1
 * continuity).  w may be NULL; otherwise it must hold w_cap >= M+1 values.
 * Needs no GPU. */
rbsog_status rbsog_sog_params(double eps, double r_shell, double* b, double* s, double* x_c,
                              int32_t* M, double* w, int32_t w_cap);

/* FP32 near-field table the mixed form evaluates the SOG Coulomb kernels
 * from (Section 2.4: near field by table lookup indexed by the bits of
 * r^2), for the split of (eps, r_shell): binades of s = r^2 from 2^e0 up to
 * past r_shell^2, 64 intervals each (interval index = exponent and six
 * leading mantissa bits of s), *n_intervals in all; per interval eight
 * floats, the cubic Hermite coefficients (ascending powers of t = s - the
 * interval's start) of CF(s) = -N'(r)/r and of CU(s) = N(r) (eqs. 8, 14-15;
 * pair force k_e q_i q_j CF r_ij, energy k_e q_i q_j CU).  coef may be NULL;
 * otherwise it must hold cap >= 8 * n_intervals floats.  Needs no GPU. */
rbsog_status rbsog_near_table(double eps, double r_shell, float* coef, int32_t cap, int32_t* e0,
                              int32_t* n_intervals);

/* Create a context on HIP device `hip_device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  Every call's device work is
 * ordered on that stream: work the library puts on its own second stream is
 * forked from and joined back to it with events. */
rbsog_status rbsog_create(rbsog_ctx** out, int hip_device, void* hip_stream);
rbsog_status rbsog_destroy(rbsog_ctx* ctx);
const char* rbsog_last_error(const rbsog_ctx* ctx);

/* Validate parameters (neutrality, box >= 2(r_shell+skin), species count,
 * fewer than 2^28 atoms per system: the cell sort keys and the staged list
 * entries keep the atom index in 28 bits),
 * set up the SOG split and the k-space sampling tables (eq. 28) and copy
 * type[N], pos[N][3] and vel[N][3] (vel may be NULL = zero) into device
 * memory.  Pointers are device pointers if ptrs_on_device != 0, else host.
 * Builds the lists.  Synchronises.  Replaces any system or batch the context
 * held; equivalent to rbsog_set_batch with one system. */
rbsog_status rbsog_set_system(rbsog_ctx* ctx, const rbsog_params* p, const int32_t* type,
                              const double* pos, const double* vel, int ptrs_on_device);

/* Batched form: n_sys independent systems (replicas, Section 2.2 applied to
 * each) held by one context and advanced together, every kernel launch
 * covering all of them.  p[n_sys] gives each system's parameters; n_atoms,
 * box, p_r, p_f, seed, replica, t_target and tau_t may differ, every other
 * field must be equal across the batch (else RBSOG_E_ARG).  type, pos and
 * vel hold the systems' rows one after another.  Each system is evaluated
 * exactly as it would be alone in its own context (same lists, shell
 * batches, modes and reduction order), so its results equal a single-system
 * run with the same parameters.  Synchronises. */
rbsog_status rbsog_set_batch(rbsog_ctx* ctx, int32_t n_sys, const rbsog_params* p, const int32_t* type,
                             const double* pos, const double* vel, int ptrs_on_device);
/* Number of systems held (1 after rbsog_set_system). */
rbsog_status rbsog_n_systems(rbsog_ctx* ctx, int32_t* n_sys);
/* Choose the system (0 <= r < n_sys) that the parity exports below
 * (list counts, lists, shell ranks, modes, rho) refer to; 0 after a set. */
rbsog_status rbsog_select_system(rbsog_ctx* ctx, int32_t r);

/* Rebuild the cell order and the core/shell-candidate lists at the current
 * positions (Section 2.2 core-shell lists). */
rbsog_status rbsog_build_lists(rbsog_ctx* ctx);

/* Replace the positions of every atom (pos[N][3], user order; device pointer
 * if ptrs_on_device != 0, else host), for a caller that moves the atoms with
 * its own integrator and asks for forces (Section 2.2 evaluates the force at
 * given positions).  Positions are wrapped into the box; velocities and lists
 * are kept.  If an atom is now more than skin/2 from its position at the last
 * list build, the lists no longer hold every pair within r_shell (eqs.
 * 24-25): rbsog_compute_forces then returns RBSOG_E_LIST_STALE until
 * rbsog_build_lists, and rbsog_step builds first (counted in n_builds).
 * Non-finite input: RBSOG_E_NONFINITE, nothing changed.  Synchronises. */
rbsog_status rbsog_set_positions(rbsog_ctx* ctx, const double* pos, int ptrs_on_device);

/* One IRBSOG force evaluation at the current positions with Philox counter
 * `eval` (shell batches of eq. 25, modes of eq. 28): F = F_core + F*_shell -
 * F_corr + F*_F (eqs. 24-27, 29), for every system held.  Writes the force
 * in user order to the device array force_out[N][3] if non-NULL.  Energies
 * are returned in e_out[n_sys] (one record per system) if non-NULL (the call
 * then synchronises and returns RBSOG_E_NONFINITE if a force is not
 * finite).  Does not move atoms.  RBSOG_E_LIST_STALE after
 * rbsog_set_positions moved an atom more than skin/2 since the last build. */
rbsog_status rbsog_compute_forces(rbsog_ctx* ctx, uint64_t eval, double* force_out, rbsog_energy* e_out);

/* Force parts of the last evaluation in user order into device arrays
 * [N][3] (any may be NULL): short range before the momentum correction
 * (eqs. 24-25), and the k-space part (eq. 29). */
rbsog_status rbsog_get_force_parts(rbsog_ctx* ctx, double* f_short, double* f_kspace);

/* n_steps velocity-Verlet steps: kick, drift (wrap), list rebuild when the
 * step number is a multiple of rebuild_every or an atom has moved more than
 * skin/2 since the last build (decided on the device), force with eval =
 * step number, kick.  Each system of a batch decides its own rebuilds.
 * e_last[n_sys] (may be NULL) receives the energies of the last step; the
 * call synchronises at the end and returns RBSOG_E_NONFINITE if a position
 * or force of any step was not finite (such a system is not rebuilt in the
 * meantime). */
rbsog_status rbsog_step(rbsog_ctx* ctx, int32_t n_steps, rbsog_energy* e_last);

/* The batched form's step call (Section 2.2 applied to every system held):
 * rbsog_step without energies, each step replayed from a captured HIP graph
 * (captured on first use per variant, as with rbsog_use_graphs) whatever the
 * rbsog_use_graphs setting; the same bits as rbsog_step.  Needs a context
 * created on a non-default stream (else RBSOG_E_STATE).  Synchronises. */
rbsog_status rbsog_step_batch(rbsog_ctx* ctx, int32_t n_steps);

/* Current positions, velocities, forces (user order, [N][3]) and the eval
 * index of the last force evaluation.  Pointers are device pointers if
 * ptrs_on_device != 0, else host (then the call synchronises).  Any may be
 * NULL. */
rbsog_status rbsog_get_state(rbsog_ctx* ctx, double* pos, double* vel, double* force, uint64_t* eval,
                             int ptrs_on_device);

/* ---- launch shapes and step graphs -------------------------------------- */

/* Per-atom list capacities (entries; one is kept as a write sink, so a list
 * holds at most cap - 1): replan the lists with these capacities and build
 * them at the current positions (a new list build).  A build that later
 * overflows them grows them again (rbsog_step restarts its call from the
 * state at its start).  got_core / got_cand (may be NULL) receive the
 * capacities in force after the build.  8..4096.  Synchronises. */
rbsog_status rbsog_set_list_capacity(rbsog_ctx* ctx, int32_t cap_core, int32_t cap_cand, int32_t* got_core,
                                     int32_t* got_cand);

/* Memory form (RBSOG_FLAG_SHELL_STORED): build the lists in `chunks`
 * launches over consecutive ranges of cells (1..64, default 8; a system
 * with fewer cells uses one chunk per cell), so the candidate rows exist for
 * about 1/chunks of the atoms at a time.  No choice changes a result bit.
 * Applies to the systems set by later rbsog_set_system / rbsog_set_batch
 * calls.  Needs no GPU work. */
rbsog_status rbsog_set_list_chunks(rbsog_ctx* ctx, int32_t chunks);

/* Launch shapes of the hot kernels and the stream of the k-space force.  No
 * choice changes a result bit: partial sums are taken per 64-atom wavefront
 * and every structure factor is summed over the atoms in the same order
 * whatever the shape. */
typedef struct {
    int32_t pair_block; /* atoms per workgroup of the pair kernel: 64, 128, 256 (default 256) */
    int32_t pair_ku;    /* neighbour positions fetched ahead per lane (shell-batch tile): 4, 8 (4) */
    int32_t rho_mpl;    /* k-modes per lane of the rho kernel (64 rho_mpl per workgroup): 1, 2 (1) */
    int32_t kf_block;   /* atoms per workgroup of the k-space force kernel: 64, 128, 256 (256) */
    int32_t kf_aux;     /* 1: the k-space force follows rho on the second stream, beside the pair
                           kernel; 0: it runs after the pair kernel on the context's stream (1) */
} rbsog_tuning;

/* Choose the launch shapes by timing from the current state (HIP events on
 * the context's stream): the k-space force workgroup alone, then every
 * combination of pair_block, pair_ku, rho_mpl and kf_aux on whole steps
 * (both streams, graphs if enabled), max(reps, 3) steps per candidate from
 * one saved device state, best of three alternating rounds; the chosen
 * shapes are returned in `chosen` (may be NULL).  Restores the saved state
 * (positions, velocities, forces, lists, counters), so the trajectory that
 * follows is bit for bit the one without tuning; holds a second copy of the
 * atom and list arrays while it runs.  Synchronises. */
rbsog_status rbsog_autotune(rbsog_ctx* ctx, int32_t reps, rbsog_tuning* chosen);
/* Set or read the shapes directly (values outside the lists: RBSOG_E_ARG). */
rbsog_status rbsog_set_tuning(rbsog_ctx* ctx, const rbsog_tuning* t);
rbsog_status rbsog_get_tuning(rbsog_ctx* ctx, rbsog_tuning* t);
/* With enable != 0, rbsog_step replays each step as one captured HIP graph
 * (captured on first use per variant: scheduled rebuild or not, energies or
 * not; recaptured after list growth or a tuning change).  Needs the context
 * to have a non-default stream; while phase timing is on, steps are launched
 * kernel by kernel.  Off by default. */
rbsog_status rbsog_use_graphs(rbsog_ctx* ctx, int enable);

/* ---- kernel timing ------------------------------------------------------ */

/* Kernel phases timed with HIP events on the stream their kernels run on:
 * the context's stream, or for KSAMPLE, RHO and KFORCE a second stream of
 * the context on which the k-space chain runs beside the pair kernel (so
 * phase times can add up to more than the step). */
typedef enum {
    RBSOG_PHASE_BUILD = 0,     /* cell sort + list build */
    RBSOG_PHASE_KSAMPLE = 1,   /* mode draws of eq. (28) */
    RBSOG_PHASE_PAIR = 2,      /* shell batch + pair forces, eqs. (15), (24)-(25) */
    RBSOG_PHASE_RHO = 3,       /* structure factors, eq. (22), and their fixed-order reduction */
    RBSOG_PHASE_REDUCE = 4,    /* fixed-order reductions: momentum correction, energies */
    RBSOG_PHASE_KFORCE = 5,    /* k-space force, eq. (29); with kf_aux = 0 fused with the total
                                  force (eqs. 26-29) and the closing half kick */
    RBSOG_PHASE_INTEGRATE = 6, /* opening half kick + drift; with kf_aux = 1 also the total force
                                  (eqs. 26-29) and the closing half kick */
    RBSOG_N_PHASES = 7
} rbsog_phase;

/* Per-phase event timing (off by default).  enable = 1: every phase launched
 * is bracketed by two HIP events; 2: only the pair, rho and k-space force
 * phases (the hot kernels; fewer events disturb the timing less); 0: off.
 * While on, steps run kernel by kernel (no graphs). */
rbsog_status rbsog_profile_enable(rbsog_ctx* ctx, int enable);
/* Synchronise, add up the timed phases since the last read and reset:
 * ms[RBSOG_N_PHASES] total milliseconds, launches[RBSOG_N_PHASES] counts. */
rbsog_status rbsog_profile_read(rbsog_ctx* ctx, double* ms, int64_t* launches);

/* ---- parity exports (host outputs, synchronise) ----------------------- */
/* These refer to the system chosen by rbsog_select_system; atom ids are that
 * system's own (0..n_atoms-1). */

/* Core and candidate list sizes n_core[N], n_cand[N]. */
rbsog_status rbsog_get_list_counts(rbsog_ctx* ctx, int32_t* n_core, int32_t* n_cand);
/* Lists of atom i: core neighbour ids ascending; candidate ids in the
 * canonical order the shell ranks refer to: by cell (grid of
 * n_c = 2 floor(L/(r_shell+skin)) cells per axis, one where
 * floor(L/(r_shell+skin)) is below 3; cell index floor(x n_c/L) with x
 * fastest), then by id.  With RBSOG_FLAG_SHELL_STORED the candidate lists
 * are not kept: cand must be NULL (else RBSOG_E_STATE). */
rbsog_status rbsog_get_lists_of(rbsog_ctx* ctx, int32_t i, int32_t* core, int32_t* cand);
/* Shell batch ranks (indices into the ordered candidate list, ascending)
 * of every atom for evaluation `eval`: ranks[N][P_R]; unused slots are -1.
 * n_ranks[N] gets min(P_R, n_cand).  Not available with
 * RBSOG_FLAG_SHELL_STORED (RBSOG_E_STATE). */
rbsog_status rbsog_get_shell_ranks(rbsog_ctx* ctx, uint64_t eval, int32_t* n_ranks, int32_t* ranks);
/* Shell samples of eq. (25) in use for the selected system: with a batch
 * drawn every evaluation, the batch of the last force evaluation (its eval
 * index); with RBSOG_FLAG_SHELL_STORED, the batch drawn at the last list
 * build.  idx[N][P_R] (host, may be NULL) receives per atom the neighbour ids
 * of the batch sorted ascending, -1 past min(P_R, n_cand); n_cand[N] (host,
 * may be NULL) the candidate count N_shell that weights it (N_shell/P_R when
 * N_shell > P_R).  Needs P_R >= 1 and, without a stored batch, a force
 * evaluation since the system was set (else RBSOG_E_STATE). */
rbsog_status rbsog_get_shell_samples(rbsog_ctx* ctx, int32_t* n_cand, int32_t* idx);
/* With RBSOG_FLAG_SHELL_STORED (else RBSOG_E_STATE): the batch drawn at the
 * last list build as atom ids in ascending rank order, ids[N][P_R] (-1 past
 * min(P_R, n_cand)), and the candidate count N_shell of each atom at that
 * build, n_cand[N].  Either may be NULL. */
rbsog_status rbsog_get_shell_batch(rbsog_ctx* ctx, int32_t* n_cand, int32_t* ids);
/* Radial distribution counts of the selected system at its current positions
 * (the pair histogram behind the RDF g_ab(r) of Section 3.1):
 * counts[(a S + b) n_bins + k] (host, S = n_species, S*S*n_bins entries,
 * overwritten) = ordered pairs i != j of species (a, b) whose minimum-image
 * r^2 satisfies e_k <= r^2 < e_{k+1}, e_k = (k D)(k D) in FP64 with
 * D = r_max / n_bins.  Taken from the lists (every pair within r_shell
 * appears in them), so r_max <= r_shell, and S*S*n_bins <= 16384; else
 * RBSOG_E_ARG.  The memory form keeps no candidate rows: RBSOG_E_STATE.
 * g_ab(r) = counts / (N_a (N_b - delta_ab) / V * shell volume).
 * Synchronises. */
rbsog_status rbsog_rdf_counts(rbsog_ctx* ctx, double r_max, int32_t n_bins, uint64_t* counts);
/* rbsog_rdf_counts for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same counts, with the device histogram kept in a
 * file-scope device array of 16384 counters per GPU (its address looked up
 * once per device at rbsog_create) instead of a buffer allocated per call;
 * no hipMalloc or hipFree.  S*S*n_bins above 16384: RBSOG_E_ARG.  Every call
 * on one GPU shares that array: calls that overlap on one GPU (two host
 * threads, two contexts) race; the array is cleared by the call itself.
 * Enqueues on the context's stream, copies into the host array counts and
 * synchronises. */
rbsog_status rbsog_rdf_counts_noalloc(rbsog_ctx* ctx, double r_max, int32_t n_bins, uint64_t* counts);
/* Mean-square displacement of the selected system (the MSD of Section 3.1),
 * per species, from an origin the caller marks.  mark != 0: the origin is the
 * current positions (each ion's unwrapped displacement D_i restarts at 0).
 * mark == 0: D_i gains the minimum-image displacement since the previous call
 * and msd[a] (host, n_species entries, may be NULL) = mean of |D_i|^2 over
 * the ions of species a (0 for a species with none), A^2.  Unwrapping is
 * exact while no ion moves half a box length between two calls (call every
 * few hundred steps at most in a melt).  RBSOG_E_STATE without a marked
 * origin; a new rbsog_set_system/batch forgets it.  Device memory: six
 * doubles per ion, kept.  Synchronises. */
rbsog_status rbsog_msd(rbsog_ctx* ctx, int32_t mark, double* msd);
/* The P_F modes m[P_F][3] drawn for evaluation `eval` and S of eq. (28). */
rbsog_status rbsog_get_kmodes(rbsog_ctx* ctx, uint64_t eval, int32_t* m, double* S);
/* Structure factors rho[P_F][2] (eq. 22) of the last force evaluation. */
rbsog_status rbsog_get_rho(rbsog_ctx* ctx, double* rho);
/* SOG split in use (see rbsog_sog_params). */
rbsog_status rbsog_get_sog(rbsog_ctx* ctx, double* b, double* s, double* x_c, int32_t* M, double* w,
                           int32_t w_cap);

#ifdef __cplusplus
}
#endif
#endif
