// Device data of the systems of a batch and the kernel launchers (defined in
// kernels.hip).  A single system is a batch of one.
#pragma once

#include "common.hpp"

namespace rbsog {

// Mode record read with one 64-byte scalar load in the k-space force kernel.
struct ModeRec {
    double mx, my, mz;  // integer mode vector as doubles
    double A, B;        // coef * Im rho, coef * Re rho
    double coef;        // S/(P_F V k^2), or F^(k)/V for the full sum
    double e;           // coef * |rho|^2
    float Af, Bf;       // A and B rounded to FP32 (mixed force kernel)
};

// Per-species constants, indexed by atom type.
struct SpeciesDev {
    double q[kMaxSpecies];
    double inv_mass_acc[kMaxSpecies];  // kAccUnit / m
    double mass[kMaxSpecies];
    double self_e[kMaxSpecies];  // k_e q^2 sum_m w_m / 2, the self term of one ion
};

// Everything the kernels read or write about one system of a batch.  Per-atom
// arrays are this system's slices of the batch arrays, in cell order, and
// every atom, cell and list index is local to the system.
struct DevSys {
    int n;
    int n_species;
    int user_off;          // first row of this system in the caller's [N][3] arrays
    double L[3], invL[3];
    double cell_scale[3];  // n_c / L
    int nf[3];             // ordering grid: 2 n_c cells per axis (1 where n_c = 1)
    double fine_scale[3];  // n_f / L
    int nc[3];
    int ncell;
    double two_pi_L[3];
    double rc2_list, lo2_list, hi2_list;  // (r_core+skin)^2, (r_core-skin)^2, (r_shell+skin)^2
    double rc2, rs2;                      // r_core^2, r_shell^2
    // bound on |r^2 from the fixed-point records - r^2 of the FP64 minimum
    // image| (A^2): pairs closer than this to a cutoff are decided in FP64
    double fix_guard;
    int species_cut;       // core radii differ between species pairs (PairCoef rc2, rc2_list, lo2_list)
    double half_skin2;
    // atoms with inner_lo <= x <= inner_hi on every axis have no list
    // neighbour across the box edge (empty range where the box is short)
    double inner_lo[3], inner_hi[3];
    double dt, coulomb_k;
    double thermo_c;       // dt / tau_t (0: no thermostat)
    double t_target;
    double dof_kb;         // (3N - 3) k_B
    int thermostat;        // kThermo* (meaningful when thermo_c > 0)
    double nh_q;           // Nose-Hoover mass g k_B T0 tau^2
    double lv_c1;          // Langevin exp(-dt / tau)
    double lv_c2[kMaxSpecies];  // Langevin sqrt((1 - c1^2) k_B T0 / m) per species, A/ps
    int p_r;
    int cap_core, cap_cand;
    // Memory form of the list (shell_stored): the shell batch is drawn at the
    // build into bat_idx and kept; candidate rows are build scratch for one
    // chunk of cells at a time (n_chunks chunks, cand_rows rows).  Otherwise
    // n_chunks = 1 and cand_idx holds a row per atom.
    int shell_stored;
    // [n] positions as 32-bit fractions of the box (floor(x/L 2^32)) and the
    // type, rewritten wherever p is: the 16-byte neighbour records of the
    // mixed pair kernel and the integer k-space phase
    uint4* ufix;
    // workgroups per list cell in the list build: a cell with many atoms (a
    // small box that is one list cell per axis) is split over several
    int list_parts;
    int n_chunks;
    int cand_rows;
    uint32_t replica;
    uint64_t seed;
    const struct SpeciesDev* spc;  // per-species constants (shared by a batch)

    // atoms (cell order); positions packed with the species so a neighbour
    // gather touches one 32-byte record
    double4* p;               // x, y, z, type (as a double)
    double *vx, *vy, *vz;
    double *fx, *fy, *fz;     // total force of the last evaluation
    double *fsx, *fsy, *fsz;  // short-range force before the momentum correction
    double *xr, *yr, *zr;     // positions at the last list build
    int32_t *type, *id, *inv;
    // sort scratch
    double4* tp;
    double *tvx, *tvy, *tvz, *tfx, *tfy, *tfz;
    int32_t *ttype, *tid, *cell_of, *slot_of, *order;
    int32_t *cell_count, *cell_start;
    // [ncell][8]: first position, within its list cell, of each of the
    // cell's eight ordering-grid sub-cells (x fastest); the cell sort keeps
    // each sub-cell's atoms contiguous, in index order
    int32_t* sub_beg;
    // lists
    int32_t *core_cnt, *core_idx, *cand_cnt, *cand_idx;
    int32_t* bat_idx;      // [ceil(n/64)][p_r][64] stored shell batch (sorted atom indices)
    // pair coefficients [S*S]
    const PairCoef* pair;
    DeviceScalars* sc;
    double* pair_part;     // [ceil(n/64)][kPairPart] wavefront partials of the pair kernel
    double* vir_part;      // [ceil(n/64)][kVirPart] wavefront virial partials (evaluations with energies)
    double* fin_part;      // [kFinBlocks][kFin] per-block sums of the evaluation's force-sum reduction
    double* kin_part;      // [ceil(n/64)] kinetic-energy wavefront partials
    double* flux_part;     // [ceil(n/64)][kFluxPart] kinetic tensor and heat-flux partials
    double4* at_ew;        // [n][2] per-atom short-range energy and virial shares of the
                           // last evaluation with energies: {e, W_xx, W_yy, W_zz}, {W_xy, W_xz, W_yz, 0}
};

struct KDev {
    int n_modes;          // P_F, or the enumerated count
    int sampled;          // 1: modes drawn each evaluation from the tables
    int n_chunks;         // atom chunks of the rho kernel
    int chunk;            // atoms per chunk
    int nm;               // Gaussians in the sampling tables
    double S;
    double coef_scale;    // S / (P_F V)
    const double* table;  // sincos table [1024][2]
    const int32_t* off;
    const int32_t* len;
    const double* g0cdf;
    const double* g2cdf;
    const double* comp_cdf;
    int32_t* m;           // [n_modes][3]
    ModeRec* modes;       // [n_modes]
    double* rho_part;     // [n_chunks][n_modes_pad][2]
    int n_modes_pad;
    double* rho;          // [n_modes][2]
    int n_sog;            // terms of F^(k): c[m] exp(-s2[m] k^2 / 2), m < n_sog
    const double* sog_c;
    const double* sog_s2;
    double* mode_g;       // [n_modes] g = G/F^ of each mode (strain derivative), set by the
                          // finalize of evaluations with energies
};

// Per-wavefront partial sums written by the pair kernel: F (3), u_core,
// u_shell; and, in evaluations with energies, the virial W (6) in vir_part.
constexpr int kPairPart = 5;
constexpr int kVirPart = 6;
// The reduction of those partials and of the modes' energies runs in two
// passes: fin_blocks(n) blocks per system (one per 256 wavefront partials,
// at most kFinBlocks), each over a fixed slice, then one wavefront per
// system adding their kFin sums in block order.  The slicing depends on the
// system's own size only, so a system sums in the same order alone and in a
// batch.
constexpr int kFinBlocks = 32;
constexpr int kFin = kPairPart + kVirPart + 1 + 6;  // pair sums, virial, mode energy, mode virial
constexpr int fin_blocks(int n)
{
    const int b = ((n + 63) / 64 + 255) / 256;
    return b < 1 ? 1 : (b > kFinBlocks ? kFinBlocks : b);
}
// Per-wavefront partials of the closing pass of an evaluation with energies:
// sum m v_a v_b (6), sum (m v^2 / 2) v (3), sum (e_i v + W_i v) (3).
constexpr int kFluxPart = 12;

// The grid of one launch over a batch: block b works on local block map[b].y
// of system map[b].x.  A null map means one system (system 0, local block b).
struct Shape {
    const int2* map = nullptr;
    int blocks = 0;
};

// Launch shapes chosen by the autotuner.  None of them changes a result bit:
// partial sums are per wavefront and each mode's sum runs in the same order.
struct Tuning {
    int pair_block = 256;  // atoms per pair-kernel workgroup (64, 128, 256)
    int pair_ku = 4;       // neighbours fetched ahead in the pair kernel (4, 8)
    int rho_mpl = 1;       // modes per lane in the rho kernel (1, 2)
    int kf_block = 256;    // atoms per k-space force workgroup (64, 128, 256)
    int kf_aux = 1;        // k-space force on the second stream (1) or after the pair kernel (0)
};

// FP32 near-field table of the mixed pair kernel (built on the host, shared
// by a batch): interval idx = (bits(r^2) >> 17) - lo, valid below n; per
// interval two float4: CF and CU cubic coefficients in t = r^2 - start.
struct NearTab {
    const float4* coef = nullptr;
    int lo = 0;
    int n = 0;  // 0: no table, the kernel evaluates the near field directly
};

// Staging capacities of the per-cell list kernel (atoms of a 27-cell stencil
// held in LDS): the smallest fits three workgroups in a CU's LDS; a build
// whose stencil overflows moves to the next; past the last, the per-atom
// kernel.
constexpr int kListCaps[3] = {1600, 2048, 4096};
constexpr int kListPerAtom = 3;

// Launch plan of a batch (or of one system of it, see api.cpp).
struct Plan {
    const DevSys* sys = nullptr;  // device array [R]
    const KDev* kd = nullptr;     // device array [R]
    DeviceScalars* sc = nullptr;  // device array [R] (sys[r].sc == sc + r)
    int R = 0;
    Shape atoms;    // 256-atom blocks of every system
    Shape pair_atoms;  // tune.pair_block-atom blocks (pair kernel)
    Shape kf_atoms;    // tune.kf_block-atom blocks (k-space force kernel)
    Shape cells;    // one block per cell
    Shape list_cells;  // list_parts blocks per cell (list build)
    // the same cells grouped by the staging capacity kListCaps[q] of their
    // system (a batch mixes small boxes, whose stencil is most of the box,
    // with large ones); used unless the build is chunked or per atom
    Shape list_by_cap[kListPerAtom];
    Shape cell_chunk[kMaxListChunks];  // the cells of each build chunk (memory form)
    Shape rows64;   // 64-row blocks over each system's candidate rows (batch draw)
    Shape atom1;    // one block per atom (per-atom list kernel)
    Shape modes64;  // 64-mode blocks of the systems that draw modes
    Shape rho;      // rho blocks: local block = mode tile * n_chunks + chunk (tiles of 64 rho_mpl modes)
    Shape modes1;   // one block per mode
    int list_mode = 0;  // < kListPerAtom: per-cell list kernel staging kListCaps[mode] atoms; else per-atom kernel
    bool stored = false;  // memory form: batch drawn at the build
    bool langevin = false;  // some system runs the Langevin thermostat
    bool iph = false;       // mixed form: k-space phases in 32-bit fixed point
    bool species_cut = false;  // species-dependent core radii
    int n_chunks = 1;     // build chunks (1 unless stored)
    int fin_grid = 1;     // largest fin_blocks over the systems (blocks per system of the first pass)
    int cap_core = 0, cap_cand = 0;
    NearTab near;
    Tuning tune;
};

void launch_set_eval(const Plan& P, uint64_t eval, hipStream_t st);
// start of a step: eval index + 1, and the opening Nose-Hoover half step
void launch_step_begin(const Plan& P, hipStream_t st);
// scalars that start at 1 (velocity factors), after the scalars are zeroed
void launch_init_scalars(const Plan& P, hipStream_t st);
void launch_clear_flags(const Plan& P, hipStream_t st);

// cell sort + lists; with gate the kernels of a system run only when its
// device-side rebuild flag is up (and lower it at the end)
void launch_build(const Plan& P, bool gate, hipStream_t st);
// the two halves of launch_build: the cell sort (atoms reordered), then the
// lists (which read the sorted positions and write only list data)
void launch_sort(const Plan& P, bool gate, hipStream_t st);
void launch_lists(const Plan& P, bool gate, hipStream_t st);

// forces
void launch_ksample(const Plan& P, hipStream_t st);
void launch_pair(const Plan& P, const SogCoef& sog, bool mixed, bool energy, hipStream_t st);
void launch_rho(const Plan& P, bool mixed, hipStream_t st);
void launch_rho_finalize(const Plan& P, hipStream_t st);
// momentum correction and energies; with `energy` also the virial
void launch_finalize(const Plan& P, bool energy, hipStream_t st);
// k-space force (eq. 29) into the total-force arrays
void launch_kforce(const Plan& P, bool mixed, hipStream_t st);
// total force = short range - momentum correction + k-space; with kick the
// closing half kick; with energy the kinetic-energy partials
void launch_combine(const Plan& P, bool kick, bool energy, hipStream_t st);
// the k-space force and the combine in one pass (no second stream).  ke: 0
// no partials, 1 kinetic-energy partials, 2 those and the per-atom k-space
// shares combined with the pair kernel's into stress and heat-flux partials
// (evaluations with energies)
void launch_kforce_fused(const Plan& P, bool mixed, bool kick, int ke, hipStream_t st);
// kinetic energy from the partials; with a thermostat also the velocity
// factor of the next step.  step_end: the partials are those of a step's
// closing kick (the Nose-Hoover closing half step is taken), else a
// measurement of the current velocities.  flux: also the stress and heat flux
void launch_kinetic_finalize(const Plan& P, bool step_end, bool flux, hipStream_t st);
// kinetic-energy partials of the current velocities
void launch_kinetic(const Plan& P, hipStream_t st);

// integrator: opening half kick and drift; raises the rebuild flag of a
// system when one of its atoms moved more than skin/2 since its build, or
// when `scheduled`
void launch_kick_drift(const Plan& P, bool scheduled, hipStream_t st);

// exports into the caller's [N][3] arrays (row user_off + id)
enum class Field { force = 0, short_force = 1, velocity = 2 };
// pair-distance histogram [S][S][n_bins] (uint64, accumulated) from the lists
void launch_rdf(const Plan& P, int n_species, double D, int n_bins, unsigned long long* counts, hipStream_t st);
// Allocation-free pair histogram: a file-scope device array of kRdfScratch
// counters per GPU.  noalloc_init looks up its address on `device` (which
// must be current) once; noalloc_scratch returns it (null before init).
constexpr int kRdfScratch = 16384;
bool noalloc_init(int device, const char** err);
unsigned long long* noalloc_scratch(int device);
// zero n counters with a fill kernel
void launch_zero_u64(unsigned long long* p, int n, hipStream_t st);
// mean-square displacement bookkeeping of one system (Plan of that system);
// part: [ceil(n/64)][2 kMaxSpecies] wavefront partials
void launch_msd(const Plan& P, double* last, double* disp, double* part, bool mark, hipStream_t st);
void launch_to_user3(const Plan& P, Field f, double* out, hipStream_t st);
void launch_pos_to_user(const Plan& P, double* out, hipStream_t st);
void launch_kspace_part(const Plan& P, double* out, hipStream_t st);
// shell ranks of one system (P.R == 1) into out[n][P_R], n_out[n] by atom id
void launch_shell_ranks(const Plan& P, int32_t* out, int32_t* n_out, hipStream_t st);
// stored shell batch of one system (P.R == 1) as atom ids into out[n][P_R]
// (-1 past the batch) and candidate counts into n_out[n], by atom id
void launch_batch_ids(const Plan& P, int32_t* out, int32_t* n_out, hipStream_t st);
// shell batch of the current evaluation of one system (P.R == 1, P_R >= 1)
// as atom ids in ascending rank order into out[n][P_R], candidate counts into
// n_out[n], by atom id
void launch_shell_samples(const Plan& P, int32_t* out, int32_t* n_out, hipStream_t st);
// positions from the caller's [N][3] array (user order, device); raises the
// stale flag of a system with an atom more than skin/2 from its build
// position and records the largest displacement
void launch_set_positions(const Plan& P, const double* pos, hipStream_t st);
void launch_from_user(const Plan& P, const int32_t* type, const double* pos, const double* vel, hipStream_t st);

}  // namespace rbsog
