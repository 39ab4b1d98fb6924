// C ABI of librbsog (declared in include/rbsog.h): context, validation,
// planning of a batch of systems, kernel sequencing, exports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <functional>
#include <memory>
#include <initializer_list>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rbsog.h"
#include "kernels.hpp"
#include "setup.hpp"

using namespace rbsog;

namespace {

struct Error : std::runtime_error {
    rbsog_status code;
    Error(rbsog_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_OK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            throw Error(e_ == hipErrorOutOfMemory ? RBSOG_E_OOM : RBSOG_E_HIP,                         \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                            \
    } while (0)

// Device buffer owned by the context.
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void alloc(size_t b)
    {
        release();
        if (b == 0) return;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error(RBSOG_E_OOM, "hipMalloc of " + std::to_string(b) + " bytes failed");
        }
        bytes = b;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const
    {
        return static_cast<T*>(p);
    }
    ~DBuf() { release(); }
};

}  // namespace

struct rbsog_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    bool have_system = false;
    int R = 0;                       // systems in the batch
    std::vector<rbsog_params> prm;   // per system, defaults filled in
    bool mixed = false;
    SogSplit sog;
    int chain = 1;
    SogCoef coef{};
    std::vector<KTables> kt;
    std::vector<double> u_self;
    std::vector<int> slot_off;       // first atom slot of each system (multiple of 256)
    int n_slots = 0;                 // atom slots of the batch arrays
    int n_user = 0;                  // atoms of the batch (rows of the caller's arrays)
    int sel = 0;                     // system the parity exports refer to
    uint64_t eval = 0;               // eval index of the last force evaluation
    bool forces_valid = false;
    // positions set by the caller moved an atom more than skin/2 from its
    // position at the last build (compute_forces refuses, step rebuilds)
    bool stale = false;
    // a step or evaluation produced a non-finite position or force: every
    // call that would use the state refuses until a system is set again
    bool nonfinite = false;

    std::vector<DevSys> hs;          // host images of the device system records
    std::vector<KDev> hk;
    Plan plan;

    // device memory
    DBuf d_sys, d_kd, d_maps;
    DBuf atoms, sortbuf, cells, lists_core, lists_cand, lists_bat, counts, pair_tab, scalars;
    // memory form of the list: build chunks asked for, and the headroom of the
    // candidate scratch over a chunk's expected atom count
    int list_chunks = 8;
    std::vector<int> list_mode_r;    // staging class of each system (kListPerAtom: per-atom kernel)
    double row_slack = 1.25;
    DBuf ktab, kcdf, kmodes, krho_part, krho, pair_part, vir_part, fin_part, kin_part, export_tmp, snap, sogk, neartab;
    DBuf flux_part, at_ew, ufix;
    // mean-square displacement: [n_user][3] last positions, then [n_user][3]
    // unwrapped displacements; which systems have a marked origin
    DBuf msd_buf;
    std::vector<char> msd_marked;

    // phase timing (hot_only: the pair, rho and k-space force phases)
    bool profiling = false;
    bool hot_only = false;
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    int open_phase = -1;
    hipEvent_t open_a = nullptr;

    hipEvent_t take_event()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) throw std::runtime_error("hipEventCreate failed");
        return e;
    }
    // phases are timed on the stream their kernels run on
    bool open_aux = false;
    void begin(int phase, bool on_aux = false)
    {
        if (!profiling) return;
        if (hot_only && phase != RBSOG_PHASE_PAIR && phase != RBSOG_PHASE_RHO && phase != RBSOG_PHASE_KFORCE) return;
        open_phase = phase;
        open_aux = on_aux;
        open_a = take_event();
        (void)hipEventRecord(open_a, on_aux ? aux : stream);
    }
    void end()
    {
        if (!profiling || open_phase < 0) return;
        hipEvent_t b = take_event();
        (void)hipEventRecord(b, open_aux ? aux : stream);
        recs.push_back(Rec{open_phase, open_a, b});
        open_phase = -1;
        open_a = nullptr;
    }

    // second stream (default priority) for the k-space chain, which runs
    // beside the pair kernel; forked from and joined to `stream` by events
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // step graphs, [scheduled rebuild][energies], captured on first use
    bool use_graph = false;
    hipGraphExec_t graphs[4] = {nullptr, nullptr, nullptr, nullptr};
    void drop_graphs()
    {
        for (auto& g : graphs) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    }

    ~rbsog_ctx()
    {
        drop_graphs();
        if (aux) {
            (void)hipStreamSynchronize(aux);
            (void)hipStreamDestroy(aux);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        for (auto& r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

namespace {

constexpr int kBlock = 256;
constexpr double kCoulombDefault = 14.399645478425668;
constexpr double kBoltzmann = 8.617333262e-5;  // eV/K

rbsog_status fail(rbsog_ctx* c, rbsog_status code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

template <class F>
rbsog_status guarded(rbsog_ctx* c, F&& f)
{
    if (!c) return RBSOG_E_ARG;
    try {
        HIP_OK(hipSetDevice(c->device));
        f();
        c->err.clear();
        return RBSOG_OK;
    } catch (const Error& e) {
        return fail(c, e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(c, RBSOG_E_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(c, RBSOG_E_HIP, e.what());
    } catch (...) {
        return fail(c, RBSOG_E_HIP, "unknown error");
    }
}

void require(bool ok, rbsog_status code, const std::string& msg)
{
    if (!ok) throw Error(code, msg);
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }
int blocks_for(int n, int b) { return (n + b - 1) / b; }

void validate(const rbsog_params* p)
{
    require(p != nullptr, RBSOG_E_ARG, "params is NULL");
    require(p->n_atoms >= 0, RBSOG_E_ARG, "n_atoms < 0");
    require(p->n_species >= 1 && p->n_species <= RBSOG_MAX_SPECIES, RBSOG_E_ARG, "n_species out of range");
    require(p->r_core > 0.0 && p->r_shell > p->r_core, RBSOG_E_ARG, "need 0 < r_core < r_shell");
    require(p->skin >= 0.0, RBSOG_E_ARG, "skin < 0");
    require(p->dt > 0.0, RBSOG_E_ARG, "dt <= 0");
    require(p->rebuild_every >= 1, RBSOG_E_ARG, "rebuild_every < 1");
    require(p->precision == RBSOG_FP64 || p->precision == RBSOG_MIXED, RBSOG_E_ARG, "unknown precision");
    require(!(p->t_target > 0.0 && p->tau_t > 0.0) || p->tau_t >= p->dt, RBSOG_E_ARG, "tau_t < dt");
    require(!(p->t_target > 0.0 && p->tau_t > 0.0) || p->n_atoms >= 2, RBSOG_E_ARG, "thermostat needs 2+ atoms");
    require((p->flags & ~(uint32_t)(RBSOG_FLAG_SHELL_STORED | RBSOG_FLAG_INT_PHASE)) == 0, RBSOG_E_ARG, "unknown flag");
    require(!(p->flags & RBSOG_FLAG_INT_PHASE) || p->precision == RBSOG_MIXED, RBSOG_E_ARG,
            "the fixed-point phase is an option of the FP32-mixed form");
    require(p->thermostat == RBSOG_THERMO_BERENDSEN || p->thermostat == RBSOG_THERMO_NOSE_HOOVER ||
                p->thermostat == RBSOG_THERMO_LANGEVIN,
            RBSOG_E_ARG, "unknown thermostat");
    require(!(p->flags & RBSOG_FLAG_SHELL_STORED) || p->p_r >= 1, RBSOG_E_ARG, "a stored shell batch needs p_r >= 1");
    for (int a = 0; a < 3; ++a) {
        require(std::isfinite(p->box[a]) && p->box[a] > 0.0, RBSOG_E_ARG, "box must be positive");
        require(p->box[a] >= 2.0 * (p->r_shell + p->skin), RBSOG_E_BOX,
                "box shorter than 2 (r_shell + skin) along an axis");
    }
    const int S = p->n_species;
    for (int i = 0; i < S; ++i) {
        require(p->species[i].mass > 0.0, RBSOG_E_ARG, "species mass must be positive");
        for (int j = 0; j < S; ++j) {
            const double r = p->r_core_pair[i * RBSOG_MAX_SPECIES + j];
            require(r == p->r_core_pair[j * RBSOG_MAX_SPECIES + i], RBSOG_E_ARG, "r_core_pair must be symmetric");
            require(r == 0.0 || (r > 0.0 && r < p->r_shell), RBSOG_E_ARG, "need 0 < r_core_pair < r_shell");
        }
        for (int j = 0; j < S; ++j) {
            const rbsog_pair& a = p->pair[i * RBSOG_MAX_SPECIES + j];
            const rbsog_pair& b = p->pair[j * RBSOG_MAX_SPECIES + i];
            require(a.A == b.A && a.sigma == b.sigma && a.rho == b.rho && a.C == b.C && a.D == b.D, RBSOG_E_ARG,
                    "pair table must be symmetric");
            require(a.rho > 0.0 || a.A == 0.0, RBSOG_E_ARG, "rho must be positive");
        }
    }
}

// Parameters that every system of a batch shares (one SOG split, one pair
// table, one integrator schedule).
void require_shared(const rbsog_params& a, const rbsog_params& b)
{
    bool same = a.n_species == b.n_species && a.r_core == b.r_core && a.r_shell == b.r_shell &&
                a.skin == b.skin && a.sog_eps == b.sog_eps && a.dt == b.dt && a.rebuild_every == b.rebuild_every &&
                a.precision == b.precision && a.coulomb_k == b.coulomb_k && a.flags == b.flags &&
                std::memcmp(a.r_core_pair, b.r_core_pair, sizeof(a.r_core_pair)) == 0;
    for (int i = 0; same && i < a.n_species; ++i) {
        same = a.species[i].q == b.species[i].q && a.species[i].mass == b.species[i].mass;
        for (int j = 0; same && j < a.n_species; ++j) {
            const rbsog_pair& x = a.pair[i * RBSOG_MAX_SPECIES + j];
            const rbsog_pair& y = b.pair[i * RBSOG_MAX_SPECIES + j];
            same = x.A == y.A && x.sigma == y.sigma && x.rho == y.rho && x.C == y.C && x.D == y.D;
        }
    }
    require(same, RBSOG_E_ARG,
            "systems of a batch must share species, pair table, radii, skin, sog_eps, dt, rebuild_every, "
            "precision, coulomb_k, flags and r_core_pair");
}

// Device copies of the system records, after a host-side change.
void upload_sys(rbsog_ctx* c)
{
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(c->d_sys.p, c->hs.data(), sizeof(DevSys) * c->R, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_kd.p, c->hk.data(), sizeof(KDev) * c->R, hipMemcpyHostToDevice));
}

// Plan of system r alone (parity exports).
Plan one(const rbsog_ctx* c, int r)
{
    Plan P;
    const DevSys& s = c->hs[r];
    const KDev& k = c->hk[r];
    P.sys = c->d_sys.as<DevSys>() + r;
    P.kd = c->d_kd.as<KDev>() + r;
    P.sc = c->scalars.as<DeviceScalars>() + r;
    P.R = 1;
    P.tune = c->plan.tune;
    P.atoms.blocks = blocks_for(s.n, kBlock);
    P.pair_atoms.blocks = blocks_for(s.n, P.tune.pair_block);
    P.kf_atoms.blocks = blocks_for(s.n, P.tune.kf_block);
    P.cells.blocks = s.n > 0 ? s.ncell : 0;
    P.list_cells.blocks = s.n > 0 ? s.ncell * s.list_parts : 0;
    P.atom1.blocks = s.n;
    // an empty system draws no modes and sums no structure factors
    P.modes64.blocks = (s.n > 0 && k.sampled) ? blocks_for(k.n_modes, 64) : 0;
    P.rho.blocks = (s.n > 0 && k.n_modes > 0) ? k.n_chunks * blocks_for(k.n_modes, 64 * P.tune.rho_mpl) : 0;
    P.modes1.blocks = s.n > 0 ? k.n_modes : 0;
    P.rows64.blocks = (s.n > 0 && s.shell_stored) ? blocks_for(s.cand_rows, 64) : 0;
    P.list_mode = c->plan.list_mode;
    if (P.list_mode < kListPerAtom && r < (int)c->list_mode_r.size()) {
        P.list_mode = c->list_mode_r[r];
        if (P.list_mode < kListPerAtom) P.list_by_cap[P.list_mode] = P.list_cells;
    }
    P.stored = c->plan.stored;
    P.n_chunks = c->plan.n_chunks;
    P.cap_core = c->plan.cap_core;
    P.cap_cand = c->plan.cap_cand;
    P.near = c->plan.near;
    P.langevin = c->plan.langevin;
    P.iph = c->plan.iph;
    P.species_cut = c->plan.species_cut;
    return P;
}

// Block maps of the batch launches (none for a single system, except the
// chunks of a memory-form build).  Called again whenever the tuning or the
// list plan changes the shapes.
void plan_launches(rbsog_ctx* c)
{
    HIP_OK(hipStreamSynchronize(c->stream));  // the old maps may still be in use
    c->drop_graphs();
    Plan& P = c->plan;
    P.sys = c->d_sys.as<DevSys>();
    P.kd = c->d_kd.as<KDev>();
    P.sc = c->scalars.as<DeviceScalars>();
    P.R = c->R;
    P.fin_grid = 1;
    for (const auto& s : c->hs) P.fin_grid = std::max(P.fin_grid, fin_blocks(s.n));
    constexpr int kShapes = 10 + kListPerAtom;
    Shape* dst[kShapes] = {&P.atoms, &P.pair_atoms, &P.kf_atoms, &P.cells, &P.atom1, &P.modes64, &P.rho,
                           &P.modes1, &P.rows64, &P.list_cells, &P.list_by_cap[0], &P.list_by_cap[1],
                           &P.list_by_cap[2]};
    static_assert(kListPerAtom == 3, "one staging-class shape per capacity");
    std::vector<std::vector<int2>> m(kShapes + kMaxListChunks);
    const bool maps = c->R > 1;
    for (int r = 0; r < c->R; ++r) {
        const Plan o = one(c, r);
        const Shape* sh[kShapes] = {&o.atoms, &o.pair_atoms, &o.kf_atoms, &o.cells, &o.atom1, &o.modes64, &o.rho,
                                    &o.modes1, &o.rows64, &o.list_cells, &o.list_by_cap[0], &o.list_by_cap[1],
                                    &o.list_by_cap[2]};
        for (int q = 0; q < kShapes; ++q) {
            if (maps)
                for (int b = 0; b < sh[q]->blocks; ++b) m[q].push_back(make_int2(r, b));
            else
                *dst[q] = *sh[q];
        }
        // cells of each build chunk, the split the kernels compute
        const DevSys& s = c->hs[r];
        if (P.stored && o.cells.blocks > 0)
            for (int k = 0; k < s.n_chunks; ++k) {
                const int c0 = (int)(((long long)k * s.ncell) / s.n_chunks);
                const int c1 = (int)(((long long)(k + 1) * s.ncell) / s.n_chunks);
                for (int cc = c0; cc < c1; ++cc)
                    for (int q = 0; q < s.list_parts; ++q) m[kShapes + k].push_back(make_int2(r, cc * s.list_parts + q));
            }
    }
    for (int k = 0; k < kMaxListChunks; ++k) P.cell_chunk[k] = Shape{};
    size_t total = 0;
    for (auto& v : m) total += v.size();
    if (total == 0) return;
    c->d_maps.alloc(sizeof(int2) * total);
    int2* d = c->d_maps.as<int2>();
    for (int q = 0; q < kShapes + kMaxListChunks; ++q) {
        if (q < kShapes && !maps) continue;
        Shape& sh = q < kShapes ? *dst[q] : P.cell_chunk[q - kShapes];
        sh.blocks = (int)m[q].size();
        sh.map = d;
        if (!m[q].empty()) HIP_OK(hipMemcpy(d, m[q].data(), sizeof(int2) * m[q].size(), hipMemcpyHostToDevice));
        d += m[q].size();
    }
}

void plan_lists(rbsog_ctx* c, int cap_core, int cap_cand)
{
    c->drop_graphs();
    c->plan.cap_core = cap_core;
    c->plan.cap_cand = cap_cand;
    const bool stored = c->R > 0 && c->hs[0].shell_stored;
    // the memory form keeps candidate rows for one chunk of cells at a time
    // (the per-atom fallback kernel needs them all); otherwise one per atom
    const int K = (stored && c->plan.list_mode != kListPerAtom) ? std::max(1, std::min(c->list_chunks, kMaxListChunks)) : 1;
    c->plan.stored = stored;
    c->plan.n_chunks = K;
    size_t bat_all = 0;
    std::vector<int> rows(c->R);
    for (int r = 0; r < c->R; ++r) {
        DevSys& s = c->hs[r];
        const int npad = round_up(std::max(s.n, 1), 64);
        s.n_chunks = std::max(1, std::min(K, s.ncell));
        if (s.n_chunks == 1) {
            rows[r] = npad;
        } else {
            // most cells in one chunk, times the mean atoms per cell, with headroom
            const int cells_max = (s.ncell + s.n_chunks - 1) / s.n_chunks;
            const double expect = (double)s.n * cells_max / s.ncell;
            rows[r] = std::min(npad, round_up((int)std::ceil(expect * c->row_slack) + 64, 64));
        }
        bat_all += stored ? (size_t)npad * s.p_r : 0;
    }
    const size_t slots = (size_t)std::max(c->n_slots, 64);
    c->lists_core.alloc(sizeof(int32_t) * slots * cap_core);
    size_t cand_rows_total = 0;
    if (stored)
        for (int r = 0; r < c->R; ++r) cand_rows_total += (size_t)rows[r];
    else
        cand_rows_total = slots;
    c->lists_cand.alloc(sizeof(int32_t) * std::max<size_t>(cand_rows_total, 1) * cap_cand);
    if (stored)
        c->lists_bat.alloc(sizeof(int32_t) * std::max<size_t>(bat_all, 1));
    else
        c->lists_bat.release();
    // every list entry holds an atom index from the start: a kernel that runs
    // after a build that overflowed (and is discarded) reads only indices
    for (DBuf* b : {&c->lists_core, &c->lists_cand, &c->lists_bat})
        if (b->p) HIP_OK(hipMemsetAsync(b->p, 0, b->bytes, c->stream));
    size_t row_off = 0, bat_off = 0;
    for (int r = 0; r < c->R; ++r) {
        DevSys& s = c->hs[r];
        s.cap_core = cap_core;
        s.cap_cand = cap_cand;
        // slot offsets are multiples of 64: whole core-list tiles per system
        s.core_idx = c->lists_core.as<int32_t>() + (size_t)c->slot_off[r] * cap_core;
        if (stored) {
            s.cand_rows = rows[r];
            s.cand_idx = c->lists_cand.as<int32_t>() + row_off * cap_cand;
            row_off += (size_t)rows[r];
            s.bat_idx = c->lists_bat.as<int32_t>() + bat_off;
            bat_off += (size_t)round_up(std::max(s.n, 1), 64) * s.p_r;
        } else {
            s.n_chunks = 1;
            s.cand_rows = round_up(std::max(s.n, 1), 64);
            s.cand_idx = c->lists_cand.as<int32_t>() + (size_t)c->slot_off[r] * cap_cand;
            s.bat_idx = nullptr;
        }
    }
    upload_sys(c);
}

void enqueue_build(rbsog_ctx* c, bool gate)
{
    c->begin(RBSOG_PHASE_BUILD);
    launch_build(c->plan, gate, c->stream);
    c->end();
}

std::vector<DeviceScalars> read_scalars(rbsog_ctx* c)
{
    std::vector<DeviceScalars> h(c->R);
    HIP_OK(hipMemcpyAsync(h.data(), c->plan.sc, sizeof(DeviceScalars) * c->R, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return h;
}

int any_overflow(const std::vector<DeviceScalars>& h)
{
    int o = 0;
    for (const auto& x : h) o |= x.overflow;
    return o;
}

// Per-atom state (cell order) and device scalars of every system at the start
// of a step call, for a restart after a list overflow.
void snapshot(rbsog_ctx* c, bool save)
{
    const size_t N = (size_t)std::max(c->n_slots, 1);
    const size_t bytes = N * (sizeof(double4) + 6 * sizeof(double) + 3 * sizeof(int32_t)) +
                         sizeof(DeviceScalars) * c->R;
    if (save && c->snap.bytes < bytes) c->snap.alloc(bytes);
    const DevSys& s = c->hs[0];  // system 0 starts at slot 0: its pointers are the batch arrays
    char* d = c->snap.as<char>();
    struct Arr {
        void* p;
        size_t b;
    };
    const Arr arr[] = {{s.p, sizeof(double4)}, {s.vx, 8}, {s.vy, 8}, {s.vz, 8}, {s.fx, 8}, {s.fy, 8},
                       {s.fz, 8},              {s.type, 4}, {s.id, 4}, {s.inv, 4},
                       {c->plan.sc, 0}};
    for (const Arr& a : arr) {
        const size_t b = a.b ? a.b * N : sizeof(DeviceScalars) * c->R;
        if (save)
            HIP_OK(hipMemcpyAsync(d, a.p, b, hipMemcpyDeviceToDevice, c->stream));
        else
            HIP_OK(hipMemcpyAsync(a.p, d, b, hipMemcpyDeviceToDevice, c->stream));
        d += b;
    }
}

// After a build that overflowed: grow what overflowed (bit 1: list
// capacities, from the true counts of the build; bit 4: the list kernel's
// stencil; bit 8: the candidate scratch of a memory-form chunk) and plan the
// lists again.  Bit 2 (a cell above the in-cell sort's capacity) is fatal.
void grow_after_overflow(rbsog_ctx* c, int o)
{
    require((o & 2) == 0, RBSOG_E_CAPACITY, "a cell holds more than 2048 atoms");
    int cap_core = c->plan.cap_core, cap_cand = c->plan.cap_cand;
    if (o & 1) {
        int mc = 0, mk = 0;
        for (const auto& h : read_scalars(c)) {
            mc = std::max(mc, h.max_core);
            mk = std::max(mk, h.max_cand);
        }
        cap_core = std::max(cap_core, round_up(mc + mc / 4 + 8, 32));
        cap_cand = std::max(cap_cand, round_up(mk + mk / 4 + 8, 32));
        require(cap_cand <= 4096 && cap_core <= 4096, RBSOG_E_CAPACITY, "neighbour list capacity above 4096");
    }
    if (o & 4) {
        // the systems whose stencil did not fit move to the next capacity
        const auto h = read_scalars(c);
        for (int r = 0; r < c->R; ++r)
            if (h[r].overflow & 4) c->list_mode_r[r] = std::min(kListPerAtom, c->list_mode_r[r] + 1);
        // the memory form and the per-atom kernel take the largest for all
        int m = 0;
        for (int v : c->list_mode_r) m = std::max(m, v);
        c->plan.list_mode = m;
    }
    if (o & 8) c->row_slack *= 2.0;
    plan_lists(c, cap_core, cap_cand);
    plan_launches(c);
}

// Build; if a list or cell capacity overflowed, grow it and build again.
void build_checked(rbsog_ctx* c)
{
    for (int attempt = 0; attempt < 6; ++attempt) {
        launch_clear_flags(c->plan, c->stream);
        enqueue_build(c, false);
        const int o = any_overflow(read_scalars(c));
        if (o == 0) return;
        grow_after_overflow(c, o);
    }
    throw Error(RBSOG_E_CAPACITY, "list capacity did not converge");
}

// A thermostat that needs the kinetic energy every step (Berendsen,
// Nose-Hoover; Langevin acts atom by atom).
bool any_thermostat(const rbsog_ctx* c)
{
    for (const auto& s : c->hs)
        if (s.thermo_c > 0.0 && s.thermostat != RBSOG_THERMO_LANGEVIN) return true;
    return false;
}

// The k-space chain (mode draws, structure factors, their reduction and the
// k-space force) reads positions and writes only mode data and the k-space
// force (into the total-force arrays), the pair kernel reads positions and
// writes only short-range forces and its partials: the chain runs on the
// second stream beside the pair kernel, and the first stream waits for it
// before the sums that need both.
// build: a step's gated list build goes in first.  Only its cell sort
// (which reorders the atoms) precedes the fork: the k-space chain needs the
// sorted positions but not the lists, so it runs beside the list kernels.
void enqueue_forces(rbsog_ctx* c, bool energy, bool kick, bool build = false)
{
    const bool ke = energy || (kick && any_thermostat(c));
    const Plan& P = c->plan;
    // an evaluation with energies takes the fused k-space pass, which forms
    // the per-atom k-space shares of the stress and heat flux
    const bool aux_kf = P.tune.kf_aux && !energy;
    hipStream_t st = c->stream;
    hipStream_t ax = c->aux;
    if (P.atoms.blocks <= 0) return;
    if (build) {
        c->begin(RBSOG_PHASE_BUILD);
        launch_sort(P, true, st);
        c->end();
    }
    HIP_OK(hipEventRecord(c->ev_fork, st));
    HIP_OK(hipStreamWaitEvent(ax, c->ev_fork, 0));
    if (P.modes64.blocks > 0) {
        c->begin(RBSOG_PHASE_KSAMPLE, true);
        launch_ksample(P, ax);
        c->end();
    }
    c->begin(RBSOG_PHASE_RHO, true);
    launch_rho(P, c->mixed, ax);
    launch_rho_finalize(P, ax);
    c->end();
    if (aux_kf) {
        c->begin(RBSOG_PHASE_KFORCE, true);
        launch_kforce(P, c->mixed, ax);
        c->end();
    }
    HIP_OK(hipEventRecord(c->ev_join, ax));
    if (build) {
        c->begin(RBSOG_PHASE_BUILD);
        launch_lists(P, true, st);
        c->end();
    }
    c->begin(RBSOG_PHASE_PAIR);
    launch_pair(P, c->coef, c->mixed, energy, st);
    HIP_OK(hipGetLastError());  // a launch the device refuses (e.g. LDS size) must not pass silently
    c->end();
    HIP_OK(hipStreamWaitEvent(st, c->ev_join, 0));
    c->begin(RBSOG_PHASE_REDUCE);
    launch_finalize(P, energy, st);
    c->end();
    if (aux_kf) {
        c->begin(RBSOG_PHASE_INTEGRATE);
        launch_combine(P, kick, ke, st);
        c->end();
    } else {
        c->begin(RBSOG_PHASE_KFORCE);
        launch_kforce_fused(P, c->mixed, kick, energy ? 2 : (ke ? 1 : 0), st);
        c->end();
    }
    if (ke) launch_kinetic_finalize(P, kick, energy, st);
}

void fill_energy(rbsog_ctx* c, const std::vector<DeviceScalars>& hv, rbsog_energy* e)
{
    for (int r = 0; r < c->R; ++r) {
        const DeviceScalars& h = hv[r];
        e[r].u_core = h.u_core;
        e[r].u_shell = h.u_shell;
        e[r].u_kspace = h.u_kspace;
        e[r].u_self = c->u_self[r];
        e[r].u_total = h.u_core + h.u_shell + h.u_kspace - c->u_self[r];
        e[r].kinetic = h.kinetic;
        for (int a = 0; a < 3; ++a) e[r].p_corr[a] = h.p_corr[a];
        e[r].max_disp = std::sqrt(h.max_disp2);
        e[r].n_builds = h.n_builds;
        for (int a = 0; a < 6; ++a) e[r].virial[a] = h.virial[a];
        for (int a = 0; a < 6; ++a) e[r].stress[a] = h.stress[a];
        for (int a = 0; a < 3; ++a) e[r].heat_flux[a] = h.heat_flux[a];
        const DevSys& s = c->hs[r];
        e[r].e_thermostat = (s.thermo_c > 0.0 && s.thermostat == RBSOG_THERMO_NOSE_HOOVER)
                                ? 0.5 * s.nh_q * h.nh_v * h.nh_v + s.dof_kb * s.t_target * h.nh_x
                                : 0.0;
    }
}

// A non-finite position or force seen by the kernels (checked before any
// capacity overflow, which NaN positions can cause).
void check_finite(rbsog_ctx* c, const std::vector<DeviceScalars>& h)
{
    for (size_t r = 0; r < h.size(); ++r)
        if (h[r].nonfinite) {
            c->nonfinite = true;
            throw Error(RBSOG_E_NONFINITE, "system " + std::to_string(r) +
                                               " produced a non-finite position or force; set the system again");
        }
}

void need_finite(const rbsog_ctx* c)
{
    require(!c->nonfinite, RBSOG_E_NONFINITE,
            "the state holds non-finite positions or forces from an earlier call; set the system again");
}

void check_flags(rbsog_ctx* c, const std::vector<DeviceScalars>& h)
{
    check_finite(c, h);
    if (any_overflow(h)) throw Error(RBSOG_E_CAPACITY, "list capacity exceeded during the step loop");
}

// One step on the stream: kick + drift, rebuild of the systems whose step is
// scheduled or where an atom moved more than skin/2 since their last build
// (decided on the device), forces, kick.
void enqueue_step(rbsog_ctx* c, bool scheduled, bool energy)
{
    c->begin(RBSOG_PHASE_INTEGRATE);
    launch_step_begin(c->plan, c->stream);
    launch_kick_drift(c->plan, scheduled, c->stream);
    c->end();
    enqueue_forces(c, energy, true, true);
}

// The same step as one HIP graph launch: the kernel sequence of each variant
// is captured once and replayed (it holds kernels only).  Needs a non-default
// stream; phase timing records no events inside a graph, so it falls back to
// plain launches while timing is on.
void launch_step(rbsog_ctx* c, bool scheduled, bool energy)
{
    if (!c->use_graph || c->profiling || c->stream == nullptr) {
        enqueue_step(c, scheduled, energy);
        return;
    }
    hipGraphExec_t& g = c->graphs[(scheduled ? 2 : 0) + (energy ? 1 : 0)];
    if (!g) {
        hipGraph_t graph = nullptr;
        HIP_OK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        enqueue_step(c, scheduled, energy);
        HIP_OK(hipStreamEndCapture(c->stream, &graph));
        const hipError_t e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_OK(e);
    }
    HIP_OK(hipGraphLaunch(g, c->stream));
}

// Event time of `reps` runs of f, or infinity if the launch is refused.
double time_ms(rbsog_ctx* c, int reps, const std::function<void()>& f)
{
    (void)hipGetLastError();
    f();  // warm
    if (hipGetLastError() != hipSuccess) return 1e300;
    hipEvent_t a = nullptr, b = nullptr;
    HIP_OK(hipEventCreate(&a));
    HIP_OK(hipEventCreate(&b));
    HIP_OK(hipEventRecord(a, c->stream));
    for (int r = 0; r < reps; ++r) f();
    HIP_OK(hipEventRecord(b, c->stream));
    HIP_OK(hipEventSynchronize(b));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

// Time each kernel under its candidate launch shapes at the current positions
// and keep the fastest.  Every candidate computes the same bits, so the
// evaluations it repeats leave the state as it was.
void autotune(rbsog_ctx* c, int reps)
{
    const bool was_profiling = c->profiling;
    c->profiling = false;
    hipStream_t st = c->stream;
    launch_set_eval(c->plan, c->eval, st);
    enqueue_forces(c, false, false);
    Tuning best = c->plan.tune;
    auto try_shape = [&](Tuning t) {
        c->plan.tune = t;
        plan_launches(c);
    };
    try_shape(best);
    launch_rho(c->plan, c->mixed, st);
    launch_rho_finalize(c->plan, st);
    launch_pair(c->plan, c->coef, c->mixed, false, st);
    launch_finalize(c->plan, false, st);
    // a first pick of the k-space force workgroup size, the kernel alone
    // (refined on whole steps below)
    double tb = 1e300;
    for (int bs : {64, 128, 256}) {
        Tuning t = best;
        t.kf_block = bs;
        try_shape(t);
        const double ms = time_ms(c, reps, [&] { launch_kforce(c->plan, c->mixed, st); });
        if (ms < tb) {
            tb = ms;
            best.kf_block = bs;
        }
    }
    // The pair kernel shares the device with the k-space chain on the second
    // stream, and the passes around it in a step (drift, gated build) change
    // what the caches hold when it starts: its shape, the rho modes per lane
    // and where the k-space force runs are chosen together on whole steps
    // (timed on back-to-back force evaluations, larger pair workgroups look
    // faster and still lengthen the step).  Every candidate runs the same
    // steps from one saved device state (atoms, list counts, lists and
    // scalars), which is put back afterwards: tuning leaves the trajectory
    // bit for bit as it was.  Alternating rounds, best of three.
    DBuf* state[] = {&c->atoms, &c->ufix, &c->counts, &c->lists_core, &c->lists_cand, &c->lists_bat, &c->scalars};
    constexpr int kState = sizeof(state) / sizeof(state[0]);
    std::unique_ptr<DBuf[]> saved(new DBuf[kState]);
    auto copy_state = [&](bool save) {
        for (int q = 0; q < kState; ++q) {
            DBuf& live = *state[q];
            if (!live.p) continue;
            if (save) saved[q].alloc(live.bytes);
            HIP_OK(hipMemcpyAsync(save ? saved[q].p : live.p, save ? live.p : saved[q].p, live.bytes,
                                  hipMemcpyDeviceToDevice, st));
        }
    };
    copy_state(true);
    const int n_steps = std::max(reps, 3);
    struct Cand {
        Tuning t;
        double ms;
    };
    std::vector<Cand> cands;
    for (int bs : {64, 128, 256})
        for (int ku : {4, 8})
            for (int mpl : {1, 2})
                for (int aux : {1, 0}) {
                    Tuning t = best;
                    t.pair_block = bs;
                    t.pair_ku = ku;
                    t.rho_mpl = mpl;
                    t.kf_aux = aux;
                    cands.push_back(Cand{t, 1e300});
                }
    auto search = [&](std::vector<Cand>& cs) {
        for (int round = 0; round < 3; ++round)
            for (Cand& cd : cs) {
                try_shape(cd.t);
                copy_state(false);
                // time_ms runs the steps once untimed first (which also
                // captures the step graph when graphs are on), then once timed
                cd.ms = std::min(cd.ms, time_ms(c, 1, [&] {
                    for (int k = 0; k < n_steps; ++k) launch_step(c, false, false);
                }));
            }
        double t_best = 1e300;
        for (const Cand& cd : cs)
            if (cd.ms < t_best) {
                t_best = cd.ms;
                best = cd.t;
            }
    };
    try {
        search(cands);
        // then the k-space force workgroup again, on whole steps with the
        // shapes just chosen (alone it ranks sizes that run beside the pair
        // kernel differently)
        std::vector<Cand> kf;
        for (int bs : {64, 128, 256}) {
            Tuning t = best;
            t.kf_block = bs;
            kf.push_back(Cand{t, 1e300});
        }
        search(kf);
    } catch (...) {
        // put the saved state back before reporting the failure
        try {
            try_shape(best);
            copy_state(false);
            (void)hipStreamSynchronize(st);
        } catch (...) {
        }
        c->profiling = was_profiling;
        throw;
    }
    try_shape(best);
    copy_state(false);
    HIP_OK(hipStreamSynchronize(st));
    c->forces_valid = true;
    c->profiling = was_profiling;
}

// Geometry, cutoffs, species and integrator constants of one system.
void init_devsys(const rbsog_params& p, int n, DevSys& s)
{
    s = DevSys{};
    s.n = n;
    s.n_species = p.n_species;
    const double cutoff = p.r_shell + p.skin;
    s.ncell = 1;
    for (int a = 0; a < 3; ++a) {
        s.L[a] = p.box[a];
        s.invL[a] = 1.0 / p.box[a];
        int nc = (int)std::floor(p.box[a] / (cutoff + 1e-9));
        if (nc < 3) nc = 1;
        s.nc[a] = nc;
        s.cell_scale[a] = (double)nc / p.box[a];
        // candidates are ordered on a grid of half-size cells
        s.nf[a] = nc >= 3 ? 2 * nc : 1;
        s.fine_scale[a] = (double)s.nf[a] / p.box[a];
        s.two_pi_L[a] = 2.0 * kPi / p.box[a];
        s.ncell *= nc;
    }
    const double rcl = p.r_core + p.skin;
    s.rc2_list = rcl * rcl;
    s.species_cut = 0;
    for (int i = 0; i < p.n_species; ++i)
        for (int j = 0; j < p.n_species; ++j) {
            const double r = p.r_core_pair[i * RBSOG_MAX_SPECIES + j];
            if (r > 0.0 && r != p.r_core) s.species_cut = 1;
        }
    const double lo = p.r_core - p.skin;
    s.lo2_list = lo > 0.0 ? lo * lo : 0.0;
    const double hi = p.r_shell + p.skin;
    s.hi2_list = hi * hi;
    s.rc2 = p.r_core * p.r_core;
    s.rs2 = p.r_shell * p.r_shell;
    {
        // A coordinate of a fixed-point record is within d = L 2^-32 below
        // the true one, so a difference is within d of the FP64 minimum
        // image and r^2 within 2 sqrt(3) r d + 3 d^2; at the cutoffs (r <=
        // r_shell) that is below the guard, kept at four times the bound.
        const double d = std::max(p.box[0], std::max(p.box[1], p.box[2])) * std::ldexp(1.0, -32);
        s.fix_guard = 4.0 * (2.0 * std::sqrt(3.0) * p.r_shell * d + 3.0 * d * d) + 1e-12 * s.rs2;
    }
    s.half_skin2 = 0.25 * p.skin * p.skin;
    // A list entry was within r_shell + skin at the build and both atoms
    // have moved at most skin/2 since, so it is now within M = r_shell +
    // 2 skin; an atom at least M inside every face sees all its entries
    // without wrap, and with M < 0.4 L their differences need no minimum image.
    const double margin = (p.r_shell + 2.0 * p.skin) * (1.0 + 1e-9);
    for (int a = 0; a < 3; ++a) {
        const bool room = p.box[a] > 2.5 * margin;
        s.inner_lo[a] = room ? margin : 1.0e300;
        s.inner_hi[a] = room ? p.box[a] - margin : -1.0e300;
    }
    s.dt = p.dt;
    s.coulomb_k = p.coulomb_k;
    const bool thermo = p.t_target > 0.0 && p.tau_t > 0.0;
    s.thermo_c = thermo ? p.dt / p.tau_t : 0.0;
    s.t_target = thermo ? p.t_target : 0.0;
    s.dof_kb = (3.0 * n - 3.0) * kBoltzmann;
    s.thermostat = p.thermostat;
    if (thermo) {
        s.nh_q = s.dof_kb * p.t_target * p.tau_t * p.tau_t;
        s.lv_c1 = std::exp(-p.dt / p.tau_t);
        for (int t = 0; t < p.n_species; ++t)
            s.lv_c2[t] = std::sqrt((1.0 - s.lv_c1 * s.lv_c1) * kBoltzmann * p.t_target * kAccUnit / p.species[t].mass);
    }
    s.p_r = p.p_r;
    // about 96 atoms (24 work units, three per wavefront) per list workgroup
    s.list_parts = std::max(1, std::min(32, (int)std::ceil((double)n / s.ncell / 96.0)));
    s.shell_stored = (p.flags & RBSOG_FLAG_SHELL_STORED) ? 1 : 0;
    s.n_chunks = 1;
    s.replica = p.replica;
    s.seed = p.seed;
}

// Host copies of the caller's arrays (validation; staging of host inputs).
void fetch_inputs(const int32_t* type, const double* pos, const double* vel, int n, int on_device,
                  std::vector<int32_t>& ht, std::vector<double>& hp, std::vector<double>& hv)
{
    ht.resize(n);
    hp.resize(3 * (size_t)n);
    hv.clear();
    if (n <= 0) return;
    if (on_device) {
        HIP_OK(hipMemcpy(ht.data(), type, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(hp.data(), pos, sizeof(double) * 3 * n, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(ht.data(), type, sizeof(int32_t) * n);
        std::memcpy(hp.data(), pos, sizeof(double) * 3 * n);
    }
    if (vel) {
        hv.resize(3 * (size_t)n);
        if (on_device)
            HIP_OK(hipMemcpy(hv.data(), vel, sizeof(double) * 3 * n, hipMemcpyDeviceToHost));
        else
            std::memcpy(hv.data(), vel, sizeof(double) * 3 * n);
    }
}

void set_batch_impl(rbsog_ctx* c, int R, const rbsog_params* params, const int32_t* type, const double* pos,
                    const double* vel, int on_device)
{
    require(R >= 1, RBSOG_E_ARG, "a batch needs at least one system");
    require(params != nullptr, RBSOG_E_ARG, "params is NULL");
    std::vector<rbsog_params> prm(params, params + R);
    for (auto& p : prm) {
        validate(&p);
        if (!(p.coulomb_k > 0.0)) p.coulomb_k = kCoulombDefault;
        if (!(p.sog_eps > 0.0)) p.sog_eps = 1e-5;
    }
    for (int r = 1; r < R; ++r) require_shared(prm[0], prm[r]);
    std::vector<int> user_off(R + 1, 0), slot_off(R + 1, 0);
    for (int r = 0; r < R; ++r) {
        const int n = prm[r].n_atoms;
        require((int64_t)user_off[r] + n < (1ll << 30), RBSOG_E_ARG, "batch too large");
        user_off[r + 1] = user_off[r] + n;
        slot_off[r + 1] = slot_off[r] + round_up(n, kBlock);
    }
    const int n_user = user_off[R];
    require(n_user == 0 || (type && pos), RBSOG_E_ARG, "type and pos are required");
    std::vector<int32_t> ht;
    std::vector<double> hp, hv;
    fetch_inputs(type, pos, vel, n_user, on_device, ht, hp, hv);
    for (double v : hp) require(std::isfinite(v), RBSOG_E_NONFINITE, "non-finite position");
    for (double v : hv) require(std::isfinite(v), RBSOG_E_NONFINITE, "non-finite velocity");
    std::vector<double> q2(R, 0.0);
    for (int r = 0; r < R; ++r) {
        double qsum = 0.0, qabs = 0.0;
        for (int i = user_off[r]; i < user_off[r + 1]; ++i) {
            require(ht[i] >= 0 && ht[i] < prm[r].n_species, RBSOG_E_ARG, "atom type out of range");
            const double q = prm[r].species[ht[i]].q;
            qsum += q;
            qabs += std::fabs(q);
            q2[r] += q * q;
        }
        require(std::fabs(qsum) <= 1e-9 * std::max(1.0, qabs), RBSOG_E_NONNEUTRAL,
                R == 1 ? "system is not charge neutral" : "a system of the batch is not charge neutral");
    }

    // SOG split and coefficients (shared)
    const rbsog_params& p0 = prm[0];
    c->mixed = p0.precision == RBSOG_MIXED;
    std::string err;
    if (!sog_split(p0.sog_eps, p0.r_shell, &c->sog, &err)) throw Error(RBSOG_E_ARG, err);
    sog_base(p0.sog_eps, &c->chain);
    if (!sog_kernel_coef(c->sog, c->chain, p0.r_shell, c->mixed, &c->coef, &err)) throw Error(RBSOG_E_ARG, err);
    double wsum = 0.0;
    for (double w : c->sog.w) wsum += w;
    // FP32 near-field table of the mixed form (shared)
    NearTable nt;
    if (c->mixed) build_near_table(c->sog, p0.r_shell, &nt);
    c->plan.near = NearTab{};
    if (nt.nbin > 0) {
        c->neartab.alloc(sizeof(float) * nt.coef.size());
        HIP_OK(hipMemcpy(c->neartab.p, nt.coef.data(), sizeof(float) * nt.coef.size(), hipMemcpyHostToDevice));
        c->plan.near.coef = c->neartab.as<float4>();
        c->plan.near.lo = (127 + nt.e0) << 6;
        c->plan.near.n = nt.nbin * kNearSub;
    }

    c->drop_graphs();
    if (!c->aux) HIP_OK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    if (!c->ev_fork) HIP_OK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    if (!c->ev_join) HIP_OK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    c->R = R;
    c->prm = prm;
    c->msd_buf.release();
    c->msd_marked.assign(R, 0);
    c->sel = 0;
    c->row_slack = 1.25;
    c->plan.tune = Tuning{};
    c->plan.langevin = false;
    c->plan.species_cut = false;
    c->plan.iph = (p0.flags & RBSOG_FLAG_INT_PHASE) != 0;
    for (const auto& p : prm)
        if (p.t_target > 0.0 && p.tau_t > 0.0 && p.thermostat == RBSOG_THERMO_LANGEVIN) c->plan.langevin = true;
    c->slot_off.assign(slot_off.begin(), slot_off.end() - 1);
    c->n_slots = slot_off[R];
    c->n_user = n_user;
    c->u_self.assign(R, 0.0);
    c->hs.assign(R, DevSys{});
    c->hk.assign(R, KDev{});
    c->kt.assign(R, KTables{});
    for (int r = 0; r < R; ++r) {
        init_devsys(prm[r], prm[r].n_atoms, c->hs[r]);
        c->hs[r].user_off = user_off[r];
        // the list kernel packs the species above a 28-bit atom index
        // the cell sort keys (sub-cell, atom index) and the list kernel packs
        // the species above the index: 28 bits of index
        require(prm[r].n_atoms < (1 << 28), RBSOG_E_ARG, "a system holds fewer than 2^28 atoms");
        if (c->hs[r].species_cut) c->plan.species_cut = true;
        c->u_self[r] = 0.5 * p0.coulomb_k * q2[r] * wsum;
    }
    c->d_sys.alloc(sizeof(DevSys) * R);
    c->d_kd.alloc(sizeof(KDev) * R);

    // per-atom arrays of the batch: a packed position record, 12 doubles,
    // 3 int32 per slot; system r owns slots [slot_off[r], slot_off[r] + n_r)
    const size_t N = (size_t)std::max(c->n_slots, 1);
    c->atoms.alloc(N * (sizeof(double4) + 12 * sizeof(double) + 3 * sizeof(int32_t)));
    c->sortbuf.alloc(N * (sizeof(double4) + 6 * sizeof(double) + 5 * sizeof(int32_t)));
    c->counts.alloc(2 * sizeof(int32_t) * N);
    HIP_OK(hipMemsetAsync(c->counts.p, 0, 2 * sizeof(int32_t) * N, c->stream));
    size_t n_cells = 0;
    for (const auto& s : c->hs) n_cells += 10 * (size_t)s.ncell + 1;
    c->cells.alloc(sizeof(int32_t) * n_cells);
    HIP_OK(hipMemsetAsync(c->cells.p, 0, sizeof(int32_t) * n_cells, c->stream));
    size_t n_waves = 0;
    for (const auto& s : c->hs) n_waves += blocks_for(s.n, 64);
    c->pair_part.alloc(sizeof(double) * kPairPart * std::max<size_t>(1, n_waves));
    c->vir_part.alloc(sizeof(double) * kVirPart * std::max<size_t>(1, n_waves));
    HIP_OK(hipMemsetAsync(c->vir_part.p, 0, c->vir_part.bytes, c->stream));
    c->fin_part.alloc(sizeof(double) * kFin * kFinBlocks * std::max(R, 1));
    HIP_OK(hipMemsetAsync(c->fin_part.p, 0, c->fin_part.bytes, c->stream));
    c->kin_part.alloc(sizeof(double) * std::max<size_t>(1, n_waves));
    c->flux_part.alloc(sizeof(double) * kFluxPart * std::max<size_t>(1, n_waves));
    c->at_ew.alloc(sizeof(double4) * 2 * N);
    c->ufix.alloc(sizeof(uint4) * N);
    c->scalars.alloc(sizeof(DeviceScalars) * R);
    HIP_OK(hipMemsetAsync(c->scalars.p, 0, sizeof(DeviceScalars) * R, c->stream));
    {
        Plan p1;
        p1.sc = c->scalars.as<DeviceScalars>();
        p1.R = R;
        launch_init_scalars(p1, c->stream);
    }
    {
        double4* P = c->atoms.as<double4>();
        double* d = reinterpret_cast<double*>(P + N);
        int32_t* ip = reinterpret_cast<int32_t*>(d + 12 * N);
        double4* TP = c->sortbuf.as<double4>();
        double* td = reinterpret_cast<double*>(TP + N);
        int32_t* tip = reinterpret_cast<int32_t*>(td + 6 * N);
        int32_t* cells = c->cells.as<int32_t>();
        size_t wav = 0;
        for (int r = 0; r < R; ++r) {
            DevSys& s = c->hs[r];
            const size_t o = (size_t)c->slot_off[r];
            s.p = P + o;
            double** slots[] = {&s.vx, &s.vy, &s.vz, &s.fx, &s.fy, &s.fz, &s.fsx, &s.fsy, &s.fsz, &s.xr, &s.yr, &s.zr};
            for (int t = 0; t < 12; ++t) *slots[t] = d + t * N + o;
            s.type = ip + o;
            s.id = ip + N + o;
            s.inv = ip + 2 * N + o;
            s.tp = TP + o;
            double** tslots[] = {&s.tvx, &s.tvy, &s.tvz, &s.tfx, &s.tfy, &s.tfz};
            for (int t = 0; t < 6; ++t) *tslots[t] = td + t * N + o;
            s.ttype = tip + o;
            s.tid = tip + N + o;
            s.cell_of = tip + 2 * N + o;
            s.slot_of = tip + 3 * N + o;
            s.order = tip + 4 * N + o;
            s.core_cnt = c->counts.as<int32_t>() + o;
            s.cand_cnt = c->counts.as<int32_t>() + N + o;
            s.cell_count = cells;
            s.cell_start = cells + s.ncell;
            s.sub_beg = cells + 2 * (size_t)s.ncell + 1;
            cells += 10 * (size_t)s.ncell + 1;
            s.pair_part = c->pair_part.as<double>() + wav * kPairPart;
            s.vir_part = c->vir_part.as<double>() + wav * kVirPart;
            s.fin_part = c->fin_part.as<double>() + (size_t)r * kFinBlocks * kFin;
            s.kin_part = c->kin_part.as<double>() + wav;
            s.flux_part = c->flux_part.as<double>() + wav * kFluxPart;
            s.at_ew = c->at_ew.as<double4>() + 2 * o;
            s.ufix = c->ufix.as<uint4>() + o;
            wav += blocks_for(s.n, 64);
            s.sc = c->scalars.as<DeviceScalars>() + r;
        }
    }

    // pair coefficient table (shared)
    std::vector<PairCoef> pcs(p0.n_species * p0.n_species);
    for (int i = 0; i < p0.n_species; ++i)
        for (int j = 0; j < p0.n_species; ++j) {
            const rbsog_pair& a = p0.pair[i * RBSOG_MAX_SPECIES + j];
            PairCoef& pc = pcs[i * p0.n_species + j];
            pc.qq = p0.coulomb_k * p0.species[i].q * p0.species[j].q;
            const double rp = p0.r_core_pair[i * RBSOG_MAX_SPECIES + j];
            const double rc = rp > 0.0 ? rp : p0.r_core;
            pc.rc2 = rc * rc;
            pc.rc2_list = (rc + p0.skin) * (rc + p0.skin);
            const double lo = rc - p0.skin;
            pc.lo2_list = lo > 0.0 ? lo * lo : 0.0;
            pc.pad = 0.0;
            pc.A = a.A;
            pc.sig = a.sigma;
            pc.irho = a.rho > 0.0 ? 1.0 / a.rho : 0.0;
            pc.C = a.C;
            pc.D = a.D;
        }
    SpeciesDev spc{};
    for (int t = 0; t < RBSOG_MAX_SPECIES; ++t) {
        spc.q[t] = t < p0.n_species ? p0.species[t].q : 0.0;
        spc.mass[t] = t < p0.n_species ? p0.species[t].mass : 1.0;
        spc.inv_mass_acc[t] = kAccUnit / spc.mass[t];
        spc.self_e[t] = 0.5 * p0.coulomb_k * spc.q[t] * spc.q[t] * wsum;
    }
    const size_t pair_bytes = round_up((int)(sizeof(PairCoef) * pcs.size()), 256);
    c->pair_tab.alloc(pair_bytes + sizeof(SpeciesDev));
    HIP_OK(hipMemcpy(c->pair_tab.p, pcs.data(), sizeof(PairCoef) * pcs.size(), hipMemcpyHostToDevice));
    SpeciesDev* d_spc = reinterpret_cast<SpeciesDev*>(c->pair_tab.as<char>() + pair_bytes);
    HIP_OK(hipMemcpy(d_spc, &spc, sizeof(SpeciesDev), hipMemcpyHostToDevice));
    for (auto& s : c->hs) {
        s.pair = c->pair_tab.as<PairCoef>();
        s.spc = d_spc;
    }

    // list capacities from the densest system; the list kernel from the
    // largest stencil
    int cap_core = 32, cap_cand = 32, list_mode = 0, n_max = 0;
    c->list_mode_r.assign(R, 0);
    for (int r = 0; r < R; ++r) {
        const rbsog_params& p = prm[r];
        const DevSys& s = c->hs[r];
        const int n = s.n;
        n_max = std::max(n_max, n);
        const double V = p.box[0] * p.box[1] * p.box[2];
        const double rho_n = n / V;
        double rc_max = p.r_core, rc_min = p.r_core;
        for (int a = 0; a < p.n_species * p.n_species; ++a) {
            const double r = p.r_core_pair[(a / p.n_species) * RBSOG_MAX_SPECIES + a % p.n_species];
            if (r > 0.0) {
                rc_max = std::max(rc_max, r);
                rc_min = std::min(rc_min, r);
            }
        }
        const double rcl = rc_max + p.skin, lo = rc_min - p.skin, hi = p.r_shell + p.skin;
        const double vc = 4.0 / 3.0 * kPi * rcl * rcl * rcl;
        const double lo3 = lo > 0.0 ? lo * lo * lo : 0.0;
        const double vk = 4.0 / 3.0 * kPi * (hi * hi * hi - lo3);
        // room for local densities well above the mean (melting lattices,
        // clusters); the step loop grows the lists if they still overflow
        cap_core = std::max(cap_core, round_up((int)(1.8 * vc * rho_n) + 32, 32));
        cap_cand = std::max(cap_cand, round_up((int)(1.5 * vk * rho_n) + 32, 32));
        double cell_vol = 1.0;
        for (int a = 0; a < 3; ++a) cell_vol *= p.box[a] / s.nc[a];
        const int ncell_st = (s.nc[0] >= 3 ? 3 : 1) * (s.nc[1] >= 3 ? 3 : 1) * (s.nc[2] >= 3 ? 3 : 1);
        const double stencil = std::min<double>(n, ncell_st * cell_vol * rho_n);
        // the smallest staging capacity that holds the stencil with room for
        // density fluctuations (a cell that still overflows moves the build
        // to the next one)
        const double need = stencil + 5.0 * std::sqrt(stencil) + 32.0;
        int mode = kListPerAtom;
        for (int q = kListPerAtom - 1; q >= 0; --q)
            if (need <= kListCaps[q]) mode = q;
        list_mode = std::max(list_mode, mode);
        c->list_mode_r[r] = mode;
    }
    cap_core = std::min(cap_core, std::max(32, round_up(n_max, 32)));
    cap_cand = std::min(cap_cand, std::max(32, round_up(n_max, 32)));
    c->plan.list_mode = list_mode;

    // k-space: the shared sincos table, then per system its sampling tables
    // (or enumerated modes) and mode arrays
    std::vector<double> table(2 * kTableSize);
    for (int j = 0; j < kTableSize; ++j) {
        table[2 * j] = std::cos(2.0 * kPi * j / kTableSize);
        table[2 * j + 1] = std::sin(2.0 * kPi * j / kTableSize);
    }
    c->ktab.alloc(sizeof(double) * table.size());
    HIP_OK(hipMemcpy(c->ktab.p, table.data(), sizeof(double) * table.size(), hipMemcpyHostToDevice));
    // terms of F^(k) for the k-space virial (shared)
    std::vector<double> sog_c, sog_s2;
    sog_kspace_terms(c->sog, &sog_c, &sog_s2);
    c->sogk.alloc(sizeof(double) * 2 * sog_c.size());
    HIP_OK(hipMemcpy(c->sogk.p, sog_c.data(), sizeof(double) * sog_c.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->sogk.as<double>() + sog_c.size(), sog_s2.data(), sizeof(double) * sog_s2.size(),
                     hipMemcpyHostToDevice));
    std::vector<std::vector<int32_t>> em(R);
    std::vector<std::vector<double>> ecoef(R);
    size_t cdf_doubles = 0, cdf_ints = 0, n_modes_all = 0, rho_part_all = 0;
    for (int r = 0; r < R; ++r) {
        const rbsog_params& p = prm[r];
        KDev& k = c->hk[r];
        k = KDev{};
        k.table = c->ktab.as<double>();
        k.n_sog = (int)sog_c.size();
        k.sog_c = c->sogk.as<double>();
        k.sog_s2 = c->sogk.as<double>() + sog_c.size();
        const double V = p.box[0] * p.box[1] * p.box[2];
        if (p.p_f > 0) {
            build_ktables(c->sog, p.box, &c->kt[r]);
            const KTables& t = c->kt[r];
            k.sampled = 1;
            k.n_modes = p.p_f;
            k.nm = t.nm;
            k.S = t.S;
            k.coef_scale = t.S / ((double)p.p_f * V);
            cdf_doubles += 2 * t.g0cdf.size() + t.comp_cdf.size();
            cdf_ints += 2 * t.off.size();
        } else {
            enumerate_modes(c->sog, p.box, &em[r], &ecoef[r]);
            k.sampled = 0;
            k.n_modes = (int)ecoef[r].size();
            k.S = 0.0;
        }
        const int n = c->hs[r].n;
        const int tiles = (k.n_modes + 63) / 64;
        k.n_modes_pad = std::max(1, tiles) * 64;
        const int max_chunks = std::max(1, (n + 255) / 256);
        k.n_chunks = std::min(max_chunks, std::max(1, (2048 + std::max(tiles, 1) - 1) / std::max(tiles, 1)));
        // a multiple of 16 atoms: the rho kernel splits a chunk into four
        // quarters read four atoms at a time
        k.chunk = (std::max(1, (n + k.n_chunks - 1) / k.n_chunks) + 15) & ~15;
        k.n_chunks = std::max(1, (n + k.chunk - 1) / k.chunk);
        n_modes_all += (size_t)k.n_modes;
        rho_part_all += 2 * (size_t)k.n_chunks * k.n_modes_pad;
    }
    c->kcdf.alloc(sizeof(double) * std::max<size_t>(1, cdf_doubles) + sizeof(int32_t) * cdf_ints);
    c->kmodes.alloc(std::max<size_t>(1, n_modes_all) * (sizeof(ModeRec) + 3 * sizeof(int32_t)));
    c->krho_part.alloc(sizeof(double) * std::max<size_t>(1, rho_part_all));
    c->krho.alloc(sizeof(double) * 3 * std::max<size_t>(1, n_modes_all));  // rho (2), g (1)
    {
        double* dd = c->kcdf.as<double>();
        int32_t* di = reinterpret_cast<int32_t*>(dd + cdf_doubles);
        ModeRec* mr = c->kmodes.as<ModeRec>();
        int32_t* mm = reinterpret_cast<int32_t*>(mr + std::max<size_t>(1, n_modes_all));
        double* rp = c->krho_part.as<double>();
        double* rh = c->krho.as<double>();
        double* gh = rh + 2 * std::max<size_t>(1, n_modes_all);
        auto put = [](void* dst, const void* src, size_t b) {
            if (b) HIP_OK(hipMemcpy(dst, src, b, hipMemcpyHostToDevice));
        };
        for (int r = 0; r < R; ++r) {
            KDev& k = c->hk[r];
            if (k.sampled) {
                const KTables& t = c->kt[r];
                const size_t nt = t.g0cdf.size();
                put(dd, t.g0cdf.data(), sizeof(double) * nt);
                put(dd + nt, t.g2cdf.data(), sizeof(double) * nt);
                put(dd + 2 * nt, t.comp_cdf.data(), sizeof(double) * t.comp_cdf.size());
                k.g0cdf = dd;
                k.g2cdf = dd + nt;
                k.comp_cdf = dd + 2 * nt;
                dd += 2 * nt + t.comp_cdf.size();
                put(di, t.off.data(), sizeof(int32_t) * t.off.size());
                put(di + t.off.size(), t.len.data(), sizeof(int32_t) * t.len.size());
                k.off = di;
                k.len = di + t.off.size();
                di += 2 * t.off.size();
            }
            k.modes = mr;
            k.m = mm;
            if (!k.sampled && k.n_modes > 0) {
                std::vector<ModeRec> recs(k.n_modes);
                for (int q = 0; q < k.n_modes; ++q)
                    recs[q] = ModeRec{(double)em[r][3 * q], (double)em[r][3 * q + 1], (double)em[r][3 * q + 2],
                                      0.0, 0.0, ecoef[r][q], 0.0, 0.0f, 0.0f};
                put(k.modes, recs.data(), sizeof(ModeRec) * k.n_modes);
                put(k.m, em[r].data(), sizeof(int32_t) * em[r].size());
            }
            mr += k.n_modes;
            mm += 3 * (size_t)k.n_modes;
            k.rho_part = rp;
            rp += 2 * (size_t)k.n_chunks * k.n_modes_pad;
            k.rho = rh;
            rh += 2 * (size_t)k.n_modes;
            k.mode_g = gh;
            gh += (size_t)k.n_modes;
        }
    }

    plan_lists(c, cap_core, cap_cand);  // also uploads the system records
    plan_launches(c);

    // inputs
    if (n_user > 0) {
        const int32_t* dt_ = type;
        const double* dp = pos;
        const double* dv = vel;
        DBuf stage;
        if (!on_device) {
            stage.alloc(sizeof(int32_t) * n_user + sizeof(double) * 6 * (size_t)n_user);
            double* sp = stage.as<double>();
            HIP_OK(hipMemcpy(sp, hp.data(), sizeof(double) * 3 * n_user, hipMemcpyHostToDevice));
            dp = sp;
            if (vel) {
                HIP_OK(hipMemcpy(sp + 3 * (size_t)n_user, hv.data(), sizeof(double) * 3 * n_user,
                                 hipMemcpyHostToDevice));
                dv = sp + 3 * (size_t)n_user;
            }
            int32_t* tp = reinterpret_cast<int32_t*>(sp + 6 * (size_t)n_user);
            HIP_OK(hipMemcpy(tp, ht.data(), sizeof(int32_t) * n_user, hipMemcpyHostToDevice));
            dt_ = tp;
        }
        launch_from_user(c->plan, dt_, dp, dv, c->stream);
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    c->have_system = true;
    c->eval = 0;
    c->forces_valid = false;
    c->stale = false;
    c->nonfinite = false;
    build_checked(c);
    HIP_OK(hipStreamSynchronize(c->stream));
}

void need_system(rbsog_ctx* c) { require(c->have_system, RBSOG_E_STATE, "no system set"); }

}  // namespace

extern "C" {

const char* rbsog_version(void) { return "librbsog 0.2 (gfx950)"; }

rbsog_status rbsog_sog_params(double eps, double r_shell, double* b, double* s, double* x_c, int32_t* M, double* w,
                              int32_t w_cap)
{
    try {
        if (!(r_shell > 0.0)) return RBSOG_E_ARG;
        SogSplit sp;
        std::string err;
        if (!sog_split(eps, r_shell, &sp, &err)) return RBSOG_E_ARG;
        if (b) *b = sp.b;
        if (s) *s = sp.s;
        if (x_c) *x_c = sp.x_c;
        if (M) *M = sp.M;
        if (w) {
            if (w_cap < sp.M + 1) return RBSOG_E_ARG;
            for (int m = 0; m <= sp.M; ++m) w[m] = sp.w[m];
        }
        return RBSOG_OK;
    } catch (...) {
        return RBSOG_E_ARG;
    }
}

rbsog_status rbsog_near_table(double eps, double r_shell, float* coef, int32_t cap, int32_t* e0,
                              int32_t* n_intervals)
{
    try {
        if (!(r_shell > 0.0)) return RBSOG_E_ARG;
        SogSplit sp;
        std::string err;
        if (!sog_split(eps > 0.0 ? eps : 1e-5, r_shell, &sp, &err)) return RBSOG_E_ARG;
        NearTable nt;
        build_near_table(sp, r_shell, &nt);
        const int n = nt.nbin * kNearSub;
        if (e0) *e0 = nt.e0;
        if (n_intervals) *n_intervals = n;
        if (coef) {
            if (cap < 8 * n) return RBSOG_E_ARG;
            std::memcpy(coef, nt.coef.data(), sizeof(float) * nt.coef.size());
        }
        return RBSOG_OK;
    } catch (...) {
        return RBSOG_E_ARG;
    }
}

rbsog_status rbsog_create(rbsog_ctx** out, int hip_device, void* hip_stream)
{
    if (!out) return RBSOG_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return RBSOG_E_HIP;
    if (hip_device < 0 || hip_device >= count) return RBSOG_E_ARG;
    rbsog_ctx* c = new (std::nothrow) rbsog_ctx();
    if (!c) return RBSOG_E_OOM;
    c->device = hip_device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(hip_device) != hipSuccess) {
        delete c;
        return RBSOG_E_HIP;
    }
    // device address of the allocation-free entry point's scratch, once per device
    const char* why = nullptr;
    if (!noalloc_init(hip_device, &why)) {
        delete c;
        return RBSOG_E_HIP;
    }
    *out = c;
    return RBSOG_OK;
}

rbsog_status rbsog_destroy(rbsog_ctx* ctx)
{
    if (!ctx) return RBSOG_E_ARG;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    delete ctx;
    return RBSOG_OK;
}

const char* rbsog_last_error(const rbsog_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

rbsog_status rbsog_set_system(rbsog_ctx* ctx, const rbsog_params* p, const int32_t* type, const double* pos,
                              const double* vel, int ptrs_on_device)
{
    return guarded(ctx, [&] {
        ctx->have_system = false;
        set_batch_impl(ctx, 1, p, type, pos, vel, ptrs_on_device);
    });
}

rbsog_status rbsog_set_batch(rbsog_ctx* ctx, int32_t n_sys, const rbsog_params* p, const int32_t* type,
                             const double* pos, const double* vel, int ptrs_on_device)
{
    return guarded(ctx, [&] {
        ctx->have_system = false;
        set_batch_impl(ctx, n_sys, p, type, pos, vel, ptrs_on_device);
    });
}

rbsog_status rbsog_n_systems(rbsog_ctx* ctx, int32_t* n_sys)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(n_sys != nullptr, RBSOG_E_ARG, "n_sys is NULL");
        *n_sys = ctx->R;
    });
}

rbsog_status rbsog_select_system(rbsog_ctx* ctx, int32_t r)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(r >= 0 && r < ctx->R, RBSOG_E_ARG, "system index out of range");
        ctx->sel = r;
    });
}

rbsog_status rbsog_autotune(rbsog_ctx* ctx, int32_t reps, rbsog_tuning* chosen)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(reps >= 1, RBSOG_E_ARG, "reps < 1");
        need_finite(ctx);
        require(!ctx->stale, RBSOG_E_LIST_STALE, "lists are stale; call rbsog_build_lists before tuning");
        autotune(ctx, reps);
        if (chosen) {
            const Tuning& t = ctx->plan.tune;
            *chosen = rbsog_tuning{t.pair_block, t.pair_ku, t.rho_mpl, t.kf_block, t.kf_aux};
        }
    });
}

rbsog_status rbsog_set_tuning(rbsog_ctx* ctx, const rbsog_tuning* t)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(t != nullptr, RBSOG_E_ARG, "tuning is NULL");
        auto one_of = [](int v, std::initializer_list<int> ok) {
            for (int x : ok)
                if (v == x) return true;
            return false;
        };
        require(one_of(t->pair_block, {64, 128, 256}) && one_of(t->pair_ku, {4, 8}) && one_of(t->rho_mpl, {1, 2}) &&
                    one_of(t->kf_block, {64, 128, 256}) && one_of(t->kf_aux, {0, 1}),
                RBSOG_E_ARG, "tuning value out of range");
        ctx->plan.tune = Tuning{t->pair_block, t->pair_ku, t->rho_mpl, t->kf_block, t->kf_aux};
        plan_launches(ctx);
    });
}

rbsog_status rbsog_get_tuning(rbsog_ctx* ctx, rbsog_tuning* t)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(t != nullptr, RBSOG_E_ARG, "tuning is NULL");
        const Tuning& u = ctx->plan.tune;
        *t = rbsog_tuning{u.pair_block, u.pair_ku, u.rho_mpl, u.kf_block, u.kf_aux};
    });
}

rbsog_status rbsog_use_graphs(rbsog_ctx* ctx, int enable)
{
    return guarded(ctx, [&] {
        ctx->drop_graphs();
        ctx->use_graph = enable != 0;
    });
}

rbsog_status rbsog_build_lists(rbsog_ctx* ctx)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        need_finite(ctx);
        build_checked(ctx);
        ctx->stale = false;
    });
}

rbsog_status rbsog_set_positions(rbsog_ctx* ctx, const double* pos, int ptrs_on_device)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        need_finite(ctx);
        require(pos != nullptr || ctx->n_user == 0, RBSOG_E_ARG, "pos is NULL");
        const int n = ctx->n_user;
        if (n == 0) return;
        std::vector<double> hp(3 * (size_t)n);
        if (ptrs_on_device)
            HIP_OK(hipMemcpy(hp.data(), pos, sizeof(double) * hp.size(), hipMemcpyDeviceToHost));
        else
            std::memcpy(hp.data(), pos, sizeof(double) * hp.size());
        for (double v : hp) require(std::isfinite(v), RBSOG_E_NONFINITE, "non-finite position");
        ctx->export_tmp.alloc(sizeof(double) * hp.size());
        HIP_OK(hipMemcpyAsync(ctx->export_tmp.p, hp.data(), sizeof(double) * hp.size(), hipMemcpyHostToDevice,
                              ctx->stream));
        launch_set_positions(ctx->plan, ctx->export_tmp.as<double>(), ctx->stream);
        HIP_OK(hipGetLastError());
        bool stale = false;
        for (const auto& h : read_scalars(ctx)) stale = stale || h.stale != 0;
        ctx->stale = stale;
        ctx->forces_valid = false;
    });
}

rbsog_status rbsog_compute_forces(rbsog_ctx* ctx, uint64_t eval, double* force_out, rbsog_energy* e_out)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        need_finite(ctx);
        require(!ctx->stale, RBSOG_E_LIST_STALE,
                "an atom moved more than skin/2 since the last list build; call rbsog_build_lists");
        launch_set_eval(ctx->plan, eval, ctx->stream);
        enqueue_forces(ctx, e_out != nullptr, false);
        ctx->eval = eval;
        ctx->forces_valid = true;
        if (force_out) launch_to_user3(ctx->plan, Field::force, force_out, ctx->stream);
        if (e_out) {
            const auto h = read_scalars(ctx);
            check_flags(ctx, h);
            fill_energy(ctx, h, e_out);
        }
    });
}

rbsog_status rbsog_get_force_parts(rbsog_ctx* ctx, double* f_short, double* f_kspace)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(ctx->forces_valid, RBSOG_E_STATE, "no force evaluation yet");
        if (f_short) launch_to_user3(ctx->plan, Field::short_force, f_short, ctx->stream);
        if (f_kspace) launch_kspace_part(ctx->plan, f_kspace, ctx->stream);
    });
}

}  // extern "C"

namespace {

void step_impl(rbsog_ctx* ctx, int32_t n_steps, rbsog_energy* e_last)
{
    {
        need_system(ctx);
        need_finite(ctx);
        require(n_steps >= 0, RBSOG_E_ARG, "n_steps < 0");
        if (n_steps == 0) return;
        if (ctx->stale) {
            // positions set by the caller outran the lists: an extra build
            build_checked(ctx);
            ctx->stale = false;
            ctx->forces_valid = false;
        }
        if (!ctx->forces_valid) {
            // forces at the current positions start the integrator
            launch_set_eval(ctx->plan, ctx->eval, ctx->stream);
            enqueue_forces(ctx, false, false);
            ctx->forces_valid = true;
        }
        launch_set_eval(ctx->plan, ctx->eval, ctx->stream);
        if (any_thermostat(ctx)) {
            // velocity factor of the first step from the current velocities
            launch_kinetic(ctx->plan, ctx->stream);
            launch_kinetic_finalize(ctx->plan, false, false, ctx->stream);
        }
        const int every = ctx->prm[0].rebuild_every;
        // a list overflow inside the loop restarts the call from a snapshot
        // with larger lists
        for (int attempt = 0;; ++attempt) {
            snapshot(ctx, true);
            for (int k = 0; k < n_steps; ++k) {
                const uint64_t step = ctx->eval + 1 + (uint64_t)k;
                const bool scheduled = step % (uint64_t)every == 0;
                const bool energy = e_last != nullptr && k == n_steps - 1;
                launch_step(ctx, scheduled, energy);
            }
            const auto h = read_scalars(ctx);
            check_finite(ctx, h);
            const int o = any_overflow(h);
            if (o == 0) {
                ctx->eval += (uint64_t)n_steps;
                if (e_last) fill_energy(ctx, h, e_last);
                return;
            }
            require(attempt < 4 && (o & 2) == 0, RBSOG_E_CAPACITY, "list capacity exceeded in the step loop");
            grow_after_overflow(ctx, o);
            snapshot(ctx, false);
            build_checked(ctx);
            launch_set_eval(ctx->plan, ctx->eval, ctx->stream);
            if (any_thermostat(ctx)) {
                launch_kinetic(ctx->plan, ctx->stream);
                launch_kinetic_finalize(ctx->plan, false, false, ctx->stream);
            }
        }
    }
}

}  // namespace

extern "C" {

rbsog_status rbsog_step(rbsog_ctx* ctx, int32_t n_steps, rbsog_energy* e_last)
{
    return guarded(ctx, [&] { step_impl(ctx, n_steps, e_last); });
}

rbsog_status rbsog_step_batch(rbsog_ctx* ctx, int32_t n_steps)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(ctx->stream != nullptr, RBSOG_E_STATE,
                "rbsog_step_batch replays captured step graphs: create the context on a non-default stream");
        struct Restore {
            rbsog_ctx* c;
            bool was;
            ~Restore() { c->use_graph = was; }
        } restore{ctx, ctx->use_graph};
        ctx->use_graph = true;
        step_impl(ctx, n_steps, nullptr);
    });
}

rbsog_status rbsog_get_state(rbsog_ctx* ctx, double* pos, double* vel, double* force, uint64_t* eval,
                             int ptrs_on_device)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const int n = ctx->n_user;
        const size_t bytes = sizeof(double) * 3 * (size_t)n;
        double* outs[3] = {pos, vel, force};
        if (!ptrs_on_device && n > 0 && (pos || vel || force)) ctx->export_tmp.alloc(bytes);
        for (int q = 0; q < 3; ++q) {
            if (!outs[q] || n <= 0) continue;
            double* dst = ptrs_on_device ? outs[q] : ctx->export_tmp.as<double>();
            if (q == 0)
                launch_pos_to_user(ctx->plan, dst, ctx->stream);
            else
                launch_to_user3(ctx->plan, q == 1 ? Field::velocity : Field::force, dst, ctx->stream);
            if (!ptrs_on_device) {
                HIP_OK(hipMemcpyAsync(outs[q], dst, bytes, hipMemcpyDeviceToHost, ctx->stream));
                HIP_OK(hipStreamSynchronize(ctx->stream));
            }
        }
        if (eval) *eval = ctx->eval;
    });
}

rbsog_status rbsog_profile_enable(rbsog_ctx* ctx, int enable)
{
    return guarded(ctx, [&] {
        require(enable >= 0 && enable <= 2, RBSOG_E_ARG, "profile mode is 0, 1 or 2");
        ctx->profiling = enable != 0;
        ctx->hot_only = enable == 2;
    });
}

rbsog_status rbsog_profile_read(rbsog_ctx* ctx, double* ms, int64_t* launches)
{
    return guarded(ctx, [&] {
        HIP_OK(hipStreamSynchronize(ctx->stream));
        double acc[RBSOG_N_PHASES] = {0};
        int64_t cnt[RBSOG_N_PHASES] = {0};
        for (auto& r : ctx->recs) {
            float t = 0.f;
            HIP_OK(hipEventElapsedTime(&t, r.a, r.b));
            acc[r.phase] += t;
            cnt[r.phase] += 1;
            ctx->pool.push_back(r.a);
            ctx->pool.push_back(r.b);
        }
        ctx->recs.clear();
        for (int q = 0; q < RBSOG_N_PHASES; ++q) {
            if (ms) ms[q] = acc[q];
            if (launches) launches[q] = cnt[q];
        }
    });
}

rbsog_status rbsog_get_list_counts(rbsog_ctx* ctx, int32_t* n_core, int32_t* n_cand)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const DevSys& s = ctx->hs[ctx->sel];
        const int n = s.n;
        std::vector<int32_t> nc(n), nk(n), id(n);
        HIP_OK(hipStreamSynchronize(ctx->stream));
        if (n > 0) {
            HIP_OK(hipMemcpy(nc.data(), s.core_cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(nk.data(), s.cand_cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(id.data(), s.id, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        }
        for (int t = 0; t < n; ++t) {
            if (n_core) n_core[id[t]] = nc[t];
            if (n_cand) n_cand[id[t]] = nk[t];
        }
    });
}

rbsog_status rbsog_get_lists_of(rbsog_ctx* ctx, int32_t i, int32_t* core, int32_t* cand)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const DevSys& s = ctx->hs[ctx->sel];
        require(i >= 0 && i < s.n, RBSOG_E_ARG, "atom index out of range");
        HIP_OK(hipStreamSynchronize(ctx->stream));
        std::vector<int32_t> id(s.n);
        HIP_OK(hipMemcpy(id.data(), s.id, sizeof(int32_t) * s.n, hipMemcpyDeviceToHost));
        int32_t t = 0, nc = 0, nk = 0;
        HIP_OK(hipMemcpy(&t, s.inv + i, sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(&nc, s.core_cnt + t, sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(&nk, s.cand_cnt + t, sizeof(int32_t), hipMemcpyDeviceToHost));
        nc = std::min(nc, s.cap_core - 1);
        nk = std::min(nk, s.cap_cand - 1);
        if (core) {
            std::vector<int32_t> tile((size_t)s.cap_core * 64);
            const int32_t* src = s.core_idx + (size_t)(t >> 6) * s.cap_core * 64;
            HIP_OK(hipMemcpy(tile.data(), src, sizeof(int32_t) * tile.size(), hipMemcpyDeviceToHost));
            std::vector<int32_t> ids(nc);
            for (int q = 0; q < nc; ++q) ids[q] = id[tile[(size_t)q * 64 + (t & 63)]];
            std::sort(ids.begin(), ids.end());
            std::copy(ids.begin(), ids.end(), core);
        }
        require(!(cand && s.shell_stored), RBSOG_E_STATE,
                "the stored-batch form keeps no candidate lists after the build");
        if (cand) {
            std::vector<int32_t> row(std::max(nk, 1));
            if (nk > 0)
                HIP_OK(hipMemcpy(row.data(), s.cand_idx + (size_t)t * s.cap_cand, sizeof(int32_t) * nk,
                                 hipMemcpyDeviceToHost));
            for (int q = 0; q < nk; ++q) cand[q] = id[row[q]];
        }
    });
}

rbsog_status rbsog_msd(rbsog_ctx* ctx, int32_t mark, double* msd)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const int r = ctx->sel;
        const DevSys& s = ctx->hs[r];
        require(mark != 0 || ctx->msd_marked[r], RBSOG_E_STATE, "msd: no origin marked for this system");
        const size_t nu = (size_t)std::max(ctx->n_user, 1);
        if (!ctx->msd_buf.p) ctx->msd_buf.alloc(sizeof(double) * 6 * nu);
        const size_t waves = (size_t)std::max(1, (s.n + 63) / 64);
        DBuf part;
        part.alloc(sizeof(double) * 2 * kMaxSpecies * waves);
        HIP_OK(hipMemsetAsync(part.p, 0, part.bytes, ctx->stream));
        double* last = ctx->msd_buf.as<double>();
        const Plan P1 = one(ctx, r);
        launch_msd(P1, last, last + 3 * nu, part.as<double>(), mark != 0, ctx->stream);
        HIP_OK(hipGetLastError());
        std::vector<double> h(2 * kMaxSpecies * waves);
        HIP_OK(hipMemcpyAsync(h.data(), part.p, part.bytes, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
        if (mark) ctx->msd_marked[r] = 1;
        if (msd)
            for (int a = 0; a < s.n_species; ++a) {
                double q = 0.0, n = 0.0;
                for (size_t w = 0; w < waves; ++w) {
                    q += h[w * 2 * kMaxSpecies + a];
                    n += h[w * 2 * kMaxSpecies + kMaxSpecies + a];
                }
                msd[a] = n > 0.0 ? q / n : 0.0;
            }
    });
}

rbsog_status rbsog_rdf_counts(rbsog_ctx* ctx, double r_max, int32_t n_bins, uint64_t* counts)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const DevSys& s = ctx->hs[ctx->sel];
        const rbsog_params& p = ctx->prm[ctx->sel];
        require(n_bins >= 1 && r_max > 0.0 && r_max <= p.r_shell, RBSOG_E_ARG,
                "rdf: need n_bins >= 1 and 0 < r_max <= r_shell");
        const int S = s.n_species;
        require((long long)S * S * n_bins <= 16384, RBSOG_E_ARG, "rdf: n_species^2 * n_bins > 16384");
        require(!s.shell_stored, RBSOG_E_STATE, "rdf: the memory form keeps no candidate rows");
        require(counts != nullptr, RBSOG_E_ARG, "rdf: counts is NULL");
        const size_t nh = (size_t)S * S * n_bins;
        DBuf out;
        out.alloc(sizeof(unsigned long long) * nh);
        HIP_OK(hipMemsetAsync(out.p, 0, out.bytes, ctx->stream));
        const Plan P1 = one(ctx, ctx->sel);
        launch_rdf(P1, S, r_max / (double)n_bins, n_bins, out.as<unsigned long long>(), ctx->stream);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(counts, out.p, out.bytes, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
    });
}

rbsog_status rbsog_rdf_counts_noalloc(rbsog_ctx* ctx, double r_max, int32_t n_bins, uint64_t* counts)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const DevSys& s = ctx->hs[ctx->sel];
        const rbsog_params& p = ctx->prm[ctx->sel];
        require(n_bins >= 1 && r_max > 0.0 && r_max <= p.r_shell, RBSOG_E_ARG,
                "rdf: need n_bins >= 1 and 0 < r_max <= r_shell");
        const int S = s.n_species;
        require((long long)S * S * n_bins <= kRdfScratch, RBSOG_E_ARG,
                "rdf (allocation-free): n_species^2 * n_bins exceeds the 16384 counters of the static scratch");
        require(!s.shell_stored, RBSOG_E_STATE, "rdf: the memory form keeps no candidate rows");
        require(counts != nullptr, RBSOG_E_ARG, "rdf: counts is NULL");
        unsigned long long* d = noalloc_scratch(ctx->device);
        require(d != nullptr, RBSOG_E_STATE, "allocation-free scratch not set up on this device");
        const int nh = S * S * n_bins;
        launch_zero_u64(d, nh, ctx->stream);
        const Plan P1 = one(ctx, ctx->sel);
        launch_rdf(P1, S, r_max / (double)n_bins, n_bins, d, ctx->stream);
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(counts, d, sizeof(unsigned long long) * (size_t)nh, hipMemcpyDeviceToHost, ctx->stream));
        HIP_OK(hipStreamSynchronize(ctx->stream));
    });
}

rbsog_status rbsog_get_shell_ranks(rbsog_ctx* ctx, uint64_t eval, int32_t* n_ranks, int32_t* ranks)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const DevSys& s = ctx->hs[ctx->sel];
        require(!s.shell_stored, RBSOG_E_STATE, "a stored shell batch is exported by rbsog_get_shell_batch");
        const Plan P1 = one(ctx, ctx->sel);
        const int P = std::max(s.p_r, 1);
        DBuf out;
        out.alloc(sizeof(int32_t) * ((size_t)s.n * P + s.n + 1));
        int32_t* r = out.as<int32_t>();
        int32_t* cnt = r + (size_t)s.n * P;
        launch_set_eval(P1, eval, ctx->stream);
        launch_shell_ranks(P1, r, cnt, ctx->stream);
        launch_set_eval(P1, ctx->eval, ctx->stream);
        HIP_OK(hipStreamSynchronize(ctx->stream));
        std::vector<int32_t> h((size_t)s.n * P), hc(s.n);
        if (s.n > 0) {
            HIP_OK(hipMemcpy(h.data(), r, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(hc.data(), cnt, sizeof(int32_t) * hc.size(), hipMemcpyDeviceToHost));
        }
        for (int u = 0; u < s.n; ++u) {
            if (n_ranks) n_ranks[u] = hc[u];
            if (ranks && s.p_r > 0) {
                int32_t* row = h.data() + (size_t)u * P;
                std::sort(row, row + hc[u]);
                for (int q = 0; q < P; ++q) ranks[(size_t)u * P + q] = q < hc[u] ? row[q] : -1;
            }
        }
    });
}

rbsog_status rbsog_get_shell_batch(rbsog_ctx* ctx, int32_t* n_cand, int32_t* ids)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const DevSys& s = ctx->hs[ctx->sel];
        require(s.shell_stored, RBSOG_E_STATE, "no stored shell batch (RBSOG_FLAG_SHELL_STORED is off)");
        const Plan P1 = one(ctx, ctx->sel);
        const int P = s.p_r;
        DBuf out;
        out.alloc(sizeof(int32_t) * ((size_t)s.n * P + s.n + 1));
        int32_t* d = out.as<int32_t>();
        int32_t* cnt = d + (size_t)s.n * P;
        launch_batch_ids(P1, d, cnt, ctx->stream);
        HIP_OK(hipStreamSynchronize(ctx->stream));
        if (s.n > 0) {
            if (ids) HIP_OK(hipMemcpy(ids, d, sizeof(int32_t) * (size_t)s.n * P, hipMemcpyDeviceToHost));
            if (n_cand) HIP_OK(hipMemcpy(n_cand, cnt, sizeof(int32_t) * s.n, hipMemcpyDeviceToHost));
        }
    });
}

rbsog_status rbsog_get_shell_samples(rbsog_ctx* ctx, int32_t* n_cand, int32_t* idx)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const DevSys& s = ctx->hs[ctx->sel];
        require(s.p_r >= 1, RBSOG_E_STATE, "p_r <= 0: every candidate is taken, there is no sample to export");
        require(s.shell_stored || ctx->forces_valid, RBSOG_E_STATE, "no force evaluation yet");
        const Plan P1 = one(ctx, ctx->sel);
        const int P = s.p_r;
        DBuf out;
        out.alloc(sizeof(int32_t) * ((size_t)s.n * P + s.n + 1));
        int32_t* d = out.as<int32_t>();
        int32_t* cnt = d + (size_t)s.n * P;
        if (s.shell_stored)
            launch_batch_ids(P1, d, cnt, ctx->stream);
        else
            launch_shell_samples(P1, d, cnt, ctx->stream);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(ctx->stream));
        std::vector<int32_t> h((size_t)s.n * P), hc(s.n);
        if (s.n > 0) {
            HIP_OK(hipMemcpy(h.data(), d, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(hc.data(), cnt, sizeof(int32_t) * hc.size(), hipMemcpyDeviceToHost));
        }
        for (int u = 0; u < s.n; ++u) {
            if (n_cand) n_cand[u] = hc[u];
            if (idx) {
                int32_t* row = h.data() + (size_t)u * P;
                const int k = std::min(hc[u], P);
                std::sort(row, row + k);
                std::copy(row, row + P, idx + (size_t)u * P);
            }
        }
    });
}

rbsog_status rbsog_set_list_capacity(rbsog_ctx* ctx, int32_t cap_core, int32_t cap_cand, int32_t* got_core,
                                     int32_t* got_cand)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(cap_core >= 8 && cap_core <= 4096 && cap_cand >= 8 && cap_cand <= 4096, RBSOG_E_ARG,
                "capacities out of range (8..4096)");
        need_finite(ctx);
        plan_lists(ctx, cap_core, cap_cand);
        plan_launches(ctx);
        build_checked(ctx);
        ctx->stale = false;
        ctx->forces_valid = false;
        if (got_core) *got_core = ctx->plan.cap_core;
        if (got_cand) *got_cand = ctx->plan.cap_cand;
    });
}

rbsog_status rbsog_set_list_chunks(rbsog_ctx* ctx, int32_t chunks)
{
    return guarded(ctx, [&] {
        require(chunks >= 1 && chunks <= kMaxListChunks, RBSOG_E_ARG, "chunks out of range (1..64)");
        ctx->list_chunks = chunks;  // used by the next rbsog_set_system / rbsog_set_batch
    });
}

rbsog_status rbsog_get_kmodes(rbsog_ctx* ctx, uint64_t eval, int32_t* m, double* S)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const KDev& k = ctx->hk[ctx->sel];
        if (S) *S = k.S;
        if (!m || k.n_modes <= 0) return;
        if (k.sampled) {
            const Plan P1 = one(ctx, ctx->sel);
            launch_set_eval(P1, eval, ctx->stream);
            launch_ksample(P1, ctx->stream);
            launch_set_eval(P1, ctx->eval, ctx->stream);
        }
        HIP_OK(hipStreamSynchronize(ctx->stream));
        HIP_OK(hipMemcpy(m, k.m, sizeof(int32_t) * 3 * (size_t)k.n_modes, hipMemcpyDeviceToHost));
    });
}

rbsog_status rbsog_get_rho(rbsog_ctx* ctx, double* rho)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(rho != nullptr, RBSOG_E_ARG, "rho is NULL");
        const KDev& k = ctx->hk[ctx->sel];
        HIP_OK(hipStreamSynchronize(ctx->stream));
        if (k.n_modes > 0)
            HIP_OK(hipMemcpy(rho, k.rho, sizeof(double) * 2 * (size_t)k.n_modes, hipMemcpyDeviceToHost));
    });
}

rbsog_status rbsog_get_sog(rbsog_ctx* ctx, double* b, double* s, double* x_c, int32_t* M, double* w, int32_t w_cap)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        const SogSplit& sp = ctx->sog;
        if (b) *b = sp.b;
        if (s) *s = sp.s;
        if (x_c) *x_c = sp.x_c;
        if (M) *M = sp.M;
        if (w) {
            require(w_cap >= sp.M + 1, RBSOG_E_ARG, "w_cap too small");
            for (int m = 0; m <= sp.M; ++m) w[m] = sp.w[m];
        }
    });
}

}  // extern "C"
