// C ABI of librbsog (declared in include/rbsog.h): context, validation,
// planning, kernel sequencing, HIP-graph replay of the step loop, exports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
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
    rbsog_params prm{};
    bool mixed = false;
    SogSplit sog;
    int chain = 1;
    SogCoef coef{};
    KTables kt;
    double u_self = 0.0;
    uint64_t eval = 0;       // eval index of the last force evaluation
    bool forces_valid = false;

    DevSys s{};
    KDev k{};
    int n_pair_blocks = 0;
    int n_kin_blocks = 0;

    // device memory
    DBuf atoms, sortbuf, cells, lists_core, lists_cand, counts, pair_tab, scalars;
    DBuf ktab, kcdf, kmodes, krho_part, krho, pair_part, kin_part, export_tmp, snap;

    // phase timing
    bool profiling = false;
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
    void begin(int phase)
    {
        if (!profiling) return;
        open_phase = phase;
        open_a = take_event();
        (void)hipEventRecord(open_a, stream);
    }
    void end()
    {
        if (!profiling || open_phase < 0) return;
        hipEvent_t b = take_event();
        (void)hipEventRecord(b, stream);
        recs.push_back(Rec{open_phase, open_a, b});
        open_phase = -1;
        open_a = nullptr;
    }

    // step graph
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_kind = -1;  // 0: plain step, 1: step with rebuild

    ~rbsog_ctx()
    {
        drop_graph();
        for (auto& r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }

    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        graph_kind = -1;
    }
};

namespace {

constexpr int kBlock = 256;

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
    for (int a = 0; a < 3; ++a) {
        require(std::isfinite(p->box[a]) && p->box[a] > 0.0, RBSOG_E_ARG, "box must be positive");
        require(p->box[a] >= 2.0 * (p->r_shell + p->skin), RBSOG_E_BOX,
                "box shorter than 2 (r_shell + skin) along an axis");
    }
    const int S = p->n_species;
    for (int i = 0; i < S; ++i) {
        require(p->species[i].mass > 0.0, RBSOG_E_ARG, "species mass must be positive");
        for (int j = 0; j < S; ++j) {
            const rbsog_pair& a = p->pair[i * RBSOG_MAX_SPECIES + j];
            const rbsog_pair& b = p->pair[j * RBSOG_MAX_SPECIES + i];
            require(a.A == b.A && a.sigma == b.sigma && a.rho == b.rho && a.C == b.C && a.D == b.D, RBSOG_E_ARG,
                    "pair table must be symmetric");
            require(a.rho > 0.0 || a.A == 0.0, RBSOG_E_ARG, "rho must be positive");
        }
    }
}

DevSys& sys(rbsog_ctx* c) { return c->s; }

void plan_lists(rbsog_ctx* c, int cap_core, int cap_cand)
{
    DevSys& s = c->s;
    const int n = s.n;
    s.cap_core = cap_core;
    s.cap_cand = cap_cand;
    const size_t tiles = (size_t)(n + 63) / 64;
    c->lists_core.alloc(sizeof(int32_t) * std::max<size_t>(1, tiles * 64 * cap_core));
    c->lists_cand.alloc(sizeof(int32_t) * std::max<size_t>(1, (size_t)n * cap_cand));
    s.core_idx = c->lists_core.as<int32_t>();
    s.cand_idx = c->lists_cand.as<int32_t>();
}

void enqueue_build(rbsog_ctx* c, bool gate)
{
    DevSys& s = c->s;
    if (s.n <= 0) return;
    c->begin(RBSOG_PHASE_BUILD);
    launch_build(s, gate, c->stream);
    c->end();
}

DeviceScalars read_scalars(rbsog_ctx* c)
{
    DeviceScalars h{};
    HIP_OK(hipMemcpyAsync(&h, c->s.sc, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return h;
}

// Per-atom state (cell order) and device scalars at the start of a step call,
// for a restart after a list overflow.
void snapshot(rbsog_ctx* c, bool save)
{
    DevSys& s = c->s;
    const size_t N = (size_t)std::max(s.n, 1);
    const size_t bytes = N * (10 * sizeof(double) + 3 * sizeof(int32_t)) + sizeof(DeviceScalars);
    if (save && c->snap.bytes < bytes) c->snap.alloc(bytes);
    double* d = c->snap.as<double>();
    double* arr[6] = {s.vx, s.vy, s.vz, s.fx, s.fy, s.fz};
    int32_t* iar[3] = {s.type, s.id, s.inv};
    int32_t* ip = reinterpret_cast<int32_t*>(d + 10 * N);
    auto cp = [&](void* dst, const void* src, size_t b) {
        HIP_OK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, c->stream));
    };
    if (save)
        cp(d, s.p, sizeof(double4) * s.n);
    else
        cp(s.p, d, sizeof(double4) * s.n);
    for (int q = 0; q < 6; ++q) {
        if (save)
            cp(d + (4 + q) * N, arr[q], sizeof(double) * s.n);
        else
            cp(arr[q], d + (4 + q) * N, sizeof(double) * s.n);
    }
    for (int q = 0; q < 3; ++q) {
        if (save)
            cp(ip + q * N, iar[q], sizeof(int32_t) * s.n);
        else
            cp(iar[q], ip + q * N, sizeof(int32_t) * s.n);
    }
    void* sc_copy = ip + 3 * N;
    if (save)
        cp(sc_copy, s.sc, sizeof(DeviceScalars));
    else
        cp(s.sc, sc_copy, sizeof(DeviceScalars));
}

// Grow list capacities from the true counts of the last build.
void grow_lists(rbsog_ctx* c)
{
    const DeviceScalars h = read_scalars(c);
    const int mc = h.max_core, mk = h.max_cand;
    const int cap_core = std::max(c->s.cap_core, round_up(mc + mc / 4 + 8, 32));
    const int cap_cand = std::max(c->s.cap_cand, round_up(mk + mk / 4 + 8, 32));
    require(cap_cand <= 4096 && cap_core <= 4096, RBSOG_E_CAPACITY, "neighbour list capacity above 4096");
    c->drop_graph();
    plan_lists(c, cap_core, cap_cand);
}

// Build; if a list or cell capacity overflowed, grow the lists and build again.
void build_checked(rbsog_ctx* c)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        launch_clear_flags(c->s.sc, c->stream);
        enqueue_build(c, false);
        DeviceScalars h = read_scalars(c);
        if (h.overflow == 0) return;
        if (h.overflow & 2) throw Error(RBSOG_E_CAPACITY, "a cell holds more than 2048 atoms");
        if (h.overflow & 4) {
            // a cell's stencil did not fit in LDS: larger stencil, then per-atom lists
            c->s.list_mode = std::min(2, c->s.list_mode + 1);
            c->drop_graph();
            continue;
        }
        grow_lists(c);
    }
    throw Error(RBSOG_E_CAPACITY, "list capacity did not converge");
}

void enqueue_forces(rbsog_ctx* c, bool energy, bool kick)
{
    const bool ke = energy || (kick && c->s.thermo_c > 0.0);
    DevSys& s = c->s;
    KDev& k = c->k;
    hipStream_t st = c->stream;
    if (s.n <= 0) return;
    if (k.sampled) {
        c->begin(RBSOG_PHASE_KSAMPLE);
        launch_ksample(s, k, st);
        c->end();
    }
    c->begin(RBSOG_PHASE_PAIR);
    launch_pair(s, c->coef, c->mixed, energy, c->pair_part.as<double>(), c->n_pair_blocks, st);
    c->end();
    c->begin(RBSOG_PHASE_RHO);
    launch_rho(s, k, c->mixed, st);
    c->end();
    c->begin(RBSOG_PHASE_REDUCE);
    launch_rho_finalize(s, k, st);
    launch_finalize(s, k, c->pair_part.as<double>(), c->n_pair_blocks, st);
    c->end();
    c->begin(RBSOG_PHASE_KFORCE);
    launch_kforce(s, k, c->mixed, kick, ke, c->kin_part.as<double>(), st);
    c->end();
    if (ke) launch_kinetic_finalize(s, c->kin_part.as<double>(), c->n_kin_blocks, st);
}

void fill_energy(rbsog_ctx* c, const DeviceScalars& h, rbsog_energy* e)
{
    e->u_core = h.u_core;
    e->u_shell = h.u_shell;
    e->u_kspace = h.u_kspace;
    e->u_self = c->u_self;
    e->u_total = h.u_core + h.u_shell + h.u_kspace - c->u_self;
    e->kinetic = h.kinetic;
    for (int a = 0; a < 3; ++a) e->p_corr[a] = h.p_corr[a];
    e->max_disp = std::sqrt(h.max_disp2);
    e->n_builds = h.n_builds;
}

void check_flags(const DeviceScalars& h)
{
    if (h.overflow) throw Error(RBSOG_E_CAPACITY, "list capacity exceeded during the step loop");
}

// One step on the stream: kick + drift, rebuild if scheduled or if an atom
// moved more than skin/2 since the last build (decided on the device),
// forces, kick.
void enqueue_step(rbsog_ctx* c, bool scheduled, bool energy)
{
    c->begin(RBSOG_PHASE_INTEGRATE);
    launch_bump_eval(c->s.sc, c->stream);
    launch_kick_drift(c->s, scheduled, c->stream);
    c->end();
    enqueue_build(c, true);
    enqueue_forces(c, energy, true);
}

void set_system_impl(rbsog_ctx* c, const rbsog_params* p, const int32_t* type, const double* pos,
                     const double* vel, int on_device)
{
    validate(p);
    const int n = p->n_atoms;
    require(n == 0 || (type && pos), RBSOG_E_ARG, "type and pos are required");
    // host copies of the inputs for validation
    std::vector<int32_t> ht(n);
    std::vector<double> hp(3 * (size_t)n), hv;
    if (n > 0) {
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
    double qsum = 0.0, qabs = 0.0;
    for (int i = 0; i < n; ++i) {
        require(ht[i] >= 0 && ht[i] < p->n_species, RBSOG_E_ARG, "atom type out of range");
        qsum += p->species[ht[i]].q;
        qabs += std::fabs(p->species[ht[i]].q);
    }
    for (double v : hp) require(std::isfinite(v), RBSOG_E_NONFINITE, "non-finite position");
    for (double v : hv) require(std::isfinite(v), RBSOG_E_NONFINITE, "non-finite velocity");
    require(std::fabs(qsum) <= 1e-9 * std::max(1.0, qabs), RBSOG_E_NONNEUTRAL, "system is not charge neutral");

    // SOG split and coefficients
    c->drop_graph();
    c->prm = *p;
    if (!(c->prm.coulomb_k > 0.0)) c->prm.coulomb_k = 14.399645478425668;
    if (!(c->prm.sog_eps > 0.0)) c->prm.sog_eps = 1e-5;
    c->mixed = p->precision == RBSOG_MIXED;
    std::string err;
    if (!sog_split(c->prm.sog_eps, p->r_shell, &c->sog, &err)) throw Error(RBSOG_E_ARG, err);
    sog_base(c->prm.sog_eps, &c->chain);
    if (!sog_kernel_coef(c->sog, c->chain, p->r_shell, c->mixed, &c->coef, &err)) throw Error(RBSOG_E_ARG, err);
    double wsum = 0.0;
    for (double w : c->sog.w) wsum += w;
    double q2 = 0.0;
    for (int i = 0; i < n; ++i) q2 += p->species[ht[i]].q * p->species[ht[i]].q;
    c->u_self = 0.5 * c->prm.coulomb_k * q2 * wsum;

    DevSys& s = c->s;
    s = DevSys{};
    s.n = n;
    s.n_species = p->n_species;
    const double cutoff = p->r_shell + p->skin;
    s.ncell = 1;
    for (int a = 0; a < 3; ++a) {
        s.L[a] = p->box[a];
        s.invL[a] = 1.0 / p->box[a];
        int nc = (int)std::floor(p->box[a] / (cutoff + 1e-9));
        if (nc < 3) nc = 1;
        s.nc[a] = nc;
        s.cell_scale[a] = (double)nc / p->box[a];
        s.two_pi_L[a] = 2.0 * kPi / p->box[a];
        s.ncell *= nc;
    }
    const double rcl = p->r_core + p->skin;
    s.rc2_list = rcl * rcl;
    const double lo = p->r_core - p->skin;
    s.lo2_list = lo > 0.0 ? lo * lo : 0.0;
    const double hi = p->r_shell + p->skin;
    s.hi2_list = hi * hi;
    s.rc2 = p->r_core * p->r_core;
    s.rs2 = p->r_shell * p->r_shell;
    s.half_skin2 = 0.25 * p->skin * p->skin;
    s.dt = p->dt;
    s.coulomb_k = c->prm.coulomb_k;
    const bool thermo = p->t_target > 0.0 && p->tau_t > 0.0;
    s.thermo_c = thermo ? p->dt / p->tau_t : 0.0;
    s.t_target = thermo ? p->t_target : 0.0;
    s.dof_kb = (3.0 * n - 3.0) * 8.617333262e-5;
    s.p_r = p->p_r;
    s.replica = p->replica;
    s.seed = p->seed;
    for (int t = 0; t < RBSOG_MAX_SPECIES; ++t) {
        s.q[t] = t < p->n_species ? p->species[t].q : 0.0;
        s.mass[t] = t < p->n_species ? p->species[t].mass : 1.0;
        s.inv_mass_acc[t] = kAccUnit / s.mass[t];
    }

    // per-atom arrays: a packed position record, 12 doubles, 3 int32
    const size_t N = (size_t)std::max(n, 1);
    c->atoms.alloc(N * (sizeof(double4) + 12 * sizeof(double) + 3 * sizeof(int32_t)));
    {
        s.p = c->atoms.as<double4>();
        double* d = reinterpret_cast<double*>(s.p + N);
        double** slots[] = {&s.vx, &s.vy, &s.vz, &s.fx, &s.fy, &s.fz, &s.fsx, &s.fsy, &s.fsz, &s.xr, &s.yr, &s.zr};
        for (int t = 0; t < 12; ++t) *slots[t] = d + t * N;
        int32_t* ip = reinterpret_cast<int32_t*>(d + 12 * N);
        s.type = ip;
        s.id = ip + N;
        s.inv = ip + 2 * N;
    }
    c->sortbuf.alloc(N * (sizeof(double4) + 6 * sizeof(double) + 5 * sizeof(int32_t)));
    {
        s.tp = c->sortbuf.as<double4>();
        double* d = reinterpret_cast<double*>(s.tp + N);
        double** slots[] = {&s.tvx, &s.tvy, &s.tvz, &s.tfx, &s.tfy, &s.tfz};
        for (int t = 0; t < 6; ++t) *slots[t] = d + t * N;
        int32_t* ip = reinterpret_cast<int32_t*>(d + 6 * N);
        s.ttype = ip;
        s.tid = ip + N;
        s.cell_of = ip + 2 * N;
        s.slot_of = ip + 3 * N;
        s.order = ip + 4 * N;
    }
    c->cells.alloc(sizeof(int32_t) * (2 * (size_t)s.ncell + 1));
    s.cell_count = c->cells.as<int32_t>();
    s.cell_start = s.cell_count + s.ncell;
    HIP_OK(hipMemsetAsync(s.cell_count, 0, sizeof(int32_t) * s.ncell, c->stream));
    c->counts.alloc(2 * sizeof(int32_t) * N);
    s.core_cnt = c->counts.as<int32_t>();
    s.cand_cnt = s.core_cnt + N;
    HIP_OK(hipMemsetAsync(s.core_cnt, 0, 2 * sizeof(int32_t) * N, c->stream));

    // pair coefficient table
    std::vector<PairCoef> pcs(p->n_species * p->n_species);
    for (int i = 0; i < p->n_species; ++i)
        for (int j = 0; j < p->n_species; ++j) {
            const rbsog_pair& a = p->pair[i * RBSOG_MAX_SPECIES + j];
            PairCoef& pc = pcs[i * p->n_species + j];
            pc.qq = c->prm.coulomb_k * p->species[i].q * p->species[j].q;
            pc.A = a.A;
            pc.sig = a.sigma;
            pc.irho = a.rho > 0.0 ? 1.0 / a.rho : 0.0;
            pc.C = a.C;
            pc.D = a.D;
        }
    c->pair_tab.alloc(sizeof(PairCoef) * pcs.size());
    HIP_OK(hipMemcpy(c->pair_tab.p, pcs.data(), sizeof(PairCoef) * pcs.size(), hipMemcpyHostToDevice));
    s.pair = c->pair_tab.as<PairCoef>();
    c->scalars.alloc(sizeof(DeviceScalars));
    s.sc = c->scalars.as<DeviceScalars>();
    HIP_OK(hipMemsetAsync(s.sc, 0, sizeof(DeviceScalars), c->stream));

    // list capacities from the density
    const double V = p->box[0] * p->box[1] * p->box[2];
    const double rho_n = n / V;
    const double vc = 4.0 / 3.0 * kPi * rcl * rcl * rcl;
    const double lo3 = lo > 0.0 ? lo * lo * lo : 0.0;
    const double vk = 4.0 / 3.0 * kPi * (hi * hi * hi - lo3);
    // room for local densities well above the mean (melting lattices, clusters);
    // the step loop grows the lists if they still overflow
    const int cap_core = std::min(std::max(round_up((int)(1.8 * vc * rho_n) + 32, 32), 32), std::max(32, round_up(n, 32)));
    const int cap_cand = std::min(std::max(round_up((int)(1.5 * vk * rho_n) + 32, 32), 32), std::max(32, round_up(n, 32)));
    plan_lists(c, cap_core, cap_cand);
    {
        double cell_vol = 1.0;
        for (int a = 0; a < 3; ++a) cell_vol *= p->box[a] / s.nc[a];
        const int ncell_st = (s.nc[0] >= 3 ? 3 : 1) * (s.nc[1] >= 3 ? 3 : 1) * (s.nc[2] >= 3 ? 3 : 1);
        const double stencil = std::min<double>(n, ncell_st * cell_vol * rho_n);
        s.list_mode = stencil * 1.3 + 64 <= 2048 ? 0 : (stencil * 1.3 + 64 <= 4096 ? 1 : 2);
    }

    // k-space
    KDev& k = c->k;
    k = KDev{};
    std::vector<double> table(2 * kTableSize);
    for (int j = 0; j < kTableSize; ++j) {
        table[2 * j] = std::cos(2.0 * kPi * j / kTableSize);
        table[2 * j + 1] = std::sin(2.0 * kPi * j / kTableSize);
    }
    c->ktab.alloc(sizeof(double) * table.size());
    HIP_OK(hipMemcpy(c->ktab.p, table.data(), sizeof(double) * table.size(), hipMemcpyHostToDevice));
    k.table = c->ktab.as<double>();
    std::vector<int32_t> em;
    std::vector<double> ecoef;
    if (p->p_f > 0) {
        build_ktables(c->sog, p->box, &c->kt);
        k.sampled = 1;
        k.n_modes = p->p_f;
        k.nm = c->kt.nm;
        k.S = c->kt.S;
        k.coef_scale = c->kt.S / ((double)p->p_f * V);
        const size_t nt = c->kt.g0cdf.size();
        const size_t bytes = sizeof(double) * (2 * nt + c->kt.comp_cdf.size()) + sizeof(int32_t) * 2 * c->kt.off.size();
        c->kcdf.alloc(bytes);
        double* d = c->kcdf.as<double>();
        HIP_OK(hipMemcpy(d, c->kt.g0cdf.data(), sizeof(double) * nt, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d + nt, c->kt.g2cdf.data(), sizeof(double) * nt, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d + 2 * nt, c->kt.comp_cdf.data(), sizeof(double) * c->kt.comp_cdf.size(),
                         hipMemcpyHostToDevice));
        int32_t* ip = reinterpret_cast<int32_t*>(d + 2 * nt + c->kt.comp_cdf.size());
        HIP_OK(hipMemcpy(ip, c->kt.off.data(), sizeof(int32_t) * c->kt.off.size(), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(ip + c->kt.off.size(), c->kt.len.data(), sizeof(int32_t) * c->kt.len.size(),
                         hipMemcpyHostToDevice));
        k.g0cdf = d;
        k.g2cdf = d + nt;
        k.comp_cdf = d + 2 * nt;
        k.off = ip;
        k.len = ip + c->kt.off.size();
    } else {
        enumerate_modes(c->sog, p->box, &em, &ecoef);
        k.sampled = 0;
        k.n_modes = (int)ecoef.size();
        k.S = 0.0;
        c->kt = KTables{};
    }
    const int tiles = (k.n_modes + 63) / 64;
    k.n_modes_pad = std::max(1, tiles) * 64;
    const int max_chunks = std::max(1, (n + 255) / 256);
    k.n_chunks = std::min(max_chunks, std::max(1, (2048 + std::max(tiles, 1) - 1) / std::max(tiles, 1)));
    // a multiple of 16 atoms: the rho kernel splits a chunk into four
    // quarters read four atoms at a time
    k.chunk = (std::max(1, (n + k.n_chunks - 1) / k.n_chunks) + 15) & ~15;
    k.n_chunks = std::max(1, (n + k.chunk - 1) / k.chunk);
    c->kmodes.alloc(std::max<size_t>(1, (size_t)k.n_modes) * (sizeof(ModeRec) + 3 * sizeof(int32_t)));
    k.modes = c->kmodes.as<ModeRec>();
    k.m = reinterpret_cast<int32_t*>(k.modes + std::max(1, k.n_modes));
    if (!k.sampled && k.n_modes > 0) {
        std::vector<ModeRec> recs(k.n_modes);
        for (int q = 0; q < k.n_modes; ++q) {
            recs[q] = ModeRec{(double)em[3 * q], (double)em[3 * q + 1], (double)em[3 * q + 2], 0.0, 0.0, ecoef[q], 0.0, 0.0f, 0.0f};
        }
        HIP_OK(hipMemcpy(k.modes, recs.data(), sizeof(ModeRec) * k.n_modes, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(k.m, em.data(), sizeof(int32_t) * em.size(), hipMemcpyHostToDevice));
    }
    c->krho_part.alloc(sizeof(double) * 2 * (size_t)k.n_chunks * k.n_modes_pad);
    k.rho_part = c->krho_part.as<double>();
    c->krho.alloc(sizeof(double) * 2 * std::max<size_t>(1, (size_t)k.n_modes));
    k.rho = c->krho.as<double>();

    c->n_pair_blocks = (n + kBlock - 1) / kBlock;
    c->n_kin_blocks = c->n_pair_blocks;
    c->pair_part.alloc(sizeof(double) * kPairPart * std::max(1, c->n_pair_blocks));
    c->kin_part.alloc(sizeof(double) * std::max(1, c->n_kin_blocks));

    // inputs
    if (n > 0) {
        const int32_t* dt_ = type;
        const double* dp = pos;
        const double* dv = vel;
        DBuf stage;
        if (!on_device) {
            stage.alloc(sizeof(int32_t) * n + sizeof(double) * 6 * (size_t)n);
            double* sp = stage.as<double>();
            HIP_OK(hipMemcpy(sp, hp.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice));
            dp = sp;
            if (vel) {
                HIP_OK(hipMemcpy(sp + 3 * (size_t)n, hv.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice));
                dv = sp + 3 * (size_t)n;
            }
            int32_t* tp = reinterpret_cast<int32_t*>(sp + 6 * (size_t)n);
            HIP_OK(hipMemcpy(tp, ht.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
            dt_ = tp;
        }
        launch_from_user(s, dt_, dp, dv, c->stream);
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    c->have_system = true;
    c->eval = 0;
    c->forces_valid = false;
    build_checked(c);
    HIP_OK(hipStreamSynchronize(c->stream));
}

void need_system(rbsog_ctx* c) { require(c->have_system, RBSOG_E_STATE, "no system set"); }

}  // namespace

extern "C" {

const char* rbsog_version(void) { return "librbsog 0.1 (gfx950)"; }

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
        set_system_impl(ctx, p, type, pos, vel, ptrs_on_device);
    });
}

rbsog_status rbsog_build_lists(rbsog_ctx* ctx)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        build_checked(ctx);
    });
}

rbsog_status rbsog_compute_forces(rbsog_ctx* ctx, uint64_t eval, double* force_out, rbsog_energy* e_out)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        launch_set_eval(ctx->s.sc, eval, ctx->stream);
        enqueue_forces(ctx, e_out != nullptr, false);
        ctx->eval = eval;
        ctx->forces_valid = true;
        if (force_out) launch_to_user3(ctx->s, ctx->s.fx, ctx->s.fy, ctx->s.fz, force_out, ctx->stream);
        if (e_out) {
            DeviceScalars h = read_scalars(ctx);
            fill_energy(ctx, h, e_out);
            check_flags(h);
        }
    });
}

rbsog_status rbsog_get_force_parts(rbsog_ctx* ctx, double* f_short, double* f_kspace)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(ctx->forces_valid, RBSOG_E_STATE, "no force evaluation yet");
        if (f_short) launch_to_user3(ctx->s, ctx->s.fsx, ctx->s.fsy, ctx->s.fsz, f_short, ctx->stream);
        if (f_kspace) launch_kspace_part(ctx->s, f_kspace, ctx->stream);
    });
}

rbsog_status rbsog_step(rbsog_ctx* ctx, int32_t n_steps, rbsog_energy* e_last)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        require(n_steps >= 0, RBSOG_E_ARG, "n_steps < 0");
        if (n_steps == 0) return;
        if (!ctx->forces_valid) {
            // forces at the current positions start the integrator
            launch_set_eval(ctx->s.sc, ctx->eval, ctx->stream);
            enqueue_forces(ctx, false, false);
            ctx->forces_valid = true;
        }
        launch_set_eval(ctx->s.sc, ctx->eval, ctx->stream);
        if (ctx->s.thermo_c > 0.0) {
            // velocity factor of the first step from the current velocities
            launch_kinetic(ctx->s, ctx->kin_part.as<double>(), ctx->stream);
            launch_kinetic_finalize(ctx->s, ctx->kin_part.as<double>(), ctx->n_kin_blocks, ctx->stream);
        }
        const int every = ctx->prm.rebuild_every;
        // a list overflow inside the loop restarts the call from a snapshot
        // with larger lists
        for (int attempt = 0;; ++attempt) {
            snapshot(ctx, true);
            for (int k = 0; k < n_steps; ++k) {
                const uint64_t step = ctx->eval + 1 + (uint64_t)k;
                const bool scheduled = step % (uint64_t)every == 0;
                const bool energy = e_last != nullptr && k == n_steps - 1;
                enqueue_step(ctx, scheduled, energy);
            }
            DeviceScalars h = read_scalars(ctx);
            if (h.overflow == 0) {
                ctx->eval += (uint64_t)n_steps;
                if (e_last) fill_energy(ctx, h, e_last);
                check_flags(h);
                return;
            }
            require(attempt < 4 && (h.overflow & 2) == 0, RBSOG_E_CAPACITY, "list capacity exceeded in the step loop");
            if (h.overflow & 4)
                ctx->s.list_mode = std::min(2, ctx->s.list_mode + 1);
            else
                grow_lists(ctx);
            snapshot(ctx, false);
            build_checked(ctx);
            launch_set_eval(ctx->s.sc, ctx->eval, ctx->stream);
        }
    });
}

rbsog_status rbsog_get_state(rbsog_ctx* ctx, double* pos, double* vel, double* force, uint64_t* eval,
                             int ptrs_on_device)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        DevSys& s = ctx->s;
        const size_t bytes = sizeof(double) * 3 * (size_t)s.n;
        double* outs[3] = {pos, vel, force};
        const double* src[3][3] = {{nullptr, nullptr, nullptr}, {s.vx, s.vy, s.vz}, {s.fx, s.fy, s.fz}};
        if (!ptrs_on_device && s.n > 0 && (pos || vel || force)) ctx->export_tmp.alloc(bytes);
        for (int q = 0; q < 3; ++q) {
            if (!outs[q] || s.n <= 0) continue;
            double* dst = ptrs_on_device ? outs[q] : ctx->export_tmp.as<double>();
            if (q == 0)
                launch_pos_to_user(s, dst, ctx->stream);
            else
                launch_to_user3(s, src[q][0], src[q][1], src[q][2], dst, ctx->stream);
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
    return guarded(ctx, [&] { ctx->profiling = enable != 0; });
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
        const int n = ctx->s.n;
        std::vector<int32_t> nc(n), nk(n), id(n);
        HIP_OK(hipStreamSynchronize(ctx->stream));
        if (n > 0) {
            HIP_OK(hipMemcpy(nc.data(), ctx->s.core_cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(nk.data(), ctx->s.cand_cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(id.data(), ctx->s.id, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
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
        DevSys& s = ctx->s;
        require(i >= 0 && i < s.n, RBSOG_E_ARG, "atom index out of range");
        HIP_OK(hipStreamSynchronize(ctx->stream));
        std::vector<int32_t> id(s.n);
        HIP_OK(hipMemcpy(id.data(), s.id, sizeof(int32_t) * s.n, hipMemcpyDeviceToHost));
        int32_t t = 0, nc = 0, nk = 0;
        HIP_OK(hipMemcpy(&t, s.inv + i, sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(&nc, s.core_cnt + t, sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(&nk, s.cand_cnt + t, sizeof(int32_t), hipMemcpyDeviceToHost));
        nc = std::min(nc, s.cap_core);
        nk = std::min(nk, s.cap_cand);
        if (core) {
            std::vector<int32_t> tile((size_t)s.cap_core * 64);
            const int32_t* src = s.core_idx + (size_t)(t >> 6) * s.cap_core * 64;
            HIP_OK(hipMemcpy(tile.data(), src, sizeof(int32_t) * tile.size(), hipMemcpyDeviceToHost));
            std::vector<int32_t> ids(nc);
            for (int q = 0; q < nc; ++q) ids[q] = id[tile[(size_t)q * 64 + (t & 63)]];
            std::sort(ids.begin(), ids.end());
            std::copy(ids.begin(), ids.end(), core);
        }
        if (cand) {
            std::vector<int32_t> row(std::max(nk, 1));
            if (nk > 0)
                HIP_OK(hipMemcpy(row.data(), s.cand_idx + (size_t)t * s.cap_cand, sizeof(int32_t) * nk,
                                 hipMemcpyDeviceToHost));
            for (int q = 0; q < nk; ++q) cand[q] = id[row[q]];
        }
    });
}

rbsog_status rbsog_get_shell_ranks(rbsog_ctx* ctx, uint64_t eval, int32_t* n_ranks, int32_t* ranks)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        DevSys& s = ctx->s;
        const int P = std::max(s.p_r, 1);
        DBuf out;
        out.alloc(sizeof(int32_t) * ((size_t)s.n * P + s.n + 1));
        int32_t* r = out.as<int32_t>();
        int32_t* cnt = r + (size_t)s.n * P;
        launch_set_eval(s.sc, eval, ctx->stream);
        launch_shell_ranks(s, r, cnt, ctx->stream);
        launch_set_eval(s.sc, ctx->eval, ctx->stream);
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

rbsog_status rbsog_get_kmodes(rbsog_ctx* ctx, uint64_t eval, int32_t* m, double* S)
{
    return guarded(ctx, [&] {
        need_system(ctx);
        KDev& k = ctx->k;
        if (S) *S = k.S;
        if (!m || k.n_modes <= 0) return;
        if (k.sampled) {
            launch_set_eval(ctx->s.sc, eval, ctx->stream);
            launch_ksample(ctx->s, k, ctx->stream);
            launch_set_eval(ctx->s.sc, ctx->eval, ctx->stream);
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
        HIP_OK(hipStreamSynchronize(ctx->stream));
        if (ctx->k.n_modes > 0)
            HIP_OK(hipMemcpy(rho, ctx->k.rho, sizeof(double) * 2 * (size_t)ctx->k.n_modes, hipMemcpyDeviceToHost));
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
