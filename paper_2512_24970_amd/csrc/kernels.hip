// HIP kernels of the IRBSOG evaluation for gfx950 (CDNA4, wave64).
//
// Layout: atoms in (cell, id) order as structure-of-arrays FP64; the core
// list is stored in 64-atom tiles (entry k of the 64 atoms of a tile
// contiguous) so a wavefront reads it coalesced; shell candidates are stored
// row-major per atom in (cell, id) order, the canonical order that the ranks
// of the shell batch of eq. (25) refer to.  Every reduction runs in a fixed order, so FP64
// results are bit-reproducible run to run.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <mutex>
#include <type_traits>

#include "kernels.hpp"

namespace rbsog {

// Device memory of the allocation-free pair histogram (rbsog_rdf_counts_noalloc):
// one array per GPU the library runs on, held until the process ends.  Host
// code must not use this name as an address (it is a host-side stand-in);
// it uses the device address that noalloc_init looks up.
static __device__ __align__(256) unsigned long long scratch[kRdfScratch];

namespace {

constexpr int kBlock = 256;
constexpr int kCellCap = 2048;  // atoms per cell the in-cell sort can hold

// Build kernels take `gate`: when set they run only if the rebuild flag is up
// (set by the drift kernel), so a step can enqueue them unconditionally.  A
// system that produced a non-finite value is not rebuilt (its positions may
// be NaN; the host reports the error at the end of the call).
#define RB_GATE                                        \
    if (gate && (s.sc->rebuild == 0 || s.sc->nonfinite)) return;

// Pointers read from device memory are generic (flat) to the compiler; every
// buffer here is global memory, and saying so (through an integer, which the
// compiler does not fold back) turns flat loads and stores into global ones.
template <class T>
__device__ inline T* glob(T* p)
{
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

__device__ inline DevSys global_view(DevSys s)
{
    s.p = glob(s.p);
    s.vx = glob(s.vx), s.vy = glob(s.vy), s.vz = glob(s.vz);
    s.fx = glob(s.fx), s.fy = glob(s.fy), s.fz = glob(s.fz);
    s.fsx = glob(s.fsx), s.fsy = glob(s.fsy), s.fsz = glob(s.fsz);
    s.xr = glob(s.xr), s.yr = glob(s.yr), s.zr = glob(s.zr);
    s.type = glob(s.type), s.id = glob(s.id), s.inv = glob(s.inv);
    s.tp = glob(s.tp);
    s.tvx = glob(s.tvx), s.tvy = glob(s.tvy), s.tvz = glob(s.tvz);
    s.tfx = glob(s.tfx), s.tfy = glob(s.tfy), s.tfz = glob(s.tfz);
    s.ttype = glob(s.ttype), s.tid = glob(s.tid), s.cell_of = glob(s.cell_of);
    s.slot_of = glob(s.slot_of), s.order = glob(s.order);
    s.cell_count = glob(s.cell_count), s.cell_start = glob(s.cell_start);
    s.core_cnt = glob(s.core_cnt), s.core_idx = glob(s.core_idx);
    s.cand_cnt = glob(s.cand_cnt), s.cand_idx = glob(s.cand_idx), s.bat_idx = glob(s.bat_idx);
    s.pair = glob(s.pair), s.sc = glob(s.sc), s.spc = glob(s.spc);
    s.pair_part = glob(s.pair_part), s.kin_part = glob(s.kin_part), s.vir_part = glob(s.vir_part);
    s.fin_part = glob(s.fin_part);
    s.ufix = glob(s.ufix);
    return s;
}

__device__ inline KDev global_view(KDev k)
{
    k.table = glob(k.table);
    k.off = glob(k.off), k.len = glob(k.len);
    k.g0cdf = glob(k.g0cdf), k.g2cdf = glob(k.g2cdf), k.comp_cdf = glob(k.comp_cdf);
    k.m = glob(k.m), k.modes = glob(k.modes);
    k.rho_part = glob(k.rho_part), k.rho = glob(k.rho);
    k.sog_c = glob(k.sog_c), k.sog_s2 = glob(k.sog_s2);
    return k;
}

// A launch covers every system of a batch: block b of the grid works on local
// block bmap[b].y of system bmap[b].x (no map: system 0, local block b).  The
// system record is read through the scalar unit at the start of the block.
#define RB_ARGS const DevSys* __restrict__ sys, const int2* __restrict__ bmap
#define RB_SYS(gb)                                                        \
    const int2 rb_m = bmap ? bmap[(gb)] : make_int2(0, (int)(gb));        \
    const DevSys s = global_view(sys[rb_m.x]);                            \
    const int lb = rb_m.y;


__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Per-wavefront partial sums: atom i's wavefront (atoms 64w .. 64w+63 of its
// system, whatever the block size) writes entry w.  Later reductions run
// over the entries in order, so results do not depend on the block size.
__device__ inline void wave_partial(double v, int i, int n, double* part, int stride, int c)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && (i & ~63) < n) part[(size_t)(i >> 6) * stride + c] = v;
}

// Sum of v over a block of up to 1024 threads in a fixed order; valid in
// thread 0.
__device__ inline double block_sum(double v, double* red /*[blockDim.x / 64]*/)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
    __syncthreads();
    return t;
}

// Minimum image with the operations in a fixed order (no contraction):
// d -= L * rint(d / L), d / L evaluated as d * (1/L).
__device__ inline double min_image(double d, double L, double invL)
{
    const double k = rint(d * invL);
    const double Lk = L * k;
    return d - Lk;
}

__device__ inline double wrap_coord(double x, double L, double invL)
{
    const double f = floor(x * invL);
    double v = x - L * f;
    if (v >= L) v -= L;
    if (v < 0.0) v += L;
    return v;
}

__device__ inline int cell_coord(double v, double scale, int nc)
{
    int c = (int)(v * scale);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Cell of a wrapped position on the ordering grid (x fastest); candidates
// are listed in ascending (this cell, index).
__device__ inline int fine_cell(const DevSys& s, const double4& P)
{
    const int fx = cell_coord(P.x, s.fine_scale[0], s.nf[0]);
    const int fy = cell_coord(P.y, s.fine_scale[1], s.nf[1]);
    const int fz = cell_coord(P.z, s.fine_scale[2], s.nf[2]);
    return (fz * s.nf[1] + fy) * s.nf[0] + fx;
}

// Fixed-point record of a wrapped position: floor(x/L 2^32) per axis (a
// fraction of the box, 2^32 wrapping to 0: the same point) and the type.
// The 32-bit difference of two records, read as signed, is the minimum
// image of their displacement in units of L 2^-32.
__device__ inline uint32_t frac32(double f)
{
    // f in [0, 1]: floor(f 2^32), with 2^32 wrapping to 0 (the same turn)
    return (uint32_t)(uint64_t)(f * 4294967296.0);
}

__device__ inline uint4 fix_record(const DevSys& s, double x, double y, double z, double type)
{
    return make_uint4(frac32(x * s.invL[0]), frac32(y * s.invL[1]), frac32(z * s.invL[2]), (uint32_t)type);
}

// One flag write per wavefront holding a non-finite value (every lane of the
// wavefront calls it).
__device__ inline void flag_nonfinite(bool bad, DeviceScalars* sc)
{
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&sc->nonfinite, 1);
}

__device__ inline bool finite3(double x, double y, double z) { return isfinite(x) && isfinite(y) && isfinite(z); }

// Workgroups are dealt to the 8 XCDs in turn (block b on XCD b mod 8), each
// XCD with its own L2.  Renumbering so that XCD x gets a contiguous range of
// logical blocks keeps spatially neighbouring atoms (cell order) on one L2.
__device__ inline int xcd_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, k = b >> 3;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// ---------------------------------------------------------------- scalars
__global__ void k_set_eval(DeviceScalars* sc, int R, uint64_t eval)
{
    for (int r = threadIdx.x; r < R; r += blockDim.x) sc[r].eval = eval;
}
// Nose-Hoover half step on the thermostat variables (Trotter splitting,
// one variable): from the kinetic energy K of the velocities it acts on,
// returns the velocity factor and leaves K scaled by its square.
__device__ inline double nh_half(const DevSys& s, DeviceScalars* sc, double& K)
{
    const double gkt = s.dof_kb * s.t_target;
    double v = sc->nh_v + 0.25 * s.dt * (2.0 * K - gkt) / s.nh_q;
    const double f = exp(-0.5 * s.dt * v);
    K = K * (f * f);
    sc->nh_x += 0.5 * s.dt * v;
    sc->nh_v = v + 0.25 * s.dt * (2.0 * K - gkt) / s.nh_q;
    return f;
}

__device__ inline bool is_nh(const DevSys& s) { return s.thermo_c > 0.0 && s.thermostat == kThermoNoseHoover; }

// Start of a step: the Philox counter moves on; Nose-Hoover takes its
// opening half step from the kinetic energy at the end of the last one and
// hands the opening kick the product of both pending velocity factors.
__global__ void k_step_begin(const DevSys* __restrict__ sys, int R)
{
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        const DevSys s = global_view(sys[r]);
        DeviceScalars* sc = s.sc;
        sc->eval += 1;
        if (is_nh(s)) {
            double K = sc->kinetic;
            const double f = nh_half(s, sc, K);
            sc->kinetic = K;
            sc->vscale = sc->vpend * f;
            sc->vpend = 1.0;
        }
    }
}

__global__ void k_init_scalars(DeviceScalars* sc, int R)
{
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        sc[r].vscale = 1.0;
        sc[r].vpend = 1.0;
    }
}
// Closes a build: lower the flag, restart the displacement tracking.  A
// build that overflowed is discarded and built again, so it takes no number.
__global__ void k_build_done(const DevSys* __restrict__ sys, int R, int gate)
{
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        DeviceScalars* sc = glob(sys[r].sc);
        if (gate && (sc->rebuild == 0 || sc->nonfinite)) continue;
        sc->rebuild = 0;
        sc->max_disp2 = 0.0;
        if (sc->overflow == 0) sc->n_builds += 1;
    }
}
__global__ void k_clear_flags(DeviceScalars* sc, int R)
{
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        sc[r].overflow = 0;
        sc[r].rebuild = 0;
        sc[r].nonfinite = 0;
        sc[r].max_disp2 = 0.0;
    }
}

// ---------------------------------------------------------------- cell sort
__global__ void k_bin(RB_ARGS, int gate)
{
    RB_SYS(blockIdx.x)
    RB_GATE
    const int i0 = lb * blockDim.x + threadIdx.x;
    // lanes past the end take part in the wavefront votes with a done flag
    const bool live = i0 < s.n;
    const int i = live ? i0 : s.n - 1;
    const double4 P = s.p[i];
    const double x = wrap_coord(P.x, s.L[0], s.invL[0]);
    const double y = wrap_coord(P.y, s.L[1], s.invL[1]);
    const double z = wrap_coord(P.z, s.L[2], s.invL[2]);
    // list cell = ordering-grid cell >> 1 per axis (n_f = 2 n_c, or 1 with
    // n_c = 1), so every ordering cell lies in exactly one list cell
    const int cx = cell_coord(x, s.fine_scale[0], s.nf[0]) >> 1;
    const int cy = cell_coord(y, s.fine_scale[1], s.nf[1]) >> 1;
    const int cz = cell_coord(z, s.fine_scale[2], s.nf[2]) >> 1;
    const int c = (cz * s.nc[1] + cy) * s.nc[0] + cx;
    if (live) {
        s.p[i] = make_double4(x, y, z, P.w);
        s.cell_of[i] = c;
    }
    // atoms of a wavefront mostly share a cell (cell order from the last
    // build): one atomic per distinct cell, slots handed out by ballot rank
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool done = !live;
    while (__ballot(!done)) {
        const uint64_t pending = __ballot(!done);
        const int leader = __builtin_ctzll(pending);
        const int cl = __shfl(c, leader, 64);
        const uint64_t same = __ballot(!done && c == cl);
        int base = 0;
        if (lane == leader) base = atomicAdd(&s.cell_count[cl], __popcll(same));
        base = __shfl(base, leader, 64);
        if (!done && c == cl) {
            s.slot_of[i] = base + __popcll(same & below);
            done = true;
        }
    }
}

// Exclusive scan of count[0..n) into start[0..n], one block of 1024 threads
// per system, over tiles of kScanTile counts staged in LDS (coalesced loads
// and stores); counts are zeroed for the next build.
constexpr int kScanTile = 8192;
__global__ __launch_bounds__(1024) void k_scan(const DevSys* __restrict__ sys, int gate)
{
    const DevSys s = global_view(sys[blockIdx.x]);
    RB_GATE
    int32_t* count = s.cell_count;
    int32_t* start = s.cell_start;
    const int n = s.ncell;
    __shared__ int32_t tile[kScanTile];
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    constexpr int per = kScanTile / 1024;
    int32_t carry = 0;
    for (int base = 0; base < n; base += kScanTile) {
        const int m = min(kScanTile, n - base);
#pragma unroll
        for (int k = 0; k < per; ++k) {
            const int i = t + 1024 * k;
            if (i < m) tile[i] = count[base + i];
        }
        __syncthreads();
        const int b = t * per;
        int32_t sum = 0;
#pragma unroll
        for (int k = 0; k < per; ++k)
            if (b + k < m) sum += tile[b + k];
        part[t] = sum;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int32_t v = t >= o ? part[t - o] : 0;
            __syncthreads();
            part[t] += v;
            __syncthreads();
        }
        int32_t run = carry + part[t] - sum;
#pragma unroll
        for (int k = 0; k < per; ++k)
            if (b + k < m) {
                const int32_t v = tile[b + k];
                tile[b + k] = run;
                run += v;
            }
        carry += part[1023];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < per; ++k) {
            const int i = t + 1024 * k;
            if (i < m) {
                start[base + i] = tile[i];
                count[base + i] = 0;  // ready for the next build
            }
        }
        __syncthreads();
    }
    if (t == 0) start[n] = carry;
}

__global__ void k_scatter(RB_ARGS, int gate)
{
    RB_SYS(blockIdx.x)
    RB_GATE
    const int i = lb * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const int d = s.cell_start[s.cell_of[i]] + s.slot_of[i];
    s.tp[d] = s.p[i];
    s.tvx[d] = s.vx[i];
    s.tvy[d] = s.vy[i];
    s.tvz[d] = s.vz[i];
    s.tfx[d] = s.fx[i];
    s.tfy[d] = s.fy[i];
    s.tfz[d] = s.fz[i];
    s.ttype[d] = s.type[i];
    s.tid[d] = s.id[i];
}

// Within each list cell, order atoms by (ordering sub-cell, id): the order is
// deterministic and each of the eight sub-cells is a contiguous range, whose
// first positions go to sub_beg.  Keys: sub-cell << 28 | id (ids < 2^28).
// A cell of up to 64 atoms (nearly every cell of a large box) is sorted by
// the block's first wavefront in registers, a bitonic network across its
// lanes; a larger one (a small box is one cell) by the whole block over LDS.
__global__ __launch_bounds__(kBlock) void k_cell_sort(RB_ARGS, int gate)
{
    RB_SYS(blockIdx.x)
    RB_GATE
    __shared__ int32_t key[kCellCap];
    __shared__ int32_t val[kCellCap];
    const int c = lb;
    const int lane = threadIdx.x & 63;
    const int beg = s.cell_start[c];
    const int cnt = s.cell_start[c + 1] - beg;
    int32_t* sb = s.sub_beg + (size_t)c * 8;
    if (cnt > kCellCap) {
        // keep a valid (unsorted) permutation and in-range sub-cell bounds;
        // the host reports the overflow
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) s.order[beg + t] = beg + t;
        if (threadIdx.x < 8) sb[threadIdx.x] = threadIdx.x == 0 ? 0 : cnt;
        if (threadIdx.x == 0) atomicOr(&s.sc->overflow, 2);
        return;
    }
    auto key_of = [&](int t) {
        const double4 Q = s.tp[beg + t];
        const int fx = cell_coord(Q.x, s.fine_scale[0], s.nf[0]);
        const int fy = cell_coord(Q.y, s.fine_scale[1], s.nf[1]);
        const int fz = cell_coord(Q.z, s.fine_scale[2], s.nf[2]);
        const int sub = ((fz & 1) * 2 + (fy & 1)) * 2 + (fx & 1);
        return (sub << 28) | s.tid[beg + t];
    };
    if (cnt <= 64) {
        if (threadIdx.x >= 64) return;
        // lane pairs (l, l ^ j) compare-exchange: the lower lane of a pair
        // keeps the smaller key in ascending blocks (l & size == 0) and the
        // larger in descending ones; padding keys are INT_MAX
        int k = lane < cnt ? key_of(lane) : INT_MAX;
        int v = lane < cnt ? beg + lane : -1;
        for (int size = 2; size <= 64; size <<= 1) {
            for (int j = size >> 1; j > 0; j >>= 1) {
                const int ko = __shfl_xor(k, j, 64);
                const int vo = __shfl_xor(v, j, 64);
                const bool keep_min = ((lane & size) == 0) == ((lane & j) == 0);
                if (keep_min ? ko < k : ko > k) {
                    k = ko;
                    v = vo;
                }
            }
        }
        if (lane < cnt) s.order[beg + lane] = v;
        // first sorted position whose sub-cell is >= q: the keys below q << 28
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint64_t m = __builtin_amdgcn_ballot_w64(lane < cnt && k < (q << 28));
            if (lane == q) sb[q] = __popcll(m);
        }
        return;
    }
    int P = 1;
    while (P < cnt) P <<= 1;
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        key[t] = t < cnt ? key_of(t) : INT_MAX;
        val[t] = t < cnt ? beg + t : -1;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < P; t += blockDim.x) {
                const int u = t ^ j;
                if (u > t) {
                    const bool up = (t & k) == 0;
                    const int32_t a = key[t], b = key[u];
                    if ((a > b) == up) {
                        key[t] = b;
                        key[u] = a;
                        const int32_t va = val[t];
                        val[t] = val[u];
                        val[u] = va;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) s.order[beg + t] = val[t];
    if (threadIdx.x < 8) {
        // first sorted position whose sub-cell is >= this one
        const int32_t want = (int32_t)threadIdx.x << 28;
        int lo = 0, hi = cnt;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (key[mid] < want)
                lo = mid + 1;
            else
                hi = mid;
        }
        sb[threadIdx.x] = lo;
    }
}

__global__ void k_gather(RB_ARGS, int gate)
{
    RB_SYS(blockIdx.x)
    RB_GATE
    const int t = lb * blockDim.x + threadIdx.x;
    if (t >= s.n) return;
    const int o = s.order[t];
    const double4 P = s.tp[o];
    s.p[t] = P;
    s.ufix[t] = fix_record(s, P.x, P.y, P.z, P.w);
    s.xr[t] = P.x;
    s.yr[t] = P.y;
    s.zr[t] = P.z;
    s.vx[t] = s.tvx[o];
    s.vy[t] = s.tvy[o];
    s.vz[t] = s.tvz[o];
    s.fx[t] = s.tfx[o];
    s.fy[t] = s.tfy[o];
    s.fz[t] = s.tfz[o];
    s.type[t] = s.ttype[o];
    const int id = s.tid[o];
    s.id[t] = id;
    s.inv[id] = t;
}

// ---------------------------------------------------------------- lists
// Fallback for stencils that do not fit in LDS.  One 64-thread block per
// atom: the lanes sweep the neighbouring cells, compact core and candidate
// entries with ballots, then sort the candidates into the canonical order,
// (cell of the ordering grid, index), with a bitonic network in LDS.
__global__ __launch_bounds__(64) void k_lists(RB_ARGS, int gate)
{
    RB_SYS(blockIdx.x)
    RB_GATE
    if (s.n_chunks != 1) {
        // candidate rows are per atom here: the host plans one chunk
        if (threadIdx.x == 0) atomicOr(&s.sc->overflow, 8);
        return;
    }
    extern __shared__ long long lsm64[];
    const int capP2 = [&] {
        int p = 1;
        while (p < s.cap_cand) p <<= 1;
        return p;
    }();
    long long* ckey = lsm64;
    int32_t* cval = reinterpret_cast<int32_t*>(lsm64 + capP2);
    int32_t* core = cval + capP2;

    const int i = lb;
    const int lane = threadIdx.x;
    const double4 Pi = s.p[i];
    const double xi = Pi.x, yi = Pi.y, zi = Pi.z;
    const int ci[3] = {cell_coord(xi, s.cell_scale[0], s.nc[0]), cell_coord(yi, s.cell_scale[1], s.nc[1]),
                       cell_coord(zi, s.cell_scale[2], s.nc[2])};
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int ncore = 0, ncand = 0;
    const int lo0 = s.nc[0] >= 3 ? -1 : 0, hi0 = s.nc[0] >= 3 ? 1 : 0;
    const int lo1 = s.nc[1] >= 3 ? -1 : 0, hi1 = s.nc[1] >= 3 ? 1 : 0;
    const int lo2 = s.nc[2] >= 3 ? -1 : 0, hi2 = s.nc[2] >= 3 ? 1 : 0;
    for (int oz = lo2; oz <= hi2; ++oz) {
        const int cz = (ci[2] + oz + s.nc[2]) % s.nc[2];
        for (int oy = lo1; oy <= hi1; ++oy) {
            const int cy = (ci[1] + oy + s.nc[1]) % s.nc[1];
            for (int ox = lo0; ox <= hi0; ++ox) {
                const int cx = (ci[0] + ox + s.nc[0]) % s.nc[0];
                const int c = (cz * s.nc[1] + cy) * s.nc[0] + cx;
                const int beg = s.cell_start[c], end = s.cell_start[c + 1];
                for (int base = beg; base < end; base += 64) {
                    const int j = base + lane;
                    bool is_core = false, is_cand = false;
                    long long order_key = 0;
                    if (j < end && j != i) {
                        const double4 Pj = s.p[j];
                        order_key = ((long long)fine_cell(s, Pj) << 32) | j;
                        const double dx = min_image(xi - Pj.x, s.L[0], s.invL[0]);
                        const double dy = min_image(yi - Pj.y, s.L[1], s.invL[1]);
                        const double dz = min_image(zi - Pj.z, s.L[2], s.invL[2]);
                        const double r2 = (dx * dx + dy * dy) + dz * dz;
                        double rcl = s.rc2_list, lol = s.lo2_list;
                        if (s.species_cut) {
                            const PairCoef& pcj = s.pair[(int)Pi.w * s.n_species + (int)Pj.w];
                            rcl = pcj.rc2_list;
                            lol = pcj.lo2_list;
                        }
                        is_core = r2 < rcl;
                        is_cand = r2 >= lol && r2 < s.hi2_list;
                    }
                    const uint64_t mc = __ballot(is_core);
                    const uint64_t mk = __ballot(is_cand);
                    if (is_core) {
                        const int slot = ncore + __popcll(mc & below);
                        if (slot < s.cap_core) core[slot] = j;
                    }
                    if (is_cand) {
                        const int slot = ncand + __popcll(mk & below);
                        if (slot < s.cap_cand) {
                            ckey[slot] = order_key;
                            cval[slot] = j;
                        }
                    }
                    ncore += __popcll(mc);
                    ncand += __popcll(mk);
                }
            }
        }
    }
    if (lane == 0) {
        s.core_cnt[i] = ncore;
        s.cand_cnt[i] = ncand;
        // usable capacity cap - 1, as in the per-cell kernel
        if (ncore >= s.cap_core || ncand >= s.cap_cand) {
            atomicOr(&s.sc->overflow, 1);
            atomicMax(&s.sc->max_core, ncore + 1);
            atomicMax(&s.sc->max_cand, ncand + 1);
        }
    }
    const int nk = min(ncand, s.cap_cand - 1);
    const int nc = min(ncore, s.cap_core - 1);
    int P = 1;
    while (P < nk) P <<= 1;
    for (int t = nk + lane; t < P; t += 64) {
        ckey[t] = LLONG_MAX;
        cval[t] = -1;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < P; t += 64) {
                const int u = t ^ j;
                if (u > t) {
                    const bool up = (t & k) == 0;
                    const long long a = ckey[t], b = ckey[u];
                    if ((a > b) == up) {
                        ckey[t] = b;
                        ckey[u] = a;
                        const int32_t va = cval[t];
                        cval[t] = cval[u];
                        cval[u] = va;
                    }
                }
            }
            __syncthreads();
        }
    }
    int32_t* crow = s.cand_idx + (size_t)i * s.cap_cand;
    for (int t = lane; t < nk; t += 64) crow[t] = cval[t];
    int32_t* ctile = s.core_idx + (size_t)(i >> 6) * s.cap_core * 64 + (i & 63);
    for (int t = lane; t < nc; t += 64) ctile[(size_t)t * 64] = core[t];
}

// One 512-thread block per list cell (side >= r_shell + skin).  The atoms of
// the (up to) 27 neighbouring list cells are staged in LDS and sorted there
// by cell of the ordering grid (half the side, 6 x 6 x 6 of them around the
// block's cell), stably, so the staged array is in canonical candidate order.
// A wavefront takes up to kListA atoms of one of the block's ordering cells
// (a unit) and makes two passes over the staged array.  The first keeps the
// staged atoms inside a sphere around the unit: centred on the unit's
// bounding box, of radius the largest list radius plus the distance to the
// unit's farthest atom, so by the triangle inequality every list neighbour
// of every atom of the unit is kept (a margin covers rounding).  The kept
// positions go, in staged order, into a small queue of the wavefront in LDS.
// Each time the queue holds 64 entries the second pass takes them, one per
// lane, tests them against every atom of the unit with the exact FP64
// distance of the lists, and compacts hits with ballots straight into the
// lists.  The filter only decides which candidates get the exact test, so
// the lists are the same bits as a sweep over every staged atom; about half
// the candidates of the unit's 5 x 5 x 5 window of ordering cells survive it.
constexpr int kListBlock = 512;
constexpr int kRegion = 216;  // ordering cells staged per block, at most 6 x 6 x 6
constexpr int kListA = 8;     // atoms per unit
constexpr int kQueue = 128;   // queue entries per wavefront (a power of two >= 128)

__device__ inline int wrap_index(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Rank of this lane among the set lanes of m below it (plus base).
__device__ inline int mbcnt64(uint64_t m, int base = 0)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)base));
}

// First atom of build chunk `chunk` (cells [chunk ncell / K, (chunk+1) ncell / K)).
__device__ inline int chunk_first_atom(const DevSys& s, int chunk)
{
    return s.cell_start[(int)(((long long)chunk * s.ncell) / s.n_chunks)];
}

// A wave-uniform double, kept in scalar registers.
__device__ inline double uniform_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// PC: species-dependent core radii; staged indices then carry the species in
// their top bits and the core/candidate bounds come per pair from LDS.
constexpr int kIdxBits = 28;
constexpr int kIdxMask = (1 << kIdxBits) - 1;

// Waves per SIMD that the LDS of a block staging CAP atoms leaves room for
// (3 blocks of 8 waves per CU up to about 53 KB each, else 2, else 1): the
// register budget is capped to match, so registers never cost a block.
constexpr int kListWaves(int cap) { return cap <= 1600 ? 6 : (cap <= 2048 ? 4 : 2); }

template <int CAP, bool PC>
__global__ __launch_bounds__(kListBlock) __attribute__((amdgpu_waves_per_eu(kListWaves(CAP)))) void k_lists_cell(RB_ARGS, int gate, int chunk)
{
    RB_SYS(xcd_block(blockIdx.x, gridDim.x))
    RB_GATE
    __shared__ double2 thr[PC ? kMaxSpecies * kMaxSpecies : 1];  // (rc2_list, lo2_list) per pair
    if (PC)
        for (int t = threadIdx.x; t < s.n_species * s.n_species; t += blockDim.x)
            thr[t] = make_double2(s.pair[t].rc2_list, s.pair[t].lo2_list);
    if (chunk >= s.n_chunks) return;
    // candidate rows of this chunk's atoms start at its first atom
    const int row0 = chunk_first_atom(s, chunk);
    if (chunk_first_atom(s, chunk + 1) - row0 > s.cand_rows) {
        if (threadIdx.x == 0) atomicOr(&s.sc->overflow, 8);
        return;
    }
    __shared__ int32_t val[CAP];
    __shared__ double px[CAP];
    __shared__ double py[CAP];
    __shared__ double pz[CAP];
    __shared__ int lcnt[kRegion];       // atoms per region cell
    __shared__ int gbeg[kRegion];       // first (sorted) atom of each region cell
    __shared__ int cstart[kRegion];     // first staged position of each region cell
    __shared__ int rcell[kRegion];      // region cell of each rank (ascending global index)
    __shared__ int rstart[kRegion];     // first staged position of each rank
    __shared__ int16_t queue[kListBlock / 64][kQueue];
    __shared__ int total_sm;
    __shared__ uint8_t srank[CAP];      // rank of each staged position, then its image code
    __shared__ uint8_t rcode[kRegion];  // image code of each rank (2 bits per axis)
    // block lb is part `part` of list cell c: the parts share the staging and
    // take every list_parts-th group of work units
    const int c = lb / s.list_parts;
    const int part = lb - c * s.list_parts;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cx0 = c % s.nc[0];
    const int cy0 = (c / s.nc[0]) % s.nc[1];
    const int cz0 = c / (s.nc[0] * s.nc[1]);
    // region of ordering cells: the 3 x 3 x 3 list cells around this one,
    // 6 ordering cells per split axis starting 2 below the block's first
    // (axes with fewer than 3 list cells are not split: 1 cell)
    const bool sx = s.nc[0] >= 3, sy = s.nc[1] >= 3, sz = s.nc[2] >= 3;
    const int R0 = sx ? 6 : 1, R1 = sy ? 6 : 1, R2 = sz ? 6 : 1;
    const int R = R0 * R1 * R2;
    const int gx0 = sx ? 2 * cx0 - 2 : 0, gy0 = sy ? 2 * cy0 - 2 : 0, gz0 = sz ? 2 * cz0 - 2 : 0;
    // each region cell is a contiguous range of the sorted atoms: its list
    // cell's range, cut at the sub-cell bounds the cell sort recorded
    for (int q = threadIdx.x; q < R; q += blockDim.x) {
        const int lx = q % R0, ly = (q / R0) % R1, lz = q / (R0 * R1);
        const int gx = sx ? wrap_index(gx0 + lx, s.nf[0]) : 0;
        const int gy = sy ? wrap_index(gy0 + ly, s.nf[1]) : 0;
        const int gz = sz ? wrap_index(gz0 + lz, s.nf[2]) : 0;
        const int lc = ((gz >> 1) * s.nc[1] + (gy >> 1)) * s.nc[0] + (gx >> 1);
        const int sub = ((gz & 1) * 2 + (gy & 1)) * 2 + (gx & 1);
        const int32_t* sbc = s.sub_beg + (size_t)lc * 8;
        const int cb0 = s.cell_start[lc];
        const int b0 = cb0 + sbc[sub];
        const int e0 = sub < 7 ? cb0 + sbc[sub + 1] : s.cell_start[lc + 1];
        gbeg[q] = b0;
        lcnt[q] = max(e0 - b0, 0);
    }
    // rank of each region cell in ascending global index: lexicographic in
    // (z, y, x) of the wrapped global coordinates, so per-axis ranks combine
    for (int q = threadIdx.x; q < R; q += blockDim.x) {
        const int lx = q % R0, ly = (q / R0) % R1, lz = q / (R0 * R1);
        auto axis_rank = [](int l, int g0, int n, int Ra) {
            const int g = wrap_index(g0 + l, n);
            int r = 0;
            for (int m = 0; m < Ra; ++m) r += wrap_index(g0 + m, n) < g;
            return r;
        };
        const int rank = (axis_rank(lz, gz0, s.nf[2], R2) * R1 + axis_rank(ly, gy0, s.nf[1], R1)) * R0 +
                         axis_rank(lx, gx0, s.nf[0], R0);
        rcell[rank] = q;
        // Periodic image of the cell as seen from the block: per split axis
        // k = -1 where the cell wraps from below the box (its atoms sit near
        // L, the block's near 0), +1 where it wraps from above, else 0, in
        // two bits (two's complement).
        auto image = [](int l, int g0, int n) {
            const int g = g0 + l;
            return (g < 0 ? 3 : (g >= n ? 1 : 0));
        };
        rcode[rank] = (uint8_t)((sx ? image(lx, gx0, s.nf[0]) : 0) | ((sy ? image(ly, gy0, s.nf[1]) : 0) << 2) |
                                ((sz ? image(lz, gz0, s.nf[2]) : 0) << 4));
    }
    __syncthreads();
    // first staged position of each region cell: exclusive scan over ranks
    if (wave == 0) {
        int carry = 0;
        for (int r0c = 0; r0c < R; r0c += 64) {
            const int r = r0c + lane;
            const int q = r < R ? rcell[r] : 0;
            const int v = r < R ? lcnt[q] : 0;
            int x = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (r < R) {
                cstart[q] = carry + x - v;
                rstart[r] = carry + x - v;
            }
            carry += __shfl(x, 63, 64);
        }
        if (lane == 0) total_sm = carry;
    }
    __syncthreads();
    const int total = total_sm;
    if (total > CAP) {
        // the region does not fit: the host moves to a larger staging
        // capacity or the per-atom kernel
        if (threadIdx.x == 0) atomicOr(&s.sc->overflow, 4);
        return;
    }
    // The rank of each staged position (a rank's atoms are consecutive
    // positions from its rstart) and each rank's atom-index offset, which
    // takes gbeg's place (indexed by rank from here on; one thread per rank,
    // R <= blockDim.x); then stage in rank order.
    static_assert(kRegion <= kListBlock, "one thread per rank");
    int off = 0;
    if ((int)threadIdx.x < R) {
        const int r = threadIdx.x, q = rcell[r];
        const int b = rstart[r], e = b + lcnt[q];
        off = gbeg[q] - b;
        for (int d = b; d < e; ++d) srank[d] = (uint8_t)r;
    }
    __syncthreads();
    if ((int)threadIdx.x < R) gbeg[threadIdx.x] = off;
    __syncthreads();
    for (int d = threadIdx.x; d < total; d += blockDim.x) {
        const int r = srank[d];
        const int j = d + gbeg[r];
        const double4 P = s.p[j];
        px[d] = P.x;
        py[d] = P.y;
        pz[d] = P.z;
        val[d] = PC ? (j | ((int)P.w << kIdxBits)) : j;
        srank[d] = rcode[r];
    }
    __syncthreads();
    // ordering cells of the block: 2 per split axis
    const int F0 = sx ? 2 : 1, F1 = sy ? 2 : 1, F2 = sz ? 2 : 1;
    const int F = F0 * F1 * F2;
    auto own_cell = [&](int f) {
        const int fx = f % F0, fy = (f / F0) % F1, fz = f / (F0 * F1);
        return ((sz ? 2 + fz : 0) * R1 + (sy ? 2 + fy : 0)) * R0 + (sx ? 2 + fx : 0);
    };
    // With at least 5 list cells along every axis and no stencil cell across
    // the box edge, every |d| < 2 L/n_c <= 0.4 L, so rint(d/L) = 0 and the
    // minimum image leaves d unchanged: skipping it gives the same bits.
    const bool interior = s.nc[0] >= 5 && s.nc[1] >= 5 && s.nc[2] >= 5 && cx0 > 0 && cx0 < s.nc[0] - 1 &&
                          cy0 > 0 && cy0 < s.nc[1] - 1 && cz0 > 0 && cz0 < s.nc[2] - 1;
    // largest list radius: the candidate bound, or a longer core radius
    double rl2 = fmax(s.hi2_list, s.rc2_list);
    if (PC)
        for (int t = 0; t < s.n_species * s.n_species; ++t) rl2 = fmax(rl2, thr[t].x);
    const double r_list = sqrt(rl2);
    // work units: (ordering cell f, group of kListA of its atoms), dealt to
    // the wavefronts in turn
    int n_units = 0;
    for (int f = 0; f < F; ++f) n_units += (lcnt[own_cell(f)] + kListA - 1) / kListA;
    const int cmax = s.cap_core - 1, kmax = s.cap_cand - 1;
    int16_t* qw = queue[wave];
    // Distances in the sweep, by block: kInterior, the plain difference;
    // kShift (every axis split, so each staged cell is one periodic image of
    // the block's neighbourhood), the difference minus L k with k the
    // staged cell's image code; kMinImage, the minimum image of each
    // difference.  All three give the bits of the minimum image for every
    // pair that can be in a list: a pair's image along a split axis differs
    // from the minimum image only where the two are at least L/2 apart along
    // that axis, beyond the list radius (at most a list cell, a third of L),
    // and with equal k the operations are the same: d - L k.
    enum { kInterior, kShift, kMinImage };
    auto sweep = [&](auto mode_tag, int a0, int na) {
        constexpr int MODE = decltype(mode_tag)::value;
        double xu[kListA], yu[kListA], zu[kListA];
        // per atom of the unit: core count in the low 16 bits, candidate
        // count in the high 16 (each at most the staged total <= CAP)
        static_assert(CAP < 65536, "counts fit 16 bits");
        int tu[kListA];
        uint32_t cnt2[kListA];
        const int v0 = __builtin_amdgcn_readfirstlane(val[a0]);
        const int i0 = PC ? v0 & kIdxMask : v0;
        // A unit's atoms are consecutive sorted atoms i0, i0 + 1, ... (one
        // ordering cell is one contiguous range): their candidate rows follow
        // each other from crow0, their core columns follow each other from
        // ccol0 up to the end of its 64-atom tile, and the next tile starts
        // cap_core * 64 entries on.
        int32_t* const crow0 = s.cand_idx + (size_t)(i0 - row0) * s.cap_cand;
        int32_t* const ccol0 = s.core_idx + (size_t)(i0 >> 6) * s.cap_core * 64 + (i0 & 63);
        const int tile_wrap = 64 - (i0 & 63);
        const int tile_skip = s.cap_core * 64 - 64;
        double blo[3] = {px[a0], py[a0], pz[a0]};
        double bhi[3] = {blo[0], blo[1], blo[2]};
#pragma unroll
        for (int u = 0; u < kListA; ++u) {
            const bool here = u < na;
            const int a = here ? a0 + u : a0;
            xu[u] = uniform_f64(here ? px[a] : __builtin_inf());
            yu[u] = uniform_f64(py[a]);
            zu[u] = uniform_f64(pz[a]);
            blo[0] = fmin(blo[0], px[a]), bhi[0] = fmax(bhi[0], px[a]);
            blo[1] = fmin(blo[1], yu[u]), bhi[1] = fmax(bhi[1], yu[u]);
            blo[2] = fmin(blo[2], zu[u]), bhi[2] = fmax(bhi[2], zu[u]);
            if (PC) tu[u] = here ? __builtin_amdgcn_readfirstlane(val[a]) >> kIdxBits : 0;
            cnt2[u] = 0;
        }
        // filter sphere of the unit (the atoms sit inside one ordering cell,
        // so the box is at most half a list cell per axis)
        const double cx = uniform_f64(0.5 * (blo[0] + bhi[0])), cy = uniform_f64(0.5 * (blo[1] + bhi[1])),
                     cz = uniform_f64(0.5 * (blo[2] + bhi[2]));
        double ru2 = 0.0;
#pragma unroll
        for (int u = 0; u < kListA; ++u) {
            if (u < na) {
                const double ex = xu[u] - cx, ey = yu[u] - cy, ez = zu[u] - cz;
                ru2 = fmax(ru2, ex * ex + ey * ey + ez * ez);
            }
        }
        const double rf = r_list + sqrt(ru2) + 1e-6 * (r_list + 1.0);
        const double rf2 = uniform_f64(rf * rf);
        // exact tests of queue entries [qh, qh + cnt) against the unit
        auto test_chunk = [&](int qh, int cnt) {
            // Wave-uniform values passed through an empty asm statement once
            // per chunk, so that the compiler derives the per-atom offsets and
            // conditions from them here (cheap scalar work) instead of holding
            // eight copies in scalar registers across the sweep, which spills.
            int tw = tile_wrap, ts = tile_skip, ck = s.cap_cand, nu = na, cm = cmax - 1, km = kmax - 1;
            const double4* pu_g = s.p + i0;
            asm volatile("" : "+s"(tw), "+s"(ts), "+s"(ck), "+s"(pu_g), "+s"(nu), "+s"(cm), "+s"(km));
            using cdouble = const __attribute__((address_space(4))) double;
            cdouble* pu = (cdouble*)pu_g;
            const bool in = lane < cnt;
            const int idx = in ? (int)qw[(qh + lane) & (kQueue - 1)] : 0;
            const int vj = val[idx];
            const int j = PC ? vj & kIdxMask : vj;
            const int tj = PC ? vj >> kIdxBits : 0;
            const double pxj = in ? px[idx] : __builtin_inf();
            const double pyj = py[idx], pzj = pz[idx];
            // staged position relative to the unit's first atom: lane is atom
            // u of the unit itself where rel == u
            const int rel = idx - a0;
            // L k per axis from the staged atom's image code (exact products)
            double lkx = 0.0, lky = 0.0, lkz = 0.0;
            if (MODE == kShift) {
                const uint32_t code = srank[idx];
                lkx = s.L[0] * (double)((int)(code << 30) >> 30);
                lky = s.L[1] * (double)((int)(code << 28) >> 30);
                lkz = s.L[2] * (double)((int)(code << 26) >> 30);
            }
#pragma unroll
            for (int u = 0; u < kListA; ++u) {
                if (u >= nu) break;  // wave-uniform
                // The unit atom's position, read again per chunk through the
                // scalar cache (constant address space: this kernel does not
                // write the positions); the same doubles as the staged copy.
                double dx = pu[4 * u] - pxj, dy = pu[4 * u + 1] - pyj, dz = pu[4 * u + 2] - pzj;
                if (MODE == kShift) {
                    dx = dx - lkx;
                    dy = dy - lky;
                    dz = dz - lkz;
                }
                if (MODE == kMinImage) {
                    dx = min_image(dx, s.L[0], s.invL[0]);
                    dy = min_image(dy, s.L[1], s.invL[1]);
                    dz = min_image(dz, s.L[2], s.invL[2]);
                }
                const double r2 = (dx * dx + dy * dy) + dz * dz;
                double rcl = s.rc2_list, lol = s.lo2_list;
                if (PC) {
                    const double2 th = thr[tu[u] * s.n_species + tj];
                    rcl = th.x;
                    lol = th.y;
                }
                // masks of single compares (each is the compare's own lane
                // mask), combined on the scalar unit
                const bool other = rel != u;
                const bool in_core = r2 < rcl, above = r2 >= lol, below = r2 < s.hi2_list;
                const uint64_t m_other = __builtin_amdgcn_ballot_w64(other);
                const uint64_t mc = __builtin_amdgcn_ballot_w64(in_core) & m_other;
                const uint64_t mk = __builtin_amdgcn_ballot_w64(above) & __builtin_amdgcn_ballot_w64(below) & m_other;
                const bool is_core = in_core & other;
                const bool is_cand = above & below & other;
                // Only hit lanes store (a step without hits issues no store);
                // hits past the capacity all land on the row's last usable
                // entry: the counts report the overflow and the host builds
                // again with longer rows.
                const int rc_ = min(mbcnt64(mc, (int)(cnt2[u] & 0xFFFFu)), cm);
                const int rk_ = min(mbcnt64(mk, (int)(cnt2[u] >> 16)), km);
                // byte offsets of atom i0 + u's core column and candidate row
                const uint32_t coff = (uint32_t)(u < tw ? u : u + ts) << 2;
                const uint32_t koff = (uint32_t)(u * ck) << 2;
                if (is_core) *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(ccol0) + (((uint32_t)rc_ << 8) + coff)) = j;
                if (is_cand) *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(crow0) + (((uint32_t)rk_ << 2) + koff)) = j;
                cnt2[u] += (uint32_t)__popcll(mc) + ((uint32_t)__popcll(mk) << 16);
            }
        };
        // first pass: keep the staged atoms inside the sphere, in staged
        // order; the queue never holds more than 127 entries (at most 63 left
        // over plus 64 new), so no entry is overwritten before it is tested
        int qn = 0, qh = 0;
        for (int t0 = 0; t0 < total; t0 += 64) {
            const int t = t0 + lane;
            bool keep = false;
            if (t < total) {
                double dx = cx - px[t], dy = cy - py[t], dz = cz - pz[t];
                if (MODE != kInterior) {
                    dx = min_image(dx, s.L[0], s.invL[0]);
                    dy = min_image(dy, s.L[1], s.invL[1]);
                    dz = min_image(dz, s.L[2], s.invL[2]);
                }
                keep = (dx * dx + dy * dy) + dz * dz < rf2;
            }
            const uint64_t mq = __builtin_amdgcn_ballot_w64(keep);
            if (keep) qw[(qn + mbcnt64(mq)) & (kQueue - 1)] = (int16_t)t;
            qn += __popcll(mq);
            // a wavefront's LDS accesses complete in order; the barrier keeps
            // the compiler from moving the queue reads above the writes
            __builtin_amdgcn_wave_barrier();
            if (qn - qh >= 64) {
                test_chunk(qh, 64);
                qh += 64;
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (qn > qh) test_chunk(qh, qn - qh);
#pragma unroll
        for (int u = 0; u < kListA; ++u) {
            if (lane == 0 && u < na) {
                const int va = val[a0 + u];
                const int i = PC ? va & kIdxMask : va;
                const int ncore = (int)(cnt2[u] & 0xFFFFu), ncand = (int)(cnt2[u] >> 16);
                s.core_cnt[i] = ncore;
                s.cand_cnt[i] = ncand;
                // same-address atomics serialise: only overflowing atoms
                // report; the last entry of a row is not usable here
                if (ncore >= s.cap_core || ncand >= s.cap_cand) {
                    atomicOr(&s.sc->overflow, 1);
                    atomicMax(&s.sc->max_core, ncore + 1);
                    atomicMax(&s.sc->max_cand, ncand + 1);
                }
            }
        }
    };
    constexpr int kWaves = kListBlock / 64;
    for (int unit = part * kWaves + wave; unit < n_units; unit += s.list_parts * kWaves) {
        int f = 0, g = unit;
        for (;; ++f) {
            const int nu = (lcnt[own_cell(f)] + kListA - 1) / kListA;
            if (g < nu) break;
            g -= nu;
        }
        const int q0 = own_cell(f);
        const int a0 = __builtin_amdgcn_readfirstlane(cstart[q0] + g * kListA);
        const int na = __builtin_amdgcn_readfirstlane(min(kListA, cstart[q0] + lcnt[q0] - a0));
        if (interior)
            sweep(std::integral_constant<int, kInterior>{}, a0, na);
        else if (sx && sy && sz)
            sweep(std::integral_constant<int, kShift>{}, a0, na);
        else
            sweep(std::integral_constant<int, kMinImage>{}, a0, na);
    }
}

// ---------------------------------------------------------------- pair forces
struct PairCoefF {
    float qq, A, sig, irho, C, D;
};

struct SogCoefF {
    int n_exp, chain, n_poly, pad;
    float a[kMaxExplicit];
    float fw[kMaxExplicit];
    float ew[kMaxExplicit];
    float pc[kMaxPoly];
    float pd[kMaxPoly];
};

// Pair force scalar f (F_i += f * r_ij) of eq. (15) with k_e on the Coulomb
// part, and the pair energy k_e q_i q_j N(r) + B_BMH(r), in FP64.
template <int J, bool ENERGY>
__device__ inline double pair_scalar_f64(const PairCoef& c, const SogCoef& g, double r2, double& u)
{
    const double ir = rsqrt(r2);
    const double r = r2 * ir;
    const double ir2 = ir * ir;
    const int n = g.n_exp;
    double fsum = 0.0, esum = 0.0;
    if (J == 1) {
        double gm = exp(-r2 * g.a[n - 1]);
        fsum = g.fw[n - 1] * gm;
        if (ENERGY) esum = g.ew[n - 1] * gm;
        for (int m = n - 2; m >= 0; --m) {
            gm = gm * gm;
            fsum = fma(g.fw[m], gm, fsum);
            if (ENERGY) esum = fma(g.ew[m], gm, esum);
        }
    } else {
        double ga = exp(-r2 * g.a[n - 1]);  // g_{m+2}
        double gb = exp(-r2 * g.a[n - 2]);  // g_{m+1}
        fsum = fma(g.fw[n - 2], gb, g.fw[n - 1] * ga);
        if (ENERGY) esum = fma(g.ew[n - 2], gb, g.ew[n - 1] * ga);
        for (int m = n - 3; m >= 0; --m) {
            const double gm = ga * ga;
            ga = gb;
            gb = gm;
            fsum = fma(g.fw[m], gm, fsum);
            if (ENERGY) esum = fma(g.ew[m], gm, esum);
        }
    }
    if (g.n_poly > 0) {
        double pf = g.pc[g.n_poly - 1];
        double pe = g.pd[g.n_poly - 1];
        for (int k = g.n_poly - 2; k >= 0; --k) {
            pf = fma(pf, r2, g.pc[k]);
            if (ENERGY) pe = fma(pe, r2, g.pd[k]);
        }
        fsum += pf;
        if (ENERGY) esum += pe;
    }
    const double rep = c.A * exp((c.sig - r) * c.irho);
    const double ir6 = ir2 * ir2 * ir2;
    const double ir8 = ir6 * ir2;
    const double f = c.qq * (ir2 * ir - fsum) + rep * c.irho * ir - 6.0 * c.C * ir8 - 8.0 * c.D * ir8 * ir2;
    if (ENERGY) u = c.qq * (ir - esum) + rep - c.C * ir6 - c.D * ir8;
    return f;
}

// FP32 form.  The SOG Coulomb kernels CF = -N'(r)/r and CU = N(r) come from
// the near-field table: the exponent and six leading mantissa bits of r^2
// pick the interval, whose cubic in t = r^2 - (its start) is evaluated by
// Horner (no transcendental).  Below the table (r^2 < 2^e0, never reached by
// a melt) every narrow Gaussian is evaluated by its own exponential.  The
// BMH terms are evaluated directly.
template <bool ENERGY>
__device__ inline float pair_scalar_f32(const PairCoefF& c, const SogCoefF& g, const float4* tab, int tab_lo,
                                        int tab_n, float r2, float& u)
{
    const float ir = __frsqrt_rn(r2);
    const float r = r2 * ir;
    const float ir2 = ir * ir;
    float cf, cu = 0.f;
    const uint32_t bits = __float_as_uint(r2);
    const int idx = (int)(bits >> 17) - tab_lo;
    if ((unsigned)idx < (unsigned)tab_n) {
        const float t = r2 - __uint_as_float(bits & 0xFFFE0000u);
        const float4 a = tab[ENERGY ? 2 * idx : idx];
        cf = fmaf(fmaf(fmaf(a.w, t, a.z), t, a.y), t, a.x);
        if (ENERGY) {
            const float4 b = tab[2 * idx + 1];
            cu = fmaf(fmaf(fmaf(b.w, t, b.z), t, b.y), t, b.x);
        }
    } else {
        float fsum = 0.f, esum = 0.f;
        for (int m = 0; m < g.n_exp; ++m) {
            const float gm = __expf(-r2 * g.a[m]);
            fsum = fmaf(g.fw[m], gm, fsum);
            if (ENERGY) esum = fmaf(g.ew[m], gm, esum);
        }
        if (g.n_poly > 0) {
            float pf = g.pc[g.n_poly - 1];
            float pe = g.pd[g.n_poly - 1];
            for (int k = g.n_poly - 2; k >= 0; --k) {
                pf = fmaf(pf, r2, g.pc[k]);
                if (ENERGY) pe = fmaf(pe, r2, g.pd[k]);
            }
            fsum += pf;
            if (ENERGY) esum += pe;
        }
        cf = ir2 * ir - fsum;
        if (ENERGY) cu = ir - esum;
    }
    const float rep = c.A * __expf((c.sig - r) * c.irho);
    const float ir6 = ir2 * ir2 * ir2;
    const float ir8 = ir6 * ir2;
    const float f = c.qq * cf + rep * c.irho * ir - 6.f * c.C * ir8 - 8.f * c.D * ir8 * ir2;
    if (ENERGY) u = c.qq * cu + rep - c.C * ir6 - c.D * ir8;
    return f;
}

// Floyd's selection of P_R distinct ranks out of n (Bentley & Floyd 1987) with
// a per-lane bitmask in LDS: step k draws t uniform in [0, n-P_R+k] and takes
// t, or n-P_R+k if t was already taken.
struct FloydMask {
    uint32_t* m;
    int stride;
    __device__ void clear(int n)
    {
        const int words = (n + 31) >> 5;
        for (int w = 0; w < words; ++w) m[w * stride] = 0u;
    }
    __device__ int step(PhiloxStream& st, int jj)
    {
        const uint32_t t = st.bounded((uint32_t)jj + 1u);
        const uint32_t wt = m[(t >> 5) * stride];
        int e = (int)t;
        if ((wt >> (t & 31)) & 1u) e = jj;
        m[(e >> 5) * stride] |= 1u << (e & 31);
        return e;
    }
};

// Adds one pair's force f r_ij to F and, with energies, half its energy to
// U and half of r_ij (x) f r_ij to the virial W (xx, yy, zz, xy, xz, yz).
template <bool ENERGY>
__device__ inline void add_pair(double f, double uu, double dx, double dy, double dz, double& Fx, double& Fy,
                                double& Fz, double& U, double* W)
{
    Fx = fma(f, dx, Fx);
    Fy = fma(f, dy, Fy);
    Fz = fma(f, dz, Fz);
    if (ENERGY) {
        U += 0.5 * uu;
        const double hx = 0.5 * f * dx, hy = 0.5 * f * dy;
        W[0] = fma(hx, dx, W[0]);
        W[1] = fma(hy, dy, W[1]);
        W[2] = fma(0.5 * f * dz, dz, W[2]);
        W[3] = fma(hx, dy, W[3]);
        W[4] = fma(hx, dz, W[4]);
        W[5] = fma(hy, dz, W[5]);
    }
}

// Pair forces of A atoms per workgroup (A = blockDim.x / 2): the first A
// threads (whole wavefronts) take the core lists, the other A the shell
// batches of the same atoms, so twice as many independent gather chains are
// in flight and no wavefront diverges between the two loops.  The shell
// thread adds its reweighted sum to the core sum passed through LDS, in the
// same order as one thread doing both.
template <bool MIXED, bool ENERGY, int J, int KU>
__global__ __launch_bounds__(2 * kBlock) void k_pair(RB_ARGS, SogCoef g, SogCoefF gf, NearTab nt)
{
    RB_SYS(xcd_block(blockIdx.x, gridDim.x))
    // dynamic LDS, sized by the launch: the near-field table (mixed form; F
    // coefficients, with energies also U), the core lanes' sums handed to the
    // shell lanes (F, and with energies u and the virial: 4 or 10 per atom),
    // then the Floyd masks of the per-evaluation draw.  Kept small: the
    // kernel waits on neighbour gathers, so resident waves are what counts.
    extern __shared__ float4 dyn_sm[];
    const int tab_vecs = MIXED ? nt.n * (ENERGY ? 2 : 1) : 0;
    const int A = blockDim.x >> 1;
    constexpr int kXch = ENERGY ? 10 : 4;
    float4* tab = dyn_sm;
    double* xch = reinterpret_cast<double*>(dyn_sm + tab_vecs);  // [kXch][A]
    uint32_t* mask_sm = reinterpret_cast<uint32_t*>(xch + kXch * A);
    if (MIXED) {
        const float4* src = glob(nt.coef);
        for (int t = threadIdx.x; t < tab_vecs; t += blockDim.x) tab[t] = ENERGY ? src[t] : src[2 * t];
    }
    // pair coefficients: FP64 for the FP64 form; the mixed form keeps FP32
    // copies and only the FP64 core radii (the core/shell test stays FP64)
    __shared__ PairCoef pc[MIXED ? 1 : kMaxSpecies * kMaxSpecies];
    __shared__ PairCoefF pcf[MIXED ? kMaxSpecies * kMaxSpecies : 1];
    __shared__ double rc2s[kMaxSpecies * kMaxSpecies];
    const int S = s.n_species;
    for (int t = threadIdx.x; t < S * S; t += blockDim.x) {
        const PairCoef c = s.pair[t];
        if (MIXED)
            pcf[t] = PairCoefF{(float)c.qq, (float)c.A, (float)c.sig, (float)c.irho, (float)c.C, (float)c.D};
        else
            pc[t] = c;
        rc2s[t] = c.rc2;
    }
    __syncthreads();

    const bool shell = threadIdx.x >= A;  // uniform per wavefront (A is a multiple of 64)
    const int ta = shell ? threadIdx.x - A : threadIdx.x;
    const int i = lb * A + ta;
    double Fx = 0.0, Fy = 0.0, Fz = 0.0, Uc = 0.0, Us = 0.0;
    double Sx = 0.0, Sy = 0.0, Sz = 0.0, Su = 0.0, wgt = 1.0;
    double Wv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // this lane's virial (core or shell sum)
    // A wavefront whose atoms all lie at least the list radius plus a skin
    // inside every face (inner_lo <= x <= inner_hi) has no list neighbour
    // across the box edge: each stored difference already is the minimum
    // image (|d| < 0.4 L, so rint(d / L) = 0) and the wrap is skipped, with
    // the same bits (FP64 form; the mixed form gathers fixed-point records,
    // whose differences wrap by themselves).
    bool inner = true;
    if (!MIXED && i < s.n) {
        const double4 Pi = s.p[i];
        inner = Pi.x >= s.inner_lo[0] && Pi.x <= s.inner_hi[0] && Pi.y >= s.inner_lo[1] && Pi.y <= s.inner_hi[1] &&
                Pi.z >= s.inner_lo[2] && Pi.z <= s.inner_hi[2];
    }
    const bool wave_inner = __builtin_amdgcn_ballot_w64(!inner) == 0ull;
    auto body = [&](auto inner_tag) {
    constexpr bool INNER = decltype(inner_tag)::value;
    auto mi = [&](double d, int a) { return INNER ? d : min_image(d, s.L[a], s.invL[a]); };
    if (i < s.n) {
        const double4 Pi = s.p[i];
        const double xi = Pi.x, yi = Pi.y, zi = Pi.z;
        const int ti = s.type[i];
        const uint4 Ui = MIXED ? s.ufix[i] : make_uint4(0u, 0u, 0u, 0u);
        // fixed-point units per axis (L 2^-32, exact)
        const double ux = s.L[0] * 0x1p-32, uy = s.L[1] * 0x1p-32, uz = s.L[2] * 0x1p-32;
        // pair force scalar for r2 of species pair (ti, tj)
        auto pair_f = [&](int tj, double r2, double& u) -> double {
            const int t = ti * S + tj;
            if (MIXED) {
                float uf = 0.f;
                const double f = (double)pair_scalar_f32<ENERGY>(pcf[t], gf, tab, nt.lo, nt.n, (float)r2, uf);
                u = uf;
                return f;
            }
            return pair_scalar_f64<J, ENERGY>(pc[t], g, r2, u);
        };
        // Neighbours jj[0..kU) (entries k0.. of a list of cnt; padding past
        // cnt) are fetched before any arithmetic, so the gathers overlap; the
        // sums still run in list order.  SH: the shell test r_core^2 <= r^2 <
        // r_shell^2, else the core test r^2 < r_core^2, each decided on the
        // FP64 minimum image.  The mixed form reads a neighbour's 16-byte
        // fixed-point record (one load instead of two for the FP64 one): the
        // record differences give r^2 within fix_guard of the FP64 value, and
        // the rare pair that close to a cutoff is decided (and evaluated)
        // from the FP64 positions, so the pair set is the FP64 one.
        auto visit = [&](auto shell_tag, const int* jj, int k0, int cnt, double& Ax, double& Ay, double& Az,
                         double& Au) {
            constexpr bool SH = decltype(shell_tag)::value;
            if (MIXED) {
                uint4 Q[KU];
#pragma unroll
                for (int u = 0; u < KU; ++u) Q[u] = s.ufix[jj[u]];
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    if (k0 + u >= cnt) break;
                    double dx = (double)(int32_t)(Ui.x - Q[u].x) * ux;
                    double dy = (double)(int32_t)(Ui.y - Q[u].y) * uy;
                    double dz = (double)(int32_t)(Ui.z - Q[u].z) * uz;
                    double r2 = (dx * dx + dy * dy) + dz * dz;
                    const int tj = (int)Q[u].w;
                    const double rc2 = s.species_cut ? rc2s[ti * S + tj] : s.rc2;
                    if (fabs(r2 - rc2) <= s.fix_guard || (SH && fabs(r2 - s.rs2) <= s.fix_guard)) {
                        const double4 Q64 = s.p[jj[u]];
                        dx = min_image(xi - Q64.x, s.L[0], s.invL[0]);
                        dy = min_image(yi - Q64.y, s.L[1], s.invL[1]);
                        dz = min_image(zi - Q64.z, s.L[2], s.invL[2]);
                        r2 = (dx * dx + dy * dy) + dz * dz;
                    }
                    if (SH ? (r2 >= rc2 && r2 < s.rs2) : (r2 < rc2)) {
                        double uu = 0.0;
                        const double f = pair_f(tj, r2, uu);
                        add_pair<ENERGY>(f, uu, dx, dy, dz, Ax, Ay, Az, Au, Wv);
                    }
                }
            } else {
                double X[KU], Y[KU], Z[KU];
                int T[KU];
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    const double4 Q = s.p[jj[u]];
                    X[u] = Q.x;
                    Y[u] = Q.y;
                    Z[u] = Q.z;
                    T[u] = (int)Q.w;
                }
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    if (k0 + u >= cnt) break;
                    const double dx = mi(xi - X[u], 0);
                    const double dy = mi(yi - Y[u], 1);
                    const double dz = mi(zi - Z[u], 2);
                    const double r2 = (dx * dx + dy * dy) + dz * dz;
                    const double rc2 = s.species_cut ? rc2s[ti * S + T[u]] : s.rc2;
                    if (SH ? (r2 >= rc2 && r2 < s.rs2) : (r2 < rc2)) {
                        double uu = 0.0;
                        const double f = pair_f(T[u], r2, uu);
                        add_pair<ENERGY>(f, uu, dx, dy, dz, Ax, Ay, Az, Au, Wv);
                    }
                }
            }
        };
        // Core-list lines are read once: non-temporal loads keep them from
        // evicting the positions that neighbours re-read (a candidate row is
        // re-read by its own lane, so it stays cached).
        constexpr int kU = KU;
        if (!shell) {
            // core sum, eq. (24)
            const int nc = min(s.core_cnt[i], s.cap_core - 1);
            const int32_t* ctile = s.core_idx + (size_t)(i >> 6) * s.cap_core * 64 + (i & 63);
            for (int k0 = 0; k0 < nc; k0 += kU) {
                int jj[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    jj[u] = (k0 + u < nc) ? __builtin_nontemporal_load(ctile + (size_t)(k0 + u) * 64) : i;
                visit(std::false_type{}, jj, k0, nc, Fx, Fy, Fz, Uc);
            }
        } else if (s.shell_stored) {
            // shell batch of eq. (25) drawn at the list build: a tile row per
            // atom, read coalesced like the core list
            const int n = min(s.cand_cnt[i], s.cap_cand - 1);
            const bool take_all = n <= s.p_r;
            const int cnt = take_all ? n : s.p_r;
            wgt = take_all ? 1.0 : (double)n / (double)s.p_r;
            const int32_t* btile = s.bat_idx + (size_t)(i >> 6) * s.p_r * 64 + (i & 63);
            for (int k0 = 0; k0 < cnt; k0 += kU) {
                int jj[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    jj[u] = (k0 + u < cnt) ? __builtin_nontemporal_load(btile + (size_t)(k0 + u) * 64) : i;
                visit(std::true_type{}, jj, k0, cnt, Sx, Sy, Sz, Su);
            }
        } else {
            // shell batch, eq. (25)
            const int n = min(s.cand_cnt[i], s.cap_cand - 1);
            const int32_t* crow = s.cand_idx + (size_t)i * s.cap_cand;
            const bool take_all = s.p_r <= 0 || n <= s.p_r;
            const int cnt = take_all ? n : s.p_r;
            wgt = take_all ? 1.0 : (double)n / (double)s.p_r;
            FloydMask fm{mask_sm + ta, A};
            PhiloxStream st(s.seed, (uint32_t)s.id[i], (uint32_t)s.sc->eval, kTagShell, s.replica);
            if (!take_all) {
                // draw the whole batch first, then visit the ranks in ascending
                // order: the candidate row is swept once, line by line
                fm.clear(n);
                for (int k = 0; k < cnt; ++k) fm.step(st, n - s.p_r + k);
            }
            int w_cur = 0;  // ascending walk over the set bits of the mask
            uint32_t m_cur = take_all ? 0u : fm.m[0];
            for (int k0 = 0; k0 < cnt; k0 += kU) {
                int jj[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    int e = 0;
                    if (k0 + u < cnt) {
                        if (take_all) {
                            e = k0 + u;
                        } else {
                            while (m_cur == 0u) m_cur = fm.m[(++w_cur) * fm.stride];
                            e = w_cur * 32 + __builtin_ctz(m_cur);
                            m_cur &= m_cur - 1u;
                        }
                    }
                    jj[u] = (k0 + u < cnt) ? crow[e] : i;
                }
                visit(std::true_type{}, jj, k0, cnt, Sx, Sy, Sz, Su);
            }
        }
    }
    };
    if (MIXED || wave_inner)
        body(std::true_type{});
    else
        body(std::false_type{});
    if (!shell) {
        xch[0 * A + ta] = Fx;
        xch[1 * A + ta] = Fy;
        xch[2 * A + ta] = Fz;
        xch[3 * A + ta] = Uc;
        if (ENERGY)
            for (int c = 0; c < 6; ++c) xch[(4 + c) * A + ta] = Wv[c];
    }
    __syncthreads();
    if (shell) {
        if (i < s.n) {
            Fx = fma(wgt, Sx, xch[0 * A + ta]);
            Fy = fma(wgt, Sy, xch[1 * A + ta]);
            Fz = fma(wgt, Sz, xch[2 * A + ta]);
            Uc = xch[3 * A + ta];
            if (ENERGY) {
                Us = wgt * Su;
                for (int c = 0; c < 6; ++c) Wv[c] = fma(wgt, Wv[c], xch[(4 + c) * A + ta]);
            }
            __builtin_nontemporal_store(Fx, s.fsx + i);
            __builtin_nontemporal_store(Fy, s.fsy + i);
            __builtin_nontemporal_store(Fz, s.fsz + i);
            if (ENERGY) {
                // the atom's shares of the short-range energy and virial
                s.at_ew[2 * (size_t)i] = make_double4(Uc + Us, Wv[0], Wv[1], Wv[2]);
                s.at_ew[2 * (size_t)i + 1] = make_double4(Wv[3], Wv[4], Wv[5], 0.0);
            }
        }
        wave_partial(Fx, i, s.n, s.pair_part, kPairPart, 0);
        wave_partial(Fy, i, s.n, s.pair_part, kPairPart, 1);
        wave_partial(Fz, i, s.n, s.pair_part, kPairPart, 2);
        wave_partial(Uc, i, s.n, s.pair_part, kPairPart, 3);
        wave_partial(Us, i, s.n, s.pair_part, kPairPart, 4);
        if (ENERGY)
            for (int c = 0; c < 6; ++c) wave_partial(Wv[c], i, s.n, s.vir_part, kVirPart, c);
    }
}

// Export of the shell ranks drawn by the pair kernel (same selection code).
__global__ __launch_bounds__(kBlock) void k_shell_ranks(RB_ARGS, int32_t* out, int32_t* n_out)
{
    RB_SYS(blockIdx.x)
    extern __shared__ uint32_t mask_sm[];
    const int i = lb * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const int n = min(s.cand_cnt[i], s.cap_cand - 1);
    const int P = s.p_r;
    const int uid = s.id[i];
    int32_t* o = out + (size_t)uid * (P > 0 ? P : 1);
    if (P <= 0 || n <= P) {
        n_out[uid] = n;
        for (int k = 0; k < (P > 0 ? P : 0); ++k) o[k] = k < n ? k : -1;
        return;
    }
    FloydMask fm{mask_sm + threadIdx.x, (int)blockDim.x};
    PhiloxStream st(s.seed, (uint32_t)uid, (uint32_t)s.sc->eval, kTagShell, s.replica);
    fm.clear(n);
    for (int k = 0; k < P; ++k) o[k] = fm.step(st, n - P + k);
    n_out[uid] = P;
}

// Export of the shell batch of the current evaluation as atom ids, in
// ascending rank order: the pair kernel's selection mapped through the
// candidate row (P_R >= 1).
__global__ __launch_bounds__(kBlock) void k_shell_samples(RB_ARGS, int32_t* out, int32_t* n_out)
{
    RB_SYS(blockIdx.x)
    extern __shared__ uint32_t mask_sm[];
    const int i = lb * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const int n = min(s.cand_cnt[i], s.cap_cand - 1);
    const int P = s.p_r;
    const int uid = s.id[i];
    const int32_t* crow = s.cand_idx + (size_t)i * s.cap_cand;
    int32_t* o = out + (size_t)uid * P;
    n_out[uid] = n;
    if (n <= P) {
        for (int k = 0; k < P; ++k) o[k] = k < n ? s.id[crow[k]] : -1;
        return;
    }
    FloydMask fm{mask_sm + threadIdx.x, (int)blockDim.x};
    PhiloxStream st(s.seed, (uint32_t)uid, (uint32_t)s.sc->eval, kTagShell, s.replica);
    fm.clear(n);
    for (int k = 0; k < P; ++k) fm.step(st, n - P + k);
    int w = 0;
    uint32_t m = fm.m[0];
    for (int k = 0; k < P; ++k) {
        while (m == 0u) m = fm.m[(++w) * fm.stride];
        const int e = w * 32 + __builtin_ctz(m);
        m &= m - 1u;
        o[k] = s.id[crow[e]];
    }
}

// Memory form of the list: the shell batch of each atom of build chunk
// `chunk`, drawn once at the build (Floyd's selection as in the pair kernel,
// on the stream (id, build number, kTagShellBuild)) from its candidate row,
// stored in ascending rank order as atom indices in the atom's tile row.
__global__ __launch_bounds__(64) void k_select(RB_ARGS, int gate, int chunk)
{
    RB_SYS(blockIdx.x)
    RB_GATE
    extern __shared__ uint32_t mask_sm[];
    if (chunk >= s.n_chunks) return;
    const int row0 = chunk_first_atom(s, chunk);
    const int row1 = chunk_first_atom(s, chunk + 1);
    const int t = lb * 64 + threadIdx.x;
    const int a = row0 + t;
    // rows of a chunk that did not fit were not built (the host builds again)
    if (row1 - row0 > s.cand_rows || t >= s.cand_rows || a >= row1) return;
    const int n = min(s.cand_cnt[a], s.cap_cand - 1);
    const int P = s.p_r;
    const int32_t* crow = s.cand_idx + (size_t)t * s.cap_cand;
    int32_t* btile = s.bat_idx + (size_t)(a >> 6) * P * 64 + (a & 63);
    if (n <= P) {
        for (int k = 0; k < n; ++k) btile[(size_t)k * 64] = crow[k];
        return;
    }
    FloydMask fm{mask_sm + threadIdx.x, 64};
    PhiloxStream st(s.seed, (uint32_t)s.id[a], (uint32_t)s.sc->n_builds, kTagShellBuild, s.replica);
    fm.clear(n);
    for (int k = 0; k < P; ++k) fm.step(st, n - P + k);
    int w = 0;
    uint32_t m = fm.m[0];
    for (int k = 0; k < P; ++k) {
        while (m == 0u) m = fm.m[(++w) * fm.stride];
        const int e = w * 32 + __builtin_ctz(m);
        m &= m - 1u;
        btile[(size_t)k * 64] = crow[e];
    }
}

// Export of the stored batch as atom ids (ascending rank order).
__global__ __launch_bounds__(kBlock) void k_batch_ids(RB_ARGS, int32_t* out, int32_t* n_out)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const int n = min(s.cand_cnt[i], s.cap_cand - 1);
    const int P = s.p_r;
    const int cnt = min(n, P);
    const int uid = s.id[i];
    const int32_t* btile = s.bat_idx + (size_t)(i >> 6) * P * 64 + (i & 63);
    for (int k = 0; k < P; ++k) out[(size_t)uid * P + k] = k < cnt ? s.id[btile[(size_t)k * 64]] : -1;
    n_out[uid] = n;
}

// ---------------------------------------------------------------- k-space
__device__ inline int first_above(const double* cdf, int len, double u)
{
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u < cdf[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo < len ? lo : len - 1;
}

// The same index by one wavefront: each round the lanes probe the ends of 64
// equal slices of [lo, hi) and keep the first slice that reaches above u,
// so a table of L entries takes about log64(L) dependent loads instead of
// log2(L).  Every lane returns the index.
__device__ inline int first_above_wave(const double* cdf, int len, double u)
{
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = len;  // the first index above u (len: none) lies in [lo, hi]
    while (hi - lo > 64) {
        const int step = (hi - lo + 63) >> 6;
        const int probe = lo + (lane + 1) * step - 1;
        const bool above = probe >= hi || u < cdf[probe];
        const uint64_t m = __builtin_amdgcn_ballot_w64(above);
        if (m == 0) {
            lo = hi;
            break;
        }
        const int f = __builtin_ctzll(m);
        const int nlo = f == 0 ? lo : lo + f * step;
        hi = min(lo + (f + 1) * step - 1, hi);
        lo = nlo;
    }
    if (hi - lo > 0) {
        const int idx = lo + lane;
        const bool above = idx >= hi || u < cdf[idx];
        const uint64_t m = __builtin_amdgcn_ballot_w64(above);
        lo = m == 0 ? hi : lo + __builtin_ctzll(m);
    }
    return lo < len ? lo : len - 1;
}

// Draw the P_F modes of eq. (28): component (m, d) by its mass, then the
// three axis indices from their 1D lattice distributions, then signs.  One
// wavefront per mode (the searches are wave-cooperative).
__global__ __launch_bounds__(64) void k_ksample(RB_ARGS, const KDev* __restrict__ kd)
{
    RB_SYS(blockIdx.x)
    const KDev k = global_view(kd[rb_m.x]);
    const int p = lb;
    if (!k.sampled || p >= k.n_modes) return;
    PhiloxStream st(s.seed, (uint32_t)p, (uint32_t)s.sc->eval, kTagKmode, s.replica);
    const double uc = st.uniform();
    double ua[3];
    for (int a = 0; a < 3; ++a) ua[a] = st.uniform();
    const uint32_t signs = st.next();
    const int c = first_above_wave(k.comp_cdf, k.nm * 3, uc);
    const int m = c / 3, d = c % 3;
    int mi[3];
    for (int a = 0; a < 3; ++a) {
        const int o = k.off[m * 3 + a], L = k.len[m * 3 + a];
        const double* cdf = (a == d) ? k.g2cdf + o : k.g0cdf + o;
        int nn = first_above_wave(cdf, L, ua[a]);
        if (nn > 0 && ((signs >> a) & 1u)) nn = -nn;
        mi[a] = nn;
    }
    if (threadIdx.x != 0) return;
    k.m[3 * p] = mi[0];
    k.m[3 * p + 1] = mi[1];
    k.m[3 * p + 2] = mi[2];
    double k2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double kk = s.two_pi_L[a] * (double)mi[a];
        k2 += kk * kk;
    }
    ModeRec r;
    r.mx = mi[0];
    r.my = mi[1];
    r.mz = mi[2];
    r.A = 0.0;
    r.B = 0.0;
    r.coef = k.coef_scale / k2;
    r.e = 0.0;
    r.Af = 0.0f;
    r.Bf = 0.0f;
    k.modes[p] = r;
}

// e^{2 pi i t / 1024} for a phase t in units of 2 pi / 1024: table entry
// rint(t) mod 1024 rotated by the remainder, whose sine and cosine come from
// short Taylor series (|x| <= pi/1024, truncation below 1e-18).
__device__ inline void sincos1024(double t, const double2* tab, double& c, double& s)
{
    const double j = rint(t);
    const double x = (t - j) * (2.0 * kPi / kTableSize);
    const double x2 = x * x;
    const double cd = fma(x2, fma(x2, 1.0 / 24.0, -0.5), 1.0);
    const double sd = fma(x * x2, fma(x2, 1.0 / 120.0, -1.0 / 6.0), x);
    const double2 T = tab[((int)j) & (kTableSize - 1)];
    c = fma(T.x, cd, -(T.y * sd));
    s = fma(T.y, cd, T.x * sd);
}

// Phase in turns (MIXED) or in units of 2 pi / 1024 (FP64) of one atom
// against one mode whose integer vector already carries the box scale.
__device__ inline double mode_phase(double kx, double ky, double kz, const double4& P)
{
    return fma(kz, P.z, fma(ky, P.y, kx * P.x));
}

// FP32 sine and cosine of a phase in turns: the fractional turn (one FP64
// op) is rounded to FP32 and fed to the hardware sin/cos, which take turns.
__device__ inline void sincos_turns_f32(double t, float& c, float& s)
{
    const float fr = (float)__builtin_amdgcn_fract(t);
    c = __builtin_amdgcn_cosf(fr);
    s = __builtin_amdgcn_sinf(fr);
}

// rho(k) of eq. (22) over one atom chunk for 64 MPL modes: MPL modes per
// lane, each of the four waves of the block takes a contiguous quarter of the
// chunk, four atoms per iteration, atoms read through the scalar unit (one
// read serves 64 MPL modes).  Partial sums per chunk, reduced later in a fixed
// order; MPL changes neither the per-mode summation order nor the result.
// The mixed form sums the four FP32 products q cos, q sin of an iteration in
// FP32 and adds that to the FP64 accumulators.
// Fixed-point phase (IPH, mixed form): positions as 32-bit fractions of the
// box u (the fixed-point records), the phase m . u wraps exactly modulo 2^32 (one turn), and
// its signed value times 2^-32 is the FP32 turn fed to the hardware sin/cos.
__device__ inline float turns_fix(int mx, int my, int mz, const uint4& U)
{
    const uint32_t ph = (uint32_t)mx * U.x + (uint32_t)my * U.y + (uint32_t)mz * U.z;
    return (float)(int32_t)ph * 2.3283064365386963e-10f;
}

template <bool MIXED, int MPL, bool IPH>
__global__ __launch_bounds__(kBlock) void k_rho(RB_ARGS, const KDev* __restrict__ kd)
{
    RB_SYS(blockIdx.x)
    const KDev k = global_view(kd[rb_m.x]);
    const int chunk = lb % k.n_chunks;
    const int tile = lb / k.n_chunks;
    __shared__ double2 tab[MIXED ? 1 : kTableSize];
    __shared__ double red[4][64 * MPL][2];
    using qreal = typename std::conditional<MIXED, float, double>::type;
    __shared__ qreal qs[kMaxSpecies];
    if (!MIXED)
        for (int t = threadIdx.x; t < kTableSize; t += blockDim.x)
            tab[t] = make_double2(k.table[2 * t], k.table[2 * t + 1]);
    if (threadIdx.x < kMaxSpecies) qs[threadIdx.x] = (qreal)s.spc->q[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double sc = MIXED ? 1.0 : (double)kTableSize;
    double kx[MPL], ky[MPL], kz[MPL], re[MPL], im[MPL];
    int mi[MPL][3];
#pragma unroll
    for (int j = 0; j < MPL; ++j) {
        const int p = tile * 64 * MPL + 64 * j + lane;
        const ModeRec mr = p < k.n_modes ? k.modes[p] : ModeRec{};
        kx[j] = mr.mx * (sc * s.invL[0]);
        ky[j] = mr.my * (sc * s.invL[1]);
        kz[j] = mr.mz * (sc * s.invL[2]);
        for (int a = 0; a < 3; ++a) mi[j][a] = (IPH && p < k.n_modes) ? k.m[3 * p + a] : 0;
        re[j] = 0.0;
        im[j] = 0.0;
    }
    // chunk and its quarters are multiples of four atoms (host guarantees
    // chunk % 16 == 0), so the type quadruples below are aligned
    const int qw = k.chunk >> 2;
    const int a0 = chunk * k.chunk + wave * qw;
    const int a1 = min(s.n, a0 + qw);
    int a = a0;
    if (IPH) {
        for (; a + 4 <= a1; a += 4) {
            const uint4 U0 = s.ufix[a], U1 = s.ufix[a + 1], U2 = s.ufix[a + 2], U3 = s.ufix[a + 3];
            const qreal q0 = qs[U0.w], q1 = qs[U1.w], q2 = qs[U2.w], q3 = qs[U3.w];
#pragma unroll
            for (int j = 0; j < MPL; ++j) {
                const float t0 = turns_fix(mi[j][0], mi[j][1], mi[j][2], U0);
                const float t1 = turns_fix(mi[j][0], mi[j][1], mi[j][2], U1);
                const float t2 = turns_fix(mi[j][0], mi[j][1], mi[j][2], U2);
                const float t3 = turns_fix(mi[j][0], mi[j][1], mi[j][2], U3);
                const float c0 = __builtin_amdgcn_cosf(t0), s0 = __builtin_amdgcn_sinf(t0);
                const float c1 = __builtin_amdgcn_cosf(t1), s1 = __builtin_amdgcn_sinf(t1);
                const float c2 = __builtin_amdgcn_cosf(t2), s2 = __builtin_amdgcn_sinf(t2);
                const float c3 = __builtin_amdgcn_cosf(t3), s3 = __builtin_amdgcn_sinf(t3);
                const float rs = fmaf(q3, c3, fmaf(q2, c2, fmaf(q1, c1, q0 * c0)));
                const float is = fmaf(q3, s3, fmaf(q2, s2, fmaf(q1, s1, q0 * s0)));
                re[j] += (double)rs;
                im[j] += (double)is;
            }
        }
        for (; a < a1; ++a) {
            const uint4 U = s.ufix[a];
            const qreal q = qs[U.w];
#pragma unroll
            for (int j = 0; j < MPL; ++j) {
                const float t = turns_fix(mi[j][0], mi[j][1], mi[j][2], U);
                re[j] += (double)(q * __builtin_amdgcn_cosf(t));
                im[j] += (double)(q * __builtin_amdgcn_sinf(t));
            }
        }
    }
    for (; !IPH && a + 4 <= a1; a += 4) {
        const double4 P0 = s.p[a], P1 = s.p[a + 1], P2 = s.p[a + 2], P3 = s.p[a + 3];
        const int4 T = *reinterpret_cast<const int4*>(s.type + a);
        const qreal q0 = qs[T.x], q1 = qs[T.y], q2 = qs[T.z], q3 = qs[T.w];
#pragma unroll
        for (int j = 0; j < MPL; ++j) {
            const double t0 = mode_phase(kx[j], ky[j], kz[j], P0), t1 = mode_phase(kx[j], ky[j], kz[j], P1);
            const double t2 = mode_phase(kx[j], ky[j], kz[j], P2), t3 = mode_phase(kx[j], ky[j], kz[j], P3);
            if (MIXED) {
                float c0, s0, c1, s1, c2, s2, c3, s3;
                sincos_turns_f32(t0, c0, s0);
                sincos_turns_f32(t1, c1, s1);
                sincos_turns_f32(t2, c2, s2);
                sincos_turns_f32(t3, c3, s3);
                const float rs = fmaf(q3, c3, fmaf(q2, c2, fmaf(q1, c1, q0 * c0)));
                const float is = fmaf(q3, s3, fmaf(q2, s2, fmaf(q1, s1, q0 * s0)));
                re[j] += (double)rs;
                im[j] += (double)is;
            } else {
                double c0, s0, c1, s1, c2, s2, c3, s3;
                sincos1024(t0, tab, c0, s0);
                sincos1024(t1, tab, c1, s1);
                sincos1024(t2, tab, c2, s2);
                sincos1024(t3, tab, c3, s3);
                re[j] = fma(q3, c3, fma(q2, c2, fma(q1, c1, fma(q0, c0, re[j]))));
                im[j] = fma(q3, s3, fma(q2, s2, fma(q1, s1, fma(q0, s0, im[j]))));
            }
        }
    }
    for (; !IPH && a < a1; ++a) {
        const double4 P = s.p[a];
        const qreal q = qs[s.type[a]];
#pragma unroll
        for (int j = 0; j < MPL; ++j) {
            const double t = mode_phase(kx[j], ky[j], kz[j], P);
            if (MIXED) {
                float c, sn;
                sincos_turns_f32(t, c, sn);
                re[j] += (double)(q * c);
                im[j] += (double)(q * sn);
            } else {
                double c, sn;
                sincos1024(t, tab, c, sn);
                re[j] = fma(q, c, re[j]);
                im[j] = fma(q, sn, im[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < MPL; ++j) {
        red[wave][64 * j + lane][0] = re[j];
        red[wave][64 * j + lane][1] = im[j];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < MPL; ++j) {
            const int p = tile * 64 * MPL + 64 * j + lane;
            if (p >= k.n_modes) continue;
            const int l = 64 * j + lane;
            const double r = ((red[0][l][0] + red[1][l][0]) + red[2][l][0]) + red[3][l][0];
            const double i = ((red[0][l][1] + red[1][l][1]) + red[2][l][1]) + red[3][l][1];
            double* o = k.rho_part + ((size_t)chunk * k.n_modes_pad + p) * 2;
            o[0] = r;
            o[1] = i;
        }
    }
}

// Sum of F^(k) terms at k^2 (value and -F^'(k)/k) for the mode virial.
__device__ inline double mode_g(const KDev& k, double k2)
{
    double F = 0.0, G = 0.0;
    for (int m = 0; m < k.n_sog; ++m) {
        const double e = k.sog_c[m] * exp(-0.5 * k.sog_s2[m] * k2);
        F += e;
        G = fma(e, k.sog_s2[m], G);
    }
    return F > 0.0 ? G / F : 0.0;
}

// rho_p = sum over chunks (fixed tree), then the per-mode force coefficients.
__global__ __launch_bounds__(64) void k_rho_finalize(RB_ARGS, const KDev* __restrict__ kd)
{
    RB_SYS(blockIdx.x)
    (void)s;
    const KDev k = global_view(kd[rb_m.x]);
    const int p = lb;
    const int lane = threadIdx.x;
    double re = 0.0, im = 0.0;
    // unrolled so the loads are in flight together; the sum order is unchanged
#pragma unroll 8
    for (int c = lane; c < k.n_chunks; c += 64) {
        const double* o = k.rho_part + ((size_t)c * k.n_modes_pad + p) * 2;
        re += o[0];
        im += o[1];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
        k.rho[2 * p] = re;
        k.rho[2 * p + 1] = im;
        ModeRec& r = k.modes[p];
        const double cf = r.coef;
        r.A = cf * im;
        r.B = cf * re;
        r.e = cf * (re * re + im * im);
        r.Af = (float)r.A;
        r.Bf = (float)r.B;
    }
}

// Momentum correction (eq. 26) and energy sums, first pass: block b of each
// system sums slice b of the wavefront partials and of the modes, and writes
// the kFin sums to fin_part[b].
__global__ __launch_bounds__(256) void k_finalize_part(const DevSys* __restrict__ sys, const KDev* __restrict__ kd,
                                                       int energy, int grid)
{
    const int r = blockIdx.x / grid, b = blockIdx.x - r * grid;
    const DevSys s = global_view(sys[r]);
    const int nf = fin_blocks(s.n);
    if (b >= nf) return;  // a smaller system of a batch
    const KDev k = global_view(kd[r]);
    const double* part = s.pair_part;
    const int nb = (s.n + 63) / 64;  // wavefront partials
    const int w0 = nb * b / nf, w1 = nb * (b + 1) / nf;  // nb * 32 fits 32 bits
    __shared__ double red[4];
    double v[kPairPart + kVirPart];
    for (int c = 0; c < kPairPart + kVirPart; ++c) v[c] = 0.0;
#pragma unroll 4
    for (int w = w0 + (int)threadIdx.x; w < w1; w += blockDim.x)
        for (int c = 0; c < kPairPart; ++c) v[c] += part[(size_t)w * kPairPart + c];
    if (energy) {
#pragma unroll 4
        for (int w = w0 + (int)threadIdx.x; w < w1; w += blockDim.x)
            for (int c = 0; c < kVirPart; ++c) v[kPairPart + c] += s.vir_part[(size_t)w * kVirPart + c];
    }
    const int nc = energy ? kPairPart + kVirPart : kPairPart;
    double ue = 0.0;
    double wk[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int nm = s.n > 0 ? k.n_modes : 0;  // an empty system sums no modes
    const int m0 = nm * b / nf, m1 = nm * (b + 1) / nf;
    for (int p = m0 + (int)threadIdx.x; p < m1; p += blockDim.x) {
        const ModeRec mr = k.modes[p];
        ue += mr.e;
        if (energy) {
            // strain derivative of the mode's energy: e (delta_ab - g k_a k_b)
            // g of the mode, kept for the per-atom shares of the fused pass
            const double kx = s.two_pi_L[0] * mr.mx, ky = s.two_pi_L[1] * mr.my, kz = s.two_pi_L[2] * mr.mz;
            const double g = mode_g(k, (kx * kx + ky * ky) + kz * kz);
            k.mode_g[p] = g;
            const double eg = mr.e * g;
            wk[0] += mr.e - eg * kx * kx;
            wk[1] += mr.e - eg * ky * ky;
            wk[2] += mr.e - eg * kz * kz;
            wk[3] -= eg * kx * ky;
            wk[4] -= eg * kx * kz;
            wk[5] -= eg * ky * kz;
        }
    }
    // nc and energy are uniform, so every thread takes part in each block_sum
    double* out = s.fin_part + (size_t)b * kFin;
#pragma unroll
    for (int c = 0; c < kPairPart + kVirPart; ++c) {
        const double t = c < nc ? block_sum(v[c], red) : 0.0;
        if (threadIdx.x == 0) out[c] = t;
    }
    const double ut = block_sum(ue, red);
    if (threadIdx.x == 0) out[kPairPart + kVirPart] = ut;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const double t = energy ? block_sum(wk[c], red) : 0.0;
        if (threadIdx.x == 0) out[kPairPart + kVirPart + 1 + c] = t;
    }
}

// Second pass: one wavefront per system; lane q adds quantity q of the
// system's fin_blocks(n) block sums in block order, and the evaluation's
// scalars are written from them.
__global__ __launch_bounds__(64) void k_finalize(const DevSys* __restrict__ sys, int energy)
{
    const DevSys s = global_view(sys[blockIdx.x]);
    const int q = threadIdx.x;
    double t = 0.0;
    const int nf = fin_blocks(s.n);
    // every row is read (all loads in flight together); rows past nf add 0
    if (q < kFin) {
#pragma unroll
        for (int b = 0; b < kFinBlocks; ++b) {
            const double x = s.fin_part[(size_t)b * kFin + q];
            t += b < nf ? x : 0.0;
        }
    }
    auto get = [&](int c) { return __shfl(t, c, 64); };
    double tot[kFin];
#pragma unroll
    for (int c = 0; c < kFin; ++c) tot[c] = get(c);
    if (q == 0) {
        DeviceScalars* sc = s.sc;
        const double inv_n = s.n > 0 ? 1.0 / (double)s.n : 0.0;
        sc->p_corr[0] = tot[0] * inv_n;
        sc->p_corr[1] = tot[1] * inv_n;
        sc->p_corr[2] = tot[2] * inv_n;
        sc->u_core = tot[3];
        sc->u_shell = tot[4];
        const double ut = tot[kPairPart + kVirPart];
        sc->u_kspace = 0.5 * s.coulomb_k * ut;
        if (energy)
            for (int c = 0; c < 6; ++c)
                sc->virial[c] = tot[kPairPart + c] + 0.5 * s.coulomb_k * tot[kPairPart + kVirPart + 1 + c];
    }
}

// k-space force of eq. (29) (or eq. 23) on one atom per lane, looping over all
// modes two at a time; adds the short-range force minus the momentum
// correction, optionally the closing half kick of velocity Verlet.  The mixed
// form takes Im(e^{-i theta} rho) coef in FP32 and accumulates in FP64.
// k-space force of eq. (29) (eq. (23) for the full sum) of each atom,
// F_k = -k_e q_i sum_p (2 pi m_p / L) coef_p Im(e^{-i theta} rho_p).
// FUSED = false: written into the total-force arrays, which hold it until
// k_combine adds the short-range part (it needs only the positions and rho,
// so it can run on the second stream beside the pair kernel).  FUSED: the
// total force (F_short - F_corr) + F_k, closing kick and kinetic-energy
// partials (KE > 0) in the same pass, as k_combine computes them.  KE = 2
// (evaluations with energies): also the atom's share of each mode's energy,
// (k_e/2) q_i Re(e^{-i theta} rho_p) coef_p, and of its virial, that times
// (delta_ab - g_p k_a k_b); with the pair kernel's shares and the final
// velocity they give the stress and heat-flux partials of eqs. (50)-(51).
template <bool MIXED, bool FUSED, bool KICK, int KE, bool IPH>
__global__ __launch_bounds__(kBlock) void k_kforce(RB_ARGS, const KDev* __restrict__ kd)
{
    constexpr bool ENERGY = KE > 0;
    constexpr bool FLUX = FUSED && KE == 2;
    RB_SYS(blockIdx.x)
    const KDev k = global_view(kd[rb_m.x]);
    __shared__ double2 tab[MIXED ? 1 : kTableSize];
    if (!MIXED) {
        for (int t = threadIdx.x; t < kTableSize; t += blockDim.x)
            tab[t] = make_double2(k.table[2 * t], k.table[2 * t + 1]);
        __syncthreads();
    }
    const int i = lb * blockDim.x + threadIdx.x;
    double ke = 0.0;
    bool bad = false;
    double fl[kFluxPart];
    if (FLUX)
        for (int c = 0; c < kFluxPart; ++c) fl[c] = 0.0;
    if (i < s.n) {
        const double4 Pi = s.p[i];
        const double sc = MIXED ? 1.0 : (double)kTableSize;
        // scaled position: phase = m . u
        const double4 U = make_double4(Pi.x * (sc * s.invL[0]), Pi.y * (sc * s.invL[1]),
                                       Pi.z * (sc * s.invL[2]), 0.0);
        double Gx = 0.0, Gy = 0.0, Gz = 0.0;
        // FLUX: sum_p Re(e^{-i theta} rho_p) coef_p, and that times g_p m_a m_b
        double Ek = 0.0, Txx = 0.0, Tyy = 0.0, Tzz = 0.0, Txy = 0.0, Txz = 0.0, Tyz = 0.0;
        const uint4 Uf = IPH ? s.ufix[i] : make_uint4(0, 0, 0, 0);
        auto one = [&](const ModeRec& mr, int p, double gm) {
            double w, re = 0.0;
            if (MIXED) {
                float c, sn;
                if (IPH) {
                    const float tf = turns_fix(k.m[3 * p], k.m[3 * p + 1], k.m[3 * p + 2], Uf);
                    c = __builtin_amdgcn_cosf(tf);
                    sn = __builtin_amdgcn_sinf(tf);
                } else {
                    sincos_turns_f32(mode_phase(mr.mx, mr.my, mr.mz, U), c, sn);
                }
                // Im(e^{-i theta} rho) * coef = c * A - s * B
                w = (double)fmaf(c, mr.Af, -(sn * mr.Bf));
                // Re(e^{-i theta} rho) * coef = c * B + s * A
                if (FLUX) re = (double)fmaf(c, mr.Bf, sn * mr.Af);
            } else {
                double c, sn;
                sincos1024(mode_phase(mr.mx, mr.my, mr.mz, U), tab, c, sn);
                w = fma(c, mr.A, -(sn * mr.B));
                if (FLUX) re = fma(c, mr.B, sn * mr.A);
            }
            Gx = fma(w, mr.mx, Gx);
            Gy = fma(w, mr.my, Gy);
            Gz = fma(w, mr.mz, Gz);
            if (FLUX) {
                Ek += re;
                const double rg = re * gm;
                const double ax = rg * mr.mx, ay = rg * mr.my;
                Txx = fma(ax, mr.mx, Txx);
                Tyy = fma(ay, mr.my, Tyy);
                Tzz = fma(rg * mr.mz, mr.mz, Tzz);
                Txy = fma(ax, mr.my, Txy);
                Txz = fma(ax, mr.mz, Txz);
                Tyz = fma(ay, mr.mz, Tyz);
            }
        };
        int p = 0;
        for (; p + 2 <= k.n_modes; p += 2) {
            const ModeRec m0 = k.modes[p];
            const ModeRec m1 = k.modes[p + 1];
            one(m0, p, FLUX ? k.mode_g[p] : 0.0);
            one(m1, p + 1, FLUX ? k.mode_g[p + 1] : 0.0);
        }
        if (p < k.n_modes) one(k.modes[p], p, FLUX ? k.mode_g[p] : 0.0);
        const int ti = s.type[i];
        const double qk = -s.coulomb_k * s.spc->q[ti];
        if (!FUSED) {
            s.fx[i] = qk * s.two_pi_L[0] * Gx;
            s.fy[i] = qk * s.two_pi_L[1] * Gy;
            s.fz[i] = qk * s.two_pi_L[2] * Gz;
        } else {
            const DeviceScalars* scal = s.sc;
            const double fx = s.fsx[i] - scal->p_corr[0] + qk * s.two_pi_L[0] * Gx;
            const double fy = s.fsy[i] - scal->p_corr[1] + qk * s.two_pi_L[1] * Gy;
            const double fz = s.fsz[i] - scal->p_corr[2] + qk * s.two_pi_L[2] * Gz;
            s.fx[i] = fx;
            s.fy[i] = fy;
            s.fz[i] = fz;
            bad = !finite3(fx, fy, fz);
            double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
            if (KICK) {
                const double a = 0.5 * s.dt * s.spc->inv_mass_acc[ti];
                vx += a * fx;
                vy += a * fy;
                vz += a * fz;
                s.vx[i] = vx;
                s.vy[i] = vy;
                s.vz[i] = vz;
            }
            const double m = s.spc->mass[ti];
            if (ENERGY) ke = 0.5 * m * (vx * vx + vy * vy + vz * vz);
            if (FLUX) {
                const double hq = 0.5 * s.coulomb_k * s.spc->q[ti];
                const double tx = s.two_pi_L[0], ty = s.two_pi_L[1], tz = s.two_pi_L[2];
                const double4 a0 = s.at_ew[2 * (size_t)i];
                const double4 a1 = s.at_ew[2 * (size_t)i + 1];
                const double ep = a0.x + hq * Ek - s.spc->self_e[ti];
                const double wxx = a0.y + hq * (Ek - tx * tx * Txx);
                const double wyy = a0.z + hq * (Ek - ty * ty * Tyy);
                const double wzz = a0.w + hq * (Ek - tz * tz * Tzz);
                const double wxy = a1.x - hq * (tx * ty) * Txy;
                const double wxz = a1.y - hq * (tx * tz) * Txz;
                const double wyz = a1.z - hq * (ty * tz) * Tyz;
                fl[0] = m * vx * vx;
                fl[1] = m * vy * vy;
                fl[2] = m * vz * vz;
                fl[3] = m * vx * vy;
                fl[4] = m * vx * vz;
                fl[5] = m * vy * vz;
                fl[6] = ke * vx;
                fl[7] = ke * vy;
                fl[8] = ke * vz;
                fl[9] = ep * vx + (wxx * vx + wxy * vy + wxz * vz);
                fl[10] = ep * vy + (wxy * vx + wyy * vy + wyz * vz);
                fl[11] = ep * vz + (wxz * vx + wyz * vy + wzz * vz);
            }
        }
    }
    if (FUSED) flag_nonfinite(bad, s.sc);
    if (FUSED && ENERGY) wave_partial(ke, i, s.n, s.kin_part, 1, 0);
    if (FLUX)
        for (int c = 0; c < kFluxPart; ++c) wave_partial(fl[c], i, s.n, s.flux_part, kFluxPart, c);
}

// Total force F = (F_short - F_corr) + F_k (eqs. 26-29; F_k from k_kforce),
// the closing half kick, and kinetic-energy partials.
template <bool KICK, bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_combine(RB_ARGS)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    double ke = 0.0;
    bool bad = false;
    if (i < s.n) {
        const int ti = s.type[i];
        const DeviceScalars* scal = s.sc;
        const double fx = s.fsx[i] - scal->p_corr[0] + s.fx[i];
        const double fy = s.fsy[i] - scal->p_corr[1] + s.fy[i];
        const double fz = s.fsz[i] - scal->p_corr[2] + s.fz[i];
        s.fx[i] = fx;
        s.fy[i] = fy;
        s.fz[i] = fz;
        bad = !finite3(fx, fy, fz);
        if (KICK) {
            const double a = 0.5 * s.dt * s.spc->inv_mass_acc[ti];
            const double vx = s.vx[i] + a * fx, vy = s.vy[i] + a * fy, vz = s.vz[i] + a * fz;
            s.vx[i] = vx;
            s.vy[i] = vy;
            s.vz[i] = vz;
            if (ENERGY) ke = 0.5 * s.spc->mass[ti] * (vx * vx + vy * vy + vz * vz);
        } else if (ENERGY) {
            const double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
            ke = 0.5 * s.spc->mass[ti] * (vx * vx + vy * vy + vz * vz);
        }
    }
    flag_nonfinite(bad, s.sc);
    if (ENERGY) wave_partial(ke, i, s.n, s.kin_part, 1, 0);
}

// flux: the stress tensor (eq. 50) and heat flux (eq. 51) from the partials
// of the fused k-space pass.  The partials are of the stored velocities; the
// true ones are f times them, f the Nose-Hoover factor they owe (1 without
// it), so the kinetic tensor scales by f^2, the kinetic part of the flux by
// f^3 and the potential part by f.
__global__ __launch_bounds__(1024) void k_kinetic_finalize(const DevSys* __restrict__ sys, int step_end, int flux)
{
    const DevSys s = global_view(sys[blockIdx.x]);
    const double* part = s.kin_part;
    const int nb = (s.n + 63) / 64;  // wavefront partials
    __shared__ double red[16];
    double v = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v += part[b];
    const double t = block_sum(v, red);
    double ft[kFluxPart];
    if (flux) {
        for (int c = 0; c < kFluxPart; ++c) {
            double x = 0.0;
#pragma unroll 4
            for (int b = threadIdx.x; b < nb; b += blockDim.x) x += s.flux_part[(size_t)b * kFluxPart + c];
            ft[c] = block_sum(x, red);
        }
    }
    if (threadIdx.x == 0) {
        const double ke = t / kAccUnit;
        double f = 1.0;
        if (is_nh(s)) {
            if (step_end) {
                // closing half step; the velocities owe its factor until the
                // next opening kick (exports apply it)
                double K = ke;
                f = nh_half(s, s.sc, K);
                s.sc->vpend = f;
                s.sc->kinetic = K;
            } else {
                f = s.sc->vpend;
                s.sc->kinetic = ke * (f * f);
            }
        } else {
            s.sc->kinetic = ke;
            double lam = 1.0;
            if (s.thermo_c > 0.0 && s.thermostat == kThermoBerendsen && ke > 0.0) {
                // Berendsen: lambda^2 = 1 + (dt/tau)(T0/T - 1)
                const double T = 2.0 * ke / s.dof_kb;
                const double l2 = 1.0 + s.thermo_c * (s.t_target / T - 1.0);
                lam = l2 > 0.0 ? sqrt(l2) : 0.0;
            }
            s.sc->vscale = lam;
        }
        if (flux) {
            const double f2 = (f * f) / kAccUnit, f3 = f * f * f / kAccUnit;
            for (int c = 0; c < 6; ++c) s.sc->stress[c] = f2 * ft[c] + s.sc->virial[c];
            const double iV = 1.0 / ((s.L[0] * s.L[1]) * s.L[2]);
            for (int c = 0; c < 3; ++c) s.sc->heat_flux[c] = (f3 * ft[6 + c] + f * ft[9 + c]) * iV;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_kinetic(RB_ARGS)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    double ke = 0.0;
    if (i < s.n) {
        const double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
        ke = 0.5 * s.spc->mass[s.type[i]] * (vx * vx + vy * vy + vz * vz);
    }
    wave_partial(ke, i, s.n, s.kin_part, 1, 0);
}

// ---------------------------------------------------------------- integrator
// v += dt/2 F/m; r += dt v (wrapped); the displacement since the build is
// checked against skin/2, which raises the rebuild flag, as does a build
// scheduled for this step.
// LANGEVIN: the variant launched when some system of the batch runs the
// Langevin thermostat (its noise path needs many more registers).
template <bool LANGEVIN>
__global__ __launch_bounds__(kBlock) void k_kick_drift(RB_ARGS, int scheduled)
{
    RB_SYS(blockIdx.x)
    __shared__ double red[4];
    const int i = lb * blockDim.x + threadIdx.x;
    double d2 = 0.0;
    bool bad = false;
    const bool langevin = LANGEVIN && s.thermo_c > 0.0 && s.thermostat == kThermoLangevin;
    const double lam = (s.thermo_c > 0.0 && !langevin) ? s.sc->vscale : 1.0;
    if (i < s.n) {
        const int ti = s.type[i];
        const double a = 0.5 * s.dt * s.spc->inv_mass_acc[ti];
        double vx = lam * s.vx[i] + a * s.fx[i];
        double vy = lam * s.vy[i] + a * s.fy[i];
        double vz = lam * s.vz[i] + a * s.fz[i];
        const double4 P = s.p[i];
        double px, py, pz;
        if (langevin) {
            // BAOAB: half drift, Ornstein-Uhlenbeck velocity update with
            // Box-Muller normals of the stream (id, step, kTagLangevin), half drift
            PhiloxStream st(s.seed, (uint32_t)s.id[i], (uint32_t)s.sc->eval, kTagLangevin, s.replica);
            const double u1 = st.uniform(), u2 = st.uniform(), u3 = st.uniform(), u4 = st.uniform();
            // cos(2 pi u) and sin(2 pi u) as sincospi(2u): no large-argument reduction
            double sn2, cs2, sn4, cs4;
            sincospi(2.0 * u2, &sn2, &cs2);
            sincospi(2.0 * u4, &sn4, &cs4);
            (void)sn4;
            const double r = sqrt(-2.0 * log(1.0 - u1));
            const double z0 = r * cs2, z1 = r * sn2;
            const double z2 = sqrt(-2.0 * log(1.0 - u3)) * cs4;
            // the species constant read through the pointer: a per-lane index
            // into the local copy of the system record would move that copy
            // to scratch memory
            const double h = 0.5 * s.dt, c1 = s.lv_c1, c2 = sys[rb_m.x].lv_c2[ti];
            px = P.x + h * vx;
            py = P.y + h * vy;
            pz = P.z + h * vz;
            vx = c1 * vx + c2 * z0;
            vy = c1 * vy + c2 * z1;
            vz = c1 * vz + c2 * z2;
            px = px + h * vx;
            py = py + h * vy;
            pz = pz + h * vz;
        } else {
            px = P.x + s.dt * vx;
            py = P.y + s.dt * vy;
            pz = P.z + s.dt * vz;
        }
        s.vx[i] = vx;
        s.vy[i] = vy;
        s.vz[i] = vz;
        const double x = wrap_coord(px, s.L[0], s.invL[0]);
        const double y = wrap_coord(py, s.L[1], s.invL[1]);
        const double z = wrap_coord(pz, s.L[2], s.invL[2]);
        s.p[i] = make_double4(x, y, z, P.w);
        s.ufix[i] = fix_record(s, x, y, z, P.w);
        bad = !finite3(x, y, z);
        const double dx = min_image(x - s.xr[i], s.L[0], s.invL[0]);
        const double dy = min_image(y - s.yr[i], s.L[1], s.invL[1]);
        const double dz = min_image(z - s.zr[i], s.L[2], s.invL[2]);
        d2 = (dx * dx + dy * dy) + dz * dz;
    }
    // one flag update per wavefront that saw a displacement above skin/2
    const uint64_t moved = __ballot(!(d2 <= s.half_skin2));
    if (moved && (threadIdx.x & 63) == 0) atomicOr(&s.sc->rebuild, 1);
    if (scheduled && lb == 0 && threadIdx.x == 0) atomicOr(&s.sc->rebuild, 1);
    flag_nonfinite(bad, s.sc);
    // block maximum, then a device-wide max on the bit pattern (d2 >= 0)
    double m = d2;
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double b = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        // same-address atomics serialise: only a block above the value
        // already there (which only grows until the next build) updates it
        unsigned long long* slot = (unsigned long long*)&s.sc->max_disp2;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(b);
        if (bits > __atomic_load_n(slot, __ATOMIC_RELAXED)) atomicMax(slot, bits);
    }
}

// ---------------------------------------------------------------- exports
// Pair-distance histogram at the current positions, taken from the lists
// with the split the force uses (core entries inside the pair's core radius,
// candidates from there to r_shell), so every pair within r_shell appears
// once per direction while the lists are valid.  Bin k holds
// e_k <= r^2 < e_{k+1}, e_k = (k D)^2 in FP64: an estimate from sqrt is
// corrected against the exact edges.  Per-workgroup LDS counters, one
// global atomic per nonzero bin (integer sums: the counts do not depend on
// the order).
__global__ __launch_bounds__(kBlock) void k_rdf(RB_ARGS, double D, int n_bins, unsigned long long* counts)
{
    RB_SYS(blockIdx.x)
    extern __shared__ uint32_t hist[];  // [S][S][n_bins]
    const int S = s.n_species;
    const int nh = S * S * n_bins;
    for (int t = threadIdx.x; t < nh; t += blockDim.x) hist[t] = 0u;
    __syncthreads();
    const int i = lb * blockDim.x + threadIdx.x;
    if (i < s.n) {
        const double4 Pi = s.p[i];
        const int ti = s.type[i];
        const double top = ((double)n_bins * D) * ((double)n_bins * D);
        auto edge = [&](int k) { return ((double)k * D) * ((double)k * D); };
        auto visit = [&](int j, bool core) {
            const double4 Q = s.p[j];
            const double dx = min_image(Pi.x - Q.x, s.L[0], s.invL[0]);
            const double dy = min_image(Pi.y - Q.y, s.L[1], s.invL[1]);
            const double dz = min_image(Pi.z - Q.z, s.L[2], s.invL[2]);
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            const int tj = (int)Q.w;
            const double rc2 = s.species_cut ? s.pair[ti * S + tj].rc2 : s.rc2;
            const bool in = core ? r2 < rc2 : (r2 >= rc2 && r2 < s.rs2);
            if (!in || !(r2 < top)) return;
            int k = min((int)(sqrt(r2) / D), n_bins - 1);
            while (k + 1 < n_bins && edge(k + 1) <= r2) ++k;
            while (k > 0 && edge(k) > r2) --k;
            atomicAdd(&hist[(ti * S + tj) * n_bins + k], 1u);
        };
        const int nc = min(s.core_cnt[i], s.cap_core - 1);
        const int32_t* ctile = s.core_idx + (size_t)(i >> 6) * s.cap_core * 64 + (i & 63);
        for (int k = 0; k < nc; ++k) visit(ctile[(size_t)k * 64], true);
        const int nk = min(s.cand_cnt[i], s.cap_cand - 1);
        const int32_t* crow = s.cand_idx + (size_t)i * s.cap_cand;
        for (int k = 0; k < nk; ++k) visit(crow[k], false);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nh; t += blockDim.x)
        if (hist[t]) atomicAdd(&counts[t], (unsigned long long)hist[t]);
}

// Zero fill (a kernel, not a memset node: callers may capture the stream).
__global__ void k_zero_u64(unsigned long long* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Mean-square displacement bookkeeping, per atom by user index: the
// minimum-image increment since the last call is added to the unwrapped
// displacement D and the position kept (mark: D restarts at zero from the
// current positions).  Wavefront partials of |D|^2 and of the atom count per
// species, [waves][2 kMaxSpecies].
__global__ __launch_bounds__(kBlock) void k_msd(RB_ARGS, double* last, double* disp, double* part, int mark)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    int ti = -1;
    double q = 0.0;
    if (i < s.n) {
        const size_t u = 3 * (size_t)(s.user_off + s.id[i]);
        const double4 P = s.p[i];
        double* Lp = last + u;
        double* Dp = disp + u;
        if (mark) {
            Lp[0] = P.x;
            Lp[1] = P.y;
            Lp[2] = P.z;
            Dp[0] = Dp[1] = Dp[2] = 0.0;
        } else {
            const double dx = Dp[0] + min_image(P.x - Lp[0], s.L[0], s.invL[0]);
            const double dy = Dp[1] + min_image(P.y - Lp[1], s.L[1], s.invL[1]);
            const double dz = Dp[2] + min_image(P.z - Lp[2], s.L[2], s.invL[2]);
            Dp[0] = dx;
            Dp[1] = dy;
            Dp[2] = dz;
            Lp[0] = P.x;
            Lp[1] = P.y;
            Lp[2] = P.z;
            q = (dx * dx + dy * dy) + dz * dz;
        }
        ti = s.type[i];
    }
    for (int a = 0; a < s.n_species; ++a) {
        wave_partial(ti == a ? q : 0.0, i, s.n, part, 2 * kMaxSpecies, a);
        wave_partial(ti == a ? 1.0 : 0.0, i, s.n, part, 2 * kMaxSpecies, kMaxSpecies + a);
    }
}

__global__ void k_to_user3(RB_ARGS, int field, double* out)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const double* ax = field == 0 ? s.fx : (field == 1 ? s.fsx : s.vx);
    const double* ay = field == 0 ? s.fy : (field == 1 ? s.fsy : s.vy);
    const double* az = field == 0 ? s.fz : (field == 1 ? s.fsz : s.vz);
    const size_t u = ((size_t)s.user_off + s.id[i]) * 3;
    // velocities may still owe a Nose-Hoover factor (applied at the next kick)
    const double f = field == 2 ? s.sc->vpend : 1.0;
    out[u] = f * ax[i];
    out[u + 1] = f * ay[i];
    out[u + 2] = f * az[i];
}

__global__ void k_pos_to_user(RB_ARGS, double* out)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const size_t u = ((size_t)s.user_off + s.id[i]) * 3;
    const double4 P = s.p[i];
    out[u] = P.x;
    out[u + 1] = P.y;
    out[u + 2] = P.z;
}

__global__ void k_kspace_part(RB_ARGS, double* out)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const size_t u = ((size_t)s.user_off + s.id[i]) * 3;
    const DeviceScalars* sc = s.sc;
    out[u] = s.fx[i] - (s.fsx[i] - sc->p_corr[0]);
    out[u + 1] = s.fy[i] - (s.fsy[i] - sc->p_corr[1]);
    out[u + 2] = s.fz[i] - (s.fsz[i] - sc->p_corr[2]);
}

// Initial load: user order in, identity cell order (sorted at the first build).
__global__ void k_from_user(RB_ARGS, const int32_t* type, const double* pos, const double* vel)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    if (i >= s.n) return;
    const size_t u = (size_t)s.user_off + i;
    s.p[i] = make_double4(pos[3 * u], pos[3 * u + 1], pos[3 * u + 2], (double)type[u]);
    s.vx[i] = vel ? vel[3 * u] : 0.0;
    s.vy[i] = vel ? vel[3 * u + 1] : 0.0;
    s.vz[i] = vel ? vel[3 * u + 2] : 0.0;
    s.fx[i] = 0.0;
    s.fy[i] = 0.0;
    s.fz[i] = 0.0;
    s.type[i] = type[u];
    s.id[i] = i;
    s.inv[i] = i;
}

// New positions from the caller (user order), wrapped into the box; the
// lists stay.  Raises the system's stale flag when an atom now sits more
// than skin/2 from where it was at the last build, and keeps the largest
// displacement.
__global__ void k_set_pos(RB_ARGS, const double* pos)
{
    RB_SYS(blockIdx.x)
    const int i = lb * blockDim.x + threadIdx.x;
    double d2 = 0.0;
    if (i < s.n) {
        const size_t u = (size_t)s.user_off + s.id[i];
        const double x = wrap_coord(pos[3 * u], s.L[0], s.invL[0]);
        const double y = wrap_coord(pos[3 * u + 1], s.L[1], s.invL[1]);
        const double z = wrap_coord(pos[3 * u + 2], s.L[2], s.invL[2]);
        const double w = s.p[i].w;
        s.p[i] = make_double4(x, y, z, w);
        s.ufix[i] = fix_record(s, x, y, z, w);
        const double dx = min_image(x - s.xr[i], s.L[0], s.invL[0]);
        const double dy = min_image(y - s.yr[i], s.L[1], s.invL[1]);
        const double dz = min_image(z - s.zr[i], s.L[2], s.invL[2]);
        d2 = (dx * dx + dy * dy) + dz * dz;
    }
    if (__ballot(d2 > s.half_skin2) && (threadIdx.x & 63) == 0) atomicOr(&s.sc->stale, 1);
    double m = d2;
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax((unsigned long long*)&s.sc->max_disp2, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_clear_stale(DeviceScalars* sc, int R)
{
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        sc[r].stale = 0;
        sc[r].max_disp2 = 0.0;
    }
}

inline int blocks_for(int n, int b) { return (n + b - 1) / b; }

SogCoefF to_f32(const SogCoef& g)
{
    SogCoefF f{};
    f.n_exp = g.n_exp;
    f.chain = g.chain;
    f.n_poly = g.n_poly;
    for (int m = 0; m < kMaxExplicit; ++m) {
        f.a[m] = (float)g.a[m];
        f.fw[m] = (float)g.fw[m];
        f.ew[m] = (float)g.ew[m];
    }
    for (int n = 0; n < kMaxPoly; ++n) {
        f.pc[n] = (float)g.pc[n];
        f.pd[n] = (float)g.pd[n];
    }
    return f;
}

}  // namespace

// ---------------------------------------------------------------- launchers
void launch_set_eval(const Plan& P, uint64_t eval, hipStream_t st) { k_set_eval<<<1, 64, 0, st>>>(P.sc, P.R, eval); }
void launch_step_begin(const Plan& P, hipStream_t st) { k_step_begin<<<1, 64, 0, st>>>(P.sys, P.R); }
void launch_init_scalars(const Plan& P, hipStream_t st) { k_init_scalars<<<1, 64, 0, st>>>(P.sc, P.R); }
void launch_clear_flags(const Plan& P, hipStream_t st) { k_clear_flags<<<1, 64, 0, st>>>(P.sc, P.R); }

#define RB_MAP(shape) P.sys, P.shape.map

void launch_sort(const Plan& P, bool gate, hipStream_t st)
{
    if (P.atoms.blocks <= 0) return;
    const int g = gate ? 1 : 0;
    k_bin<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), g);
    k_scan<<<P.R, 1024, 0, st>>>(P.sys, g);
    k_scatter<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), g);
    k_cell_sort<<<P.cells.blocks, kBlock, 0, st>>>(RB_MAP(cells), g);
    k_gather<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), g);
}

void launch_lists(const Plan& P, bool gate, hipStream_t st)
{
    if (P.atoms.blocks <= 0) return;
    const int g = gate ? 1 : 0;
    // the memory form builds chunk by chunk: candidate rows of one chunk of
    // cells, then the batch draw from them, in the same scratch rows
    const int K = P.stored ? P.n_chunks : 1;
    const size_t sm_sel = sizeof(uint32_t) * (size_t)((P.cap_cand + 31) / 32) * 64;
    for (int k = 0; k < K; ++k) {
        const Shape& cs = P.stored ? P.cell_chunk[k] : P.list_cells;
#define RB_LISTS(C)                                                                                    \
    do {                                                                                               \
        if (P.species_cut)                                                                             \
            k_lists_cell<kListCaps[C], true><<<cs.blocks, kListBlock, 0, st>>>(P.sys, cs.map, g, k);  \
        else                                                                                           \
            k_lists_cell<kListCaps[C], false><<<cs.blocks, kListBlock, 0, st>>>(P.sys, cs.map, g, k); \
    } while (0)
        if (P.list_mode < kListPerAtom && !P.stored) {
            // one launch per staging capacity in use (a batch can mix them)
            for (int q = 0; q < kListPerAtom; ++q) {
                const Shape& cq = P.list_by_cap[q];
                if (cq.blocks <= 0) continue;
#define RB_LISTS_Q(C)                                                                                  \
    do {                                                                                               \
        if (P.species_cut)                                                                             \
            k_lists_cell<kListCaps[C], true><<<cq.blocks, kListBlock, 0, st>>>(P.sys, cq.map, g, k);  \
        else                                                                                           \
            k_lists_cell<kListCaps[C], false><<<cq.blocks, kListBlock, 0, st>>>(P.sys, cq.map, g, k); \
    } while (0)
                if (q == 0)
                    RB_LISTS_Q(0);
                else if (q == 1)
                    RB_LISTS_Q(1);
                else
                    RB_LISTS_Q(2);
#undef RB_LISTS_Q
            }
        } else if (P.list_mode < kListPerAtom) {
            if (cs.blocks > 0) {
                if (P.list_mode == 0)
                    RB_LISTS(0);
                else if (P.list_mode == 1)
                    RB_LISTS(1);
                else
                    RB_LISTS(2);
            }
        } else {
            int capP2 = 1;
            while (capP2 < P.cap_cand) capP2 <<= 1;
            const size_t sm = sizeof(long long) * (size_t)capP2 + sizeof(int32_t) * ((size_t)capP2 + P.cap_core);
            k_lists<<<P.atom1.blocks, 64, sm, st>>>(RB_MAP(atom1), g);
        }
        if (P.stored && P.rows64.blocks > 0) k_select<<<P.rows64.blocks, 64, sm_sel, st>>>(RB_MAP(rows64), g, k);
    }
#undef RB_LISTS
    k_build_done<<<1, 64, 0, st>>>(P.sys, P.R, g);
}

void launch_build(const Plan& P, bool gate, hipStream_t st)
{
    launch_sort(P, gate, st);
    launch_lists(P, gate, st);
}

void launch_ksample(const Plan& P, hipStream_t st)
{
    // one wavefront per mode of every system (non-sampled systems return)
    if (P.modes64.blocks > 0) k_ksample<<<P.modes1.blocks, 64, 0, st>>>(RB_MAP(modes1), P.kd);
}

template <int KU>
void launch_pair_ku(const Plan& P, const SogCoef& g, const SogCoefF& gf, bool mixed, bool energy, hipStream_t st)
{
    const int bs = P.tune.pair_block;  // atoms per workgroup; twice as many threads
    // near-field table (mixed), then the Floyd masks of the per-evaluation
    // batch draw (none for a stored batch)
    const size_t tab = mixed ? sizeof(float4) * (size_t)P.near.n * (energy ? 2 : 1) : 0;
    const size_t xch = sizeof(double) * (energy ? 10 : 4) * (size_t)bs;
    const size_t sm = tab + xch + (P.stored ? 0 : sizeof(uint32_t) * (size_t)((P.cap_cand + 31) / 32) * bs);
    const int nb = P.pair_atoms.blocks;
#define RB_PAIR(M, E, J) k_pair<M, E, J, KU><<<nb, 2 * bs, sm, st>>>(RB_MAP(pair_atoms), g, gf, P.near)
    if (mixed) {
        if (energy)
            RB_PAIR(true, true, 1);
        else
            RB_PAIR(true, false, 1);
    } else if (g.chain == 1) {
        if (energy)
            RB_PAIR(false, true, 1);
        else
            RB_PAIR(false, false, 1);
    } else {
        if (energy)
            RB_PAIR(false, true, 2);
        else
            RB_PAIR(false, false, 2);
    }
#undef RB_PAIR
}

void launch_pair(const Plan& P, const SogCoef& g, bool mixed, bool energy, hipStream_t st)
{
    if (P.pair_atoms.blocks <= 0) return;
    const SogCoefF gf = to_f32(g);
    if (P.tune.pair_ku == 8)
        launch_pair_ku<8>(P, g, gf, mixed, energy, st);
    else
        launch_pair_ku<4>(P, g, gf, mixed, energy, st);
}

void launch_rho(const Plan& P, bool mixed, hipStream_t st)
{
    if (P.rho.blocks <= 0) return;
    const int nb = P.rho.blocks;
    const bool iph = mixed && P.iph;
    if (P.tune.rho_mpl == 2) {
        if (iph)
            k_rho<true, 2, true><<<nb, kBlock, 0, st>>>(RB_MAP(rho), P.kd);
        else if (mixed)
            k_rho<true, 2, false><<<nb, kBlock, 0, st>>>(RB_MAP(rho), P.kd);
        else
            k_rho<false, 2, false><<<nb, kBlock, 0, st>>>(RB_MAP(rho), P.kd);
    } else {
        if (iph)
            k_rho<true, 1, true><<<nb, kBlock, 0, st>>>(RB_MAP(rho), P.kd);
        else if (mixed)
            k_rho<true, 1, false><<<nb, kBlock, 0, st>>>(RB_MAP(rho), P.kd);
        else
            k_rho<false, 1, false><<<nb, kBlock, 0, st>>>(RB_MAP(rho), P.kd);
    }
}

void launch_rho_finalize(const Plan& P, hipStream_t st)
{
    if (P.modes1.blocks > 0) k_rho_finalize<<<P.modes1.blocks, 64, 0, st>>>(RB_MAP(modes1), P.kd);
}

void launch_finalize(const Plan& P, bool energy, hipStream_t st)
{
    if (P.R <= 0) return;
    k_finalize_part<<<P.R * P.fin_grid, 256, 0, st>>>(P.sys, P.kd, energy ? 1 : 0, P.fin_grid);
    k_finalize<<<P.R, 64, 0, st>>>(P.sys, energy ? 1 : 0);
}

void launch_kforce(const Plan& P, bool mixed, hipStream_t st)
{
    const int nb = P.kf_atoms.blocks;
    const int bs = P.tune.kf_block;
    if (nb <= 0) return;
    if (mixed && P.iph)
        k_kforce<true, false, false, 0, true><<<nb, bs, 0, st>>>(RB_MAP(kf_atoms), P.kd);
    else if (mixed)
        k_kforce<true, false, false, 0, false><<<nb, bs, 0, st>>>(RB_MAP(kf_atoms), P.kd);
    else
        k_kforce<false, false, false, 0, false><<<nb, bs, 0, st>>>(RB_MAP(kf_atoms), P.kd);
}

void launch_kforce_fused(const Plan& P, bool mixed, bool kick, int ke, hipStream_t st)
{
    const int nb = P.kf_atoms.blocks;
    const int bs = P.tune.kf_block;
    if (nb <= 0) return;
#define RB_KF(M, K, E)                                                                  \
    do {                                                                                \
        if (M && P.iph)                                                                 \
            k_kforce<M, true, K, E, M><<<nb, bs, 0, st>>>(RB_MAP(kf_atoms), P.kd);      \
        else                                                                            \
            k_kforce<M, true, K, E, false><<<nb, bs, 0, st>>>(RB_MAP(kf_atoms), P.kd);  \
    } while (0)
#define RB_KF_KE(M, K)        \
    do {                      \
        if (ke == 2)          \
            RB_KF(M, K, 2);   \
        else if (ke == 1)     \
            RB_KF(M, K, 1);   \
        else                  \
            RB_KF(M, K, 0);   \
    } while (0)
    if (mixed) {
        if (kick) RB_KF_KE(true, true); else RB_KF_KE(true, false);
    } else {
        if (kick) RB_KF_KE(false, true); else RB_KF_KE(false, false);
    }
#undef RB_KF_KE
#undef RB_KF
}

void launch_combine(const Plan& P, bool kick, bool energy, hipStream_t st)
{
    const int nb = P.atoms.blocks;
    if (nb <= 0) return;
    if (kick) {
        if (energy)
            k_combine<true, true><<<nb, kBlock, 0, st>>>(RB_MAP(atoms));
        else
            k_combine<true, false><<<nb, kBlock, 0, st>>>(RB_MAP(atoms));
    } else {
        if (energy)
            k_combine<false, true><<<nb, kBlock, 0, st>>>(RB_MAP(atoms));
        else
            k_combine<false, false><<<nb, kBlock, 0, st>>>(RB_MAP(atoms));
    }
}

void launch_kinetic_finalize(const Plan& P, bool step_end, bool flux, hipStream_t st)
{
    if (P.R > 0) k_kinetic_finalize<<<P.R, 1024, 0, st>>>(P.sys, step_end ? 1 : 0, flux ? 1 : 0);
}

void launch_kinetic(const Plan& P, hipStream_t st)
{
    if (P.atoms.blocks > 0) k_kinetic<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms));
}

void launch_kick_drift(const Plan& P, bool scheduled, hipStream_t st)
{
    if (P.atoms.blocks <= 0) return;
    if (P.langevin)
        k_kick_drift<true><<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), scheduled ? 1 : 0);
    else
        k_kick_drift<false><<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), scheduled ? 1 : 0);
}

// Per-device address of `scratch`, looked up once per device at context
// creation (with that device current).
constexpr int kMaxDevices = 64;
static unsigned long long* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

bool noalloc_init(int device, const char** err)
{
    if (device < 0 || device >= kMaxDevices) {
        *err = "device index above the allocation-free scratch table";
        return false;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return true;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        *err = hipGetErrorString(e);
        return false;
    }
    g_scratch_ptr[device] = static_cast<unsigned long long*>(ptr);
    return true;
}

unsigned long long* noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

void launch_zero_u64(unsigned long long* p, int n, hipStream_t st)
{
    if (n > 0) k_zero_u64<<<(n + kBlock - 1) / kBlock, kBlock, 0, st>>>(p, n);
}

void launch_rdf(const Plan& P, int n_species, double D, int n_bins, unsigned long long* counts, hipStream_t st)
{
    const size_t sm = sizeof(uint32_t) * (size_t)n_species * n_species * n_bins;
    if (P.atoms.blocks > 0) k_rdf<<<P.atoms.blocks, kBlock, sm, st>>>(RB_MAP(atoms), D, n_bins, counts);
}

void launch_msd(const Plan& P, double* last, double* disp, double* part, bool mark, hipStream_t st)
{
    if (P.atoms.blocks > 0) k_msd<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), last, disp, part, mark ? 1 : 0);
}

void launch_to_user3(const Plan& P, Field f, double* out, hipStream_t st)
{
    if (P.atoms.blocks > 0) k_to_user3<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), (int)f, out);
}

void launch_pos_to_user(const Plan& P, double* out, hipStream_t st)
{
    if (P.atoms.blocks > 0) k_pos_to_user<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), out);
}

void launch_kspace_part(const Plan& P, double* out, hipStream_t st)
{
    if (P.atoms.blocks > 0) k_kspace_part<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), out);
}

void launch_shell_ranks(const Plan& P, int32_t* out, int32_t* n_out, hipStream_t st)
{
    const size_t sm = sizeof(uint32_t) * (size_t)((P.cap_cand + 31) / 32) * kBlock;
    if (P.atoms.blocks > 0) k_shell_ranks<<<P.atoms.blocks, kBlock, sm, st>>>(RB_MAP(atoms), out, n_out);
}

void launch_shell_samples(const Plan& P, int32_t* out, int32_t* n_out, hipStream_t st)
{
    const size_t sm = sizeof(uint32_t) * (size_t)((P.cap_cand + 31) / 32) * kBlock;
    if (P.atoms.blocks > 0) k_shell_samples<<<P.atoms.blocks, kBlock, sm, st>>>(RB_MAP(atoms), out, n_out);
}

void launch_set_positions(const Plan& P, const double* pos, hipStream_t st)
{
    k_clear_stale<<<1, 64, 0, st>>>(P.sc, P.R);
    if (P.atoms.blocks > 0) k_set_pos<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), pos);
}

void launch_batch_ids(const Plan& P, int32_t* out, int32_t* n_out, hipStream_t st)
{
    if (P.atoms.blocks > 0) k_batch_ids<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), out, n_out);
}

void launch_from_user(const Plan& P, const int32_t* type, const double* pos, const double* vel, hipStream_t st)
{
    if (P.atoms.blocks > 0) k_from_user<<<P.atoms.blocks, kBlock, 0, st>>>(RB_MAP(atoms), type, pos, vel);
}

#undef RB_MAP

}  // namespace rbsog
