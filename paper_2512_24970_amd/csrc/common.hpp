// Shared declarations of the librbsog host code and HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rbsog {

constexpr int kMaxSpecies = 8;
constexpr int kMaxSog = 511;      // highest Gaussian index of the SOG series
constexpr int kMaxExplicit = 24;  // narrow Gaussians evaluated one by one
constexpr int kMaxPoly = 16;      // Taylor terms that replace the wide Gaussians
constexpr int kTableBits = 10;    // sincos table: e^{2 pi i j / 1024}
constexpr int kTableSize = 1 << kTableBits;
constexpr uint32_t kTagShell = 2u;
constexpr uint32_t kTagKmode = 3u;
constexpr uint32_t kTagShellBuild = 5u;  // shell batch drawn once per list build
constexpr uint32_t kTagLangevin = 6u;    // Langevin noise, counter word 1 = step number
// thermostat kinds (rbsog_params.thermostat)
constexpr int kThermoBerendsen = 0, kThermoNoseHoover = 1, kThermoLangevin = 2;
constexpr int kMaxListChunks = 64;      // launches a list build may be cut into
constexpr double kPi = 3.14159265358979323846;
// 1 eV/(Angstrom*amu) in Angstrom/ps^2
constexpr double kAccUnit = 9648.533212331;

// BMH pair coefficients of one species pair, pre-combined for the kernels.
struct PairCoef {
    double qq;    // k_e q_i q_j
    double A;     // repulsion A exp((sigma - r)/rho)
    double sig;
    double irho;  // 1/rho
    double C;
    double D;
    // core/shell split of the pair (species-dependent core radius r_c):
    double rc2;       // r_c^2 (core sum inside, shell sample outside)
    double rc2_list;  // (r_c + skin)^2, core-list bound
    double lo2_list;  // (r_c - skin)^2 (0 if negative), candidate lower bound
    double pad;
};

// Near-field SOG sum, split for the kernels.  With b^(2J) = 2 the Gaussian
// g_m(r) = exp(-r^2/(2 sigma_m^2)) satisfies g_m = g_{m+J}^2, so the narrow
// ones follow from J exponentials by squaring; the wide ones (sigma_m well
// above r_shell) are summed as a Taylor polynomial in r^2.
struct SogCoef {
    int n_exp;                 // explicit m = 0..n_exp-1
    int chain;                 // J
    int n_poly;                // polynomial terms
    int pad;
    double a[kMaxExplicit];    // 1/(2 sigma_m^2)
    double fw[kMaxExplicit];   // w_m / sigma_m^2   (force)
    double ew[kMaxExplicit];   // w_m               (energy)
    double pc[kMaxPoly];       // sum_{m>=n_exp} w_m/sigma_m^2 (-a_m)^n/n!
    double pd[kMaxPoly];       // sum_{m>=n_exp} w_m (-a_m)^n/n!
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__host__ __device__ inline void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Word stream of counter (index, eval, tag | replica << 8, block), key = seed.
struct PhiloxStream {
    uint32_t c0, c1, c2, blk, k0, k1;
    uint32_t w0, w1, w2, w3;
    int left;

    __host__ __device__ PhiloxStream(uint64_t seed, uint32_t index, uint32_t eval, uint32_t tag, uint32_t replica)
        : c0(index), c1(eval), c2((tag & 0xFFu) | (replica << 8)), blk(0), k0((uint32_t)seed),
          k1((uint32_t)(seed >> 32)), w0(0), w1(0), w2(0), w3(0), left(0)
    {
    }

    __host__ __device__ uint32_t next()
    {
        if (left == 0) {
            w0 = c0;
            w1 = c1;
            w2 = c2;
            w3 = blk;
            philox4x32_10(w0, w1, w2, w3, k0, k1);
            ++blk;
            left = 4;
        }
        const uint32_t r = w0;
        w0 = w1;
        w1 = w2;
        w2 = w3;
        --left;
        return r;
    }

    // 53-bit uniform in [0, 1): 27 high bits of one word, 26 of the next.
    __host__ __device__ double uniform()
    {
        const uint32_t a = next() >> 5;
        const uint32_t b = next() >> 6;
        return ((double)a * 67108864.0 + (double)b) * (1.0 / 9007199254740992.0);
    }

    // Integer in [0, range) by Lemire's multiply-shift with rejection.
    __host__ __device__ uint32_t bounded(uint32_t range)
    {
        uint64_t m = (uint64_t)next() * range;
        uint32_t l = (uint32_t)m;
        if (l < range) {
            const uint32_t t = (0u - range) % range;
            while (l < t) {
                m = (uint64_t)next() * range;
                l = (uint32_t)m;
            }
        }
        return (uint32_t)(m >> 32);
    }
};

// Per-evaluation scalars that live on the device.
struct DeviceScalars {
    uint64_t eval;        // Philox counter of the current force evaluation
    double p_corr[3];     // momentum correction
    double u_core, u_shell, u_kspace, kinetic;
    double max_disp2;     // largest squared displacement since the build
    int32_t overflow;     // list or cell capacity exceeded
    int32_t rebuild;      // the lists are rebuilt in this step
    int32_t nonfinite;    // a non-finite position or force was produced
    int32_t stale;        // positions set by the caller moved an atom more than skin/2 from its build position
    int64_t n_builds;     // list builds since the system was set
    int32_t max_core;     // largest core / candidate list seen (true sizes)
    int32_t max_cand;
    double vscale;        // thermostat velocity factor for the next step
    double nh_x, nh_v;    // Nose-Hoover variable and its velocity
    double vpend;         // factor the stored velocities still owe (Nose-Hoover half step at a step's end)
    double virial[6];     // W_ab of the last evaluation with energies (xx, yy, zz, xy, xz, yz)
    double stress[6];     // S_ab of eq. (50) at the end of that evaluation (same order), eV
    double heat_flux[3];  // J of eq. (51), eV / (A^2 ps)
};

}  // namespace rbsog
