// Device building blocks of the sampler: counter-based random numbers, the
// Cholesky rank-1 update used by the RAM adaptation, deterministic
// wavefront/LDS reductions, and the device-resident state of the theta chain.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hbm {

constexpr int kBlock = 256;                 // objects per workgroup = one reduction tile
constexpr int kWave = 64;                   // CDNA wavefront width
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxP = 8;                    // largest theta dimension supported

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// counter words 0 and 2 by the two published multipliers, swaps the halves
// and mixes in the key; the key advances by the two Weyl increments after
// every round.  Everything stays in registers: no generator state in memory.
// ---------------------------------------------------------------------------
struct Block4 {
    uint32_t w[4];
};

__device__ __forceinline__ Block4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t key0, uint32_t key1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo_a = 0xD2511F53u * c0;
        const uint32_t hi_a = __umulhi(0xD2511F53u, c0);
        const uint32_t lo_b = 0xCD9E8D57u * c2;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi_b ^ c1 ^ key0;
        const uint32_t n2 = hi_a ^ c3 ^ key1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
        key0 += 0x9E3779B9u;
        key1 += 0xBB67AE85u;
    }
    return Block4{{c0, c1, c2, c3}};
}

// The 128 output bits (word 0 least significant) are cut into five 24-bit
// fields; field j becomes u_j = (field_j + 1) * 2^-24, exactly representable
// in float and double and never zero.
__device__ __forceinline__ uint32_t field24(const Block4 &b, int j)
{
    switch (j) {
    case 0: return b.w[0] & 0xFFFFFFu;
    case 1: return (b.w[0] >> 24) | ((b.w[1] & 0xFFFFu) << 8);
    case 2: return (b.w[1] >> 16) | ((b.w[2] & 0xFFu) << 16);
    case 3: return b.w[2] >> 8;
    default: return b.w[3] & 0xFFFFFFu;
    }
}

template <typename T>
__device__ __forceinline__ T uniform24(const Block4 &b, int j)
{
    return static_cast<T>(field24(b, j) + 1u) * static_cast<T>(5.9604644775390625e-08);
}

__device__ __forceinline__ void sincos_2pi(float u, float *s, float *c) { sincospif(2.0f * u, s, c); }
__device__ __forceinline__ void sincos_2pi(double u, double *s, double *c) { sincospi(2.0 * u, s, c); }

// Box-Muller (1958): (u0, u1) -> z0, z1 and (u2, u3) -> z2, z3.
template <typename T, int NZ>
__device__ __forceinline__ void normals(const Block4 &b, T *z)
{
    const T r0 = sqrt(static_cast<T>(-2) * log(uniform24<T>(b, 0)));
    T s, c;
    sincos_2pi(uniform24<T>(b, 1), &s, &c);
    z[0] = r0 * c;
    if (NZ > 1) z[1] = r0 * s;
    if (NZ > 2) {
        const T r1 = sqrt(static_cast<T>(-2) * log(uniform24<T>(b, 2)));
        sincos_2pi(uniform24<T>(b, 3), &s, &c);
        z[2] = r1 * c;
        if (NZ > 3) z[3] = r1 * s;
    }
}

// ---------------------------------------------------------------------------
// Rank-1 modification of a Cholesky factor: L' L'^T = L L^T + beta x x^T.
// Column by column: r = sqrt(L_jj^2 + beta x_j^2) becomes the new diagonal,
// the column below is (L_ij L_jj + beta x_j x_i) / r, the remaining vector
// becomes x_i - (x_j / L_jj) L_ij and beta becomes beta L_jj^2 / r^2 (the
// Schur complement of the first column is again of the same form).  It is an
// update for beta > 0 and a downdate for beta < 0; in the RAM step the
// result is always positive definite because 1 + beta >= 1 - alpha* > 0.
// L is packed lower, row-major: element (r, c) at r (r + 1) / 2 + c.
// ---------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void chol_rank1(T *L, T *x, T beta)
{
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int jj = j * (j + 1) / 2 + j;
        const T ljj = L[jj];
        const T xj = x[j];
        const T r = sqrt(ljj * ljj + beta * xj * xj);
        const T inv_r = static_cast<T>(1) / r;
        const T ratio = xj / ljj;
#pragma unroll
        for (int i = j + 1; i < D; ++i) {
            const int ij = i * (i + 1) / 2 + j;
            const T lij = L[ij];
            L[ij] = (lij * ljj + beta * xj * x[i]) * inv_r;
            x[i] = x[i] - ratio * lij;
        }
        beta = beta * (ljj * inv_r) * (ljj * inv_r);
        L[jj] = r;
    }
}

// RAM adaptation of eq (2.6): S_n S_n^T = S (I + c U U^T / |U|^2) S^T, done as
// the rank-1 modification of S S^T by c v v^T with v = S U / |U|.
template <typename T, int D>
__device__ __forceinline__ void ram_adapt(T *S, const T *U, T c)
{
    if (D == 1) {
        S[0] = S[0] * sqrt(static_cast<T>(1) + c);
        return;
    }
    T n2 = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) n2 += U[j] * U[j];
    if (!(n2 > static_cast<T>(0))) return;
    const T inv_n = static_cast<T>(1) / sqrt(n2);
    T v[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        T acc = 0;
#pragma unroll
        for (int s = 0; s <= r; ++s) acc += S[r * (r + 1) / 2 + s] * U[s];
        v[r] = acc * inv_n;
    }
    chol_rank1<T, D>(S, v, c);
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  A wavefront sums with a fixed xor butterfly; a
// workgroup adds its four wave sums in fixed order.  The result depends only
// on the values and their lane positions, never on timing.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sums NV values over the workgroup; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double *v, double (*lds)[kWavesPerBlock])
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) lds[q][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = (lds[q][0] + lds[q][1]) + (lds[q][2] + lds[q][3]);
    }
}

// ---------------------------------------------------------------------------
// Device-resident state of the population-parameter chain.  Written only by
// the single lane that runs the theta step / sweep epilogue; read by every
// workgroup of the next sweep.
// ---------------------------------------------------------------------------
enum : int32_t {
    kFlagNonFiniteState = 1,   // a latent's current log density was not finite
    kFlagTraceFull = 2,        // theta trace capacity reached
    kFlagNoSums = 4,           // theta step without a preceding sweep
    kFlagBadZ = 8,             // selection normaliser not positive/finite
};

struct CycleState {
    double theta[kMaxP];           // current theta
    double chol_theta[kMaxP * kMaxP];   // proposal factor, p x p lower, row-major (stride p)
    double prop[kMaxP];            // pending proposal for sweep k + 1
    double zprop[kMaxP];           // its standard normals
    double used_prop[kMaxP];       // proposal the last sweep's sums refer to
    double used_z[kMaxP];
    double logZ_cur;               // ln Z(theta)
    double logZ_pending;           // ln Z(prop), written by the sweep's quadrature workgroup
    double logZ_used;              // ln Z(used_prop)
    double lprior_cur, lprior_prop, lprior_used;
    double eta_next;               // eta of sweep k + 1
    double eta_used;               // eta of the sweep just done (also the theta step's)
    double aux_cur, aux_prop, aux_used;   // per-theta model scalar (lnGamma(beta + 1) for LF models)
    double sum_lf;                 // sum_i log f(chi_i; theta) after the last sweep
    double sum_dlf;                // sum_i [log f(chi_i; used_prop) - log f(chi_i; theta)]
    double n_acc_last;             // accepted latent moves in the last sweep
    double delta_last, alpha_last; // last theta step
    double poplik_out;             // result slot of pop_loglik
    double poplik_logz;
    double zc_prop[4];             // FP64 constants of the pending proposal for the quadrature
    int64_t k;                     // sweeps done
    int64_t n_theta;               // theta steps done (= trace rows written)
    int32_t prop_valid, used_valid;
    int32_t sums_ready;
    int32_t accepted_last;
    int32_t flags;
    int32_t first_bad;             // smallest object index with a non-finite initial density
    float kc_f[32];                // per-sweep kernel constants, FP32 models
    double kc_d[32];               // per-sweep kernel constants, FP64 models
};
static_assert(sizeof(CycleState) % 8 == 0, "CycleState is staged through LDS in 8-byte words");

// Per-context constants that never change after init.
struct Statics {
    int64_t n;
    int64_t trace_cap;             // rows of the theta trace
    int64_t snap_cap;              // latent snapshots that fit
    int32_t thin;
    int32_t nq;
    int32_t adapt_theta;
    int32_t p;
    uint32_t key0, key1;
    double gamma;                  // eta exponent
    double alpha_star, alpha_star_theta;
    double mc[16];                 // model constants as given
    double md[16];                 // derived model constants (FP64)
    float mf[16];                  // derived model constants (FP32)
};

}  // namespace hbm
