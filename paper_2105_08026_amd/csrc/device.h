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
constexpr int kMaxStats = 6;                // most sufficient statistics of a model

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
        // one 32x32 -> 64-bit multiply each (a single v_mad_u64_u32)
        const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        // three-way XORs: one v_bitop3_b32 each (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pb >> 32), c1, key0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pa >> 32), c3, key1, 0x96);
        c0 = n0;
        c1 = static_cast<uint32_t>(pb);
        c2 = n2;
        c3 = static_cast<uint32_t>(pa);
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

// Box-Muller (1958): (u0, u1) -> z0, z1 and (u2, u3) -> z2, z3.  In single
// precision the hardware transcendentals are used directly: v_cos_f32 and
// v_sin_f32 take their argument in revolutions (cos(2 pi u) is one
// instruction), v_log_f32 is log2.  The per-object log densities keep the
// correctly rounded library functions.
__device__ __forceinline__ float ln_fast(float u) { return __builtin_amdgcn_logf(u) * 0.693147180559945309f; }

// exp and expm1 in single precision for the per-object log densities.  Both
// reduce x = k ln 2 + r with k = rint(x log2 e).  exp: 2^k times the hardware
// exp2 of (x log2 e - k), the product carried in two parts (log2 e split into
// its float value and the float of the remainder), ~1 ulp.  expm1: 2^k
// (expm1(r) + 1) - 1 = fma(2^k, expm1(r), 2^k - 1) with r = x - k ln 2 (ln 2
// in two parts) and expm1(r) from its Taylor series through r^7 (|r| <=
// ln 2 / 2: truncation below 2e-8 relative), so small arguments keep full
// relative accuracy.  Arguments are first clamped (one v_med3) to where the
// reductions stay exact: exp gives 0 below -104 and +inf above 88.73, expm1
// gives -1 below -88 and a finite 1.65e38 above 88; no other special cases.
__device__ __forceinline__ float exp_fin(float x)
{
    constexpr float kL2e = 1.44269504088896341f;
    constexpr float kL2eLo = 1.92596299e-08f;        // log2 e - kL2e
    x = __builtin_amdgcn_fmed3f(x, -104.0f, 89.0f);
    const float ph = x * kL2e;
    const float pl = fmaf(x, kL2eLo, fmaf(x, kL2e, -ph));
    const float k = __builtin_rintf(ph);
    return ldexpf(__builtin_amdgcn_exp2f((ph - k) + pl), static_cast<int>(k));
}

__device__ __forceinline__ float expm1_fin(float x)
{
    constexpr float kL2e = 1.44269504088896341f;
    constexpr float kLn2Hi = 0.693145751953125f;     // ln 2 to 16 significant bits
    constexpr float kLn2Lo = 1.42860682e-06f;        // ln 2 - kLn2Hi
    x = __builtin_amdgcn_fmed3f(x, -88.0f, 88.0f);
    const float k = __builtin_rintf(x * kL2e);
    const float r = fmaf(-k, kLn2Lo, fmaf(-k, kLn2Hi, x));
    float q = fmaf(r, 1.0f / 5040.0f, 1.0f / 720.0f);
    q = fmaf(r, q, 1.0f / 120.0f);
    q = fmaf(r, q, 1.0f / 24.0f);
    q = fmaf(r, q, 1.0f / 6.0f);
    q = fmaf(r, q, 0.5f);
    const float p = fmaf(r * r, q, r);
    const float t = ldexpf(1.0f, static_cast<int>(k));
    return fmaf(t, p, t - 1.0f);
}

template <typename T, int NZ>
__device__ __forceinline__ void normals(const Block4 &b, T *z);

template <int NZ>
__device__ __forceinline__ void normals_f(const Block4 &b, float *z)
{
    const float u1 = uniform24<float>(b, 1);
    const float r0 = __builtin_amdgcn_sqrtf(-2.0f * ln_fast(uniform24<float>(b, 0)));
    z[0] = r0 * __builtin_amdgcn_cosf(u1);
    if (NZ > 1) z[1] = r0 * __builtin_amdgcn_sinf(u1);
    if (NZ > 2) {
        const float u3 = uniform24<float>(b, 3);
        const float r1 = __builtin_amdgcn_sqrtf(-2.0f * ln_fast(uniform24<float>(b, 2)));
        z[2] = r1 * __builtin_amdgcn_cosf(u3);
        if (NZ > 3) z[3] = r1 * __builtin_amdgcn_sinf(u3);
    }
}

template <int NZ>
__device__ __forceinline__ void normals_d(const Block4 &b, double *z)
{
    double s, c;
    const double r0 = sqrt(-2.0 * log(uniform24<double>(b, 0)));
    sincospi(2.0 * uniform24<double>(b, 1), &s, &c);
    z[0] = r0 * c;
    if (NZ > 1) z[1] = r0 * s;
    if (NZ > 2) {
        const double r1 = sqrt(-2.0 * log(uniform24<double>(b, 2)));
        sincospi(2.0 * uniform24<double>(b, 3), &s, &c);
        z[2] = r1 * c;
        if (NZ > 3) z[3] = r1 * s;
    }
}

template <typename T, int NZ>
__device__ __forceinline__ void normals(const Block4 &b, T *z)
{
    if constexpr (sizeof(T) == 4) normals_f<NZ>(b, z);
    else normals_d<NZ>(b, z);
}

// ln of the accept uniform, and alpha = min(1, e^delta) for the adaptation.
__device__ __forceinline__ float ln_uniform(const Block4 &b, float) { return ln_fast(uniform24<float>(b, 4)); }
__device__ __forceinline__ double ln_uniform(const Block4 &b, double) { return log(uniform24<double>(b, 4)); }
__device__ __forceinline__ float accept_prob(float delta)
{
    return delta >= 0.0f ? 1.0f : __builtin_amdgcn_exp2f(delta * 1.44269504088896341f);
}
__device__ __forceinline__ double accept_prob(double delta) { return delta >= 0.0 ? 1.0 : exp(delta); }

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
// FP32 factors take the hardware square root and reciprocal (within 1 ulp;
// the correctly rounded library forms cost ~20 and ~10 instructions each);
// FP64 factors keep the correctly rounded forms.
__device__ __forceinline__ float ram_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ __forceinline__ double ram_sqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float ram_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double ram_rcp(double v) { return 1.0 / v; }

template <typename T, int D>
__device__ __forceinline__ void chol_rank1(T *L, T *x, T beta)
{
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const int jj = j * (j + 1) / 2 + j;
        const T ljj = L[jj];
        const T xj = x[j];
        const T r = ram_sqrt(ljj * ljj + beta * xj * xj);
        const T inv_r = ram_rcp(r);
        const T ratio = xj * ram_rcp(ljj);
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
        S[0] = S[0] * ram_sqrt(static_cast<T>(1) + c);
        return;
    }
    T n2 = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) n2 += U[j] * U[j];
    if (!(n2 > static_cast<T>(0))) return;
    const T inv_n = ram_rcp(ram_sqrt(n2));
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
// Deterministic reductions.  A wavefront sums with fixed DPP steps; a
// workgroup first adds, lane by lane, the values of its four wavefronts in a
// fixed order.  The result depends only on the values and their lane
// positions, never on timing.
// ---------------------------------------------------------------------------
// One DPP move of a double (both 32-bit halves) into the rows of kRowMask.
// Lanes of other rows keep whatever their destination register held: callers
// read only lanes of enabled rows.  The quad permutations and row rotations
// used here take every lane's source from an active lane of its own row.
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t bits = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(bits & 0xffffffffu), kCtrl, kRowMask, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(bits >> 32), kCtrl, kRowMask, 0xf, false);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(lo));
}

__device__ __forceinline__ double lane_f64(double v, int lane)
{
    const uint64_t bits = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(bits & 0xffffffffu), lane);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(bits >> 32), lane);
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Wavefront sum in a fixed order: within each quad (DPP quad_perm swaps),
// then across the four quads of each 16-lane row (DPP row rotations), which
// leaves every lane of a row holding that row's sum; then row broadcasts:
// lane 15 of rows 0 and 2 is added into rows 1 and 3, lane 31 into rows 2
// and 3 (row 2's lanes are not read).  Lane 63 ends with (r3 + r2) + (r1 +
// r0) of the row sums, read once.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x124>(v);   // row_ror:4
    v += dpp_f64<0x128>(v);   // row_ror:8
    v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return lane_f64(v, 63);
}

// Sums NV values over the workgroup; result valid in thread 0.  Every
// thread leaves its values in LDS; wavefront 0 alone adds, lane by lane, the
// four values of lanes l, l + 64, l + 128, l + 192 as (w0 + w1) + (w2 + w3)
// and reduces its 64 lane sums with wave_sum -- one wavefront's DPP steps per
// value instead of four.  lds: [NV][256] doubles.
// The same reduction over the 256 threads of one slice of a larger
// workgroup: threads with part set hold the values, lane is their position
// in the slice (0..255, the slice's first wavefront reduces), lds its own
// staging rows.  Every thread of the workgroup calls it (one barrier).
template <int NV>
__device__ __forceinline__ void block_sum_at(double *v, double (*lds)[kBlock], int lane, bool part)
{
    if (part) {
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[q][lane] = v[q];
    }
    __syncthreads();
    if (part && lane < kWave) {
        const int l = lane;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double s = (lds[q][l] + lds[q][l + kWave]) + (lds[q][l + 2 * kWave] + lds[q][l + 3 * kWave]);
            const double r = wave_sum(s);
            if (l == 0) v[q] = r;
        }
    }
}

template <int NV>
__device__ __forceinline__ void block_sum(double *v, double (*lds)[kBlock])
{
    block_sum_at<NV>(v, lds, static_cast<int>(threadIdx.x), true);
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
    double aux_cur[2], aux_used[2];       // per-theta model scalars (lnGamma(beta + 1), ln s)
    double sum_lf;                 // sum_i log f(chi_i; theta) after the last sweep
    double sum_dlf;                // sum_i [log f(chi_i; used_prop) - log f(chi_i; theta)]
    double n_acc_last;             // accepted latent moves in the last sweep
    double delta_last, alpha_last; // last theta step
    double poplik_out;             // result slot of pop_loglik
    double poplik_logz;
    double zc_prop[4];             // FP64 constants of the pending proposal for the quadrature
    double sum_dlf_raw;            // per-object part of sum_dlf as reduced from the tiles
    double stats[kMaxStats];       // sufficient statistics of the last sweep, at the theta it ran with
    int64_t k;                     // sweeps done
    int64_t n_theta;               // theta steps done (= trace rows written)
    int64_t budget;                // theta steps after which the dataset stops (0: no limit)
    int32_t prop_valid, used_valid;
    int32_t sums_ready;
    int32_t accepted_last;
    int32_t flags;
    int32_t first_bad;             // smallest object index with a non-finite initial density
    int32_t active;                // 0: the dataset's tiles and theta step are skipped
    int32_t pad_;
    float kc_f[32];                // per-sweep kernel constants, FP32 models
    double kc_d[32];               // per-sweep kernel constants, FP64 models
};
static_assert(sizeof(CycleState) % 8 == 0, "CycleState is staged through LDS in 8-byte words");

// Per-dataset constants, fixed while the dataset is loaded.  Datasets are
// packed back to back in the caller's arrays; each starts a new 256-object
// tile, so no tile straddles two datasets.
struct Statics {
    int64_t n;                     // objects of this dataset
    int64_t obj_start;             // its first object in the packed arrays
    int32_t tile_start;            // its first tile
    int32_t n_tiles;               // its tiles, ceil(n / 256)
    int64_t trace_cap;             // rows of the theta trace
    int64_t snap_cap;              // latent snapshots that fit
    int32_t thin;
    int32_t nq;
    int32_t adapt_theta;
    int32_t p;
    int32_t substeps;              // theta steps per cycle from sufficient statistics (0: generic sums)
    int32_t snap_ring;             // 1 while a streamed run uses the snapshot rows as a ring
    uint32_t key0, key1;
    double gamma;                  // eta exponent
    double alpha_star, alpha_star_theta;
    double s0;                     // initial latent factor S_1 = s0 I
    double mc[16];                 // model constants as given
    double md[16];                 // derived model constants (FP64)
    float mf[16];                  // derived model constants (FP32)
};

}  // namespace hbm
