// Device-side building blocks shared by the libnqs kernels (gfx950 / CDNA4):
// Philox4x32-10, wave64 DPP reductions, MFMA operand types, BF16 splitting,
// and the layout descriptor every kernel receives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nqs {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Layout of one context's device data.
//
// Parameters live in an augmented matrix Pm[Ma][Na] (float64):
//   Pm[j][i] = W_ji (j < M, i < N),  Pm[j][N] = b_j,  Pm[M][i] = a_i,
//   every other entry 0.
// With the augmented configuration s~ = (s_0..s_{N-1}, 1, 0..) and the
// augmented hidden activations t~ = (tanh theta_0..tanh theta_{M-1}, 1, 0..)
// the log-derivative vector of one sample is the outer product t~ (x) s~:
// O_W = t s, O_b = t, O_a = s (paper, log-derivative equation), so the QGT
// products and the force become two dense contractions over samples.
// Hidden-unit rows of activations and tables have Mw >= M + 1 entries, a
// multiple of 16 and covering 64 * QMAX with QMAX = ceil(M / 64) rounded up to
// a power of two (one wave64 spans the hidden units of one chain in the
// sampler, QMAX per lane); entries past M are zero in the tables.
// ---------------------------------------------------------------------------
struct Dims {
    int N;        // sites
    int M;        // hidden units
    int Na;       // round_up(N + 1, 16): augmented site width
    int Ma;       // round_up(M + 1, 16): augmented hidden rows
    int Mw;       // activation / table row width
    int Nw;       // round_up(N, 64): width of the hidden-major table rows
    int Kb;       // round_up(Na, 32): K extent of the BF16 theta operand
    int Kq;       // round_up(Na, 128): site extent of the CG operands (whole k-groups)
    int QM;       // ceil(M / 64): hidden units per lane in the sampler
    int vb, hb;   // visible / hidden bias present
};

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the Philox S-box with
// multipliers 0xD2511F53 / 0xCD9E8D57 and key increments 0x9E3779B9 /
// 0xBB67AE85.  Counter words: (proposal lo, proposal hi, chain, stream tag).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint64_t seed) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// index in [0, n) by multiply-shift of one random word
__device__ __forceinline__ int mulshift(uint32_t x, int n) {
    return (int)(((uint64_t)x * (uint64_t)(uint32_t)n) >> 32);
}

// 53-bit uniform in [0, 1): 27 bits of x1, 26 bits of x2
__device__ __forceinline__ double unit53(uint32_t x1, uint32_t x2) {
    return ((double)(x1 >> 5) * 67108864.0 + (double)(x2 >> 6)) * 1.1102230246251565e-16;
}

// ---------------------------------------------------------------------------
// wave64 reductions with DPP inside rows of 16 lanes, then readlane across
// the four rows.  Every lane of the wave must be active.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// DPP controls: quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E, row_ror:4 = 0x124,
// row_ror:8 = 0x128.  After the four steps every lane holds its row's result.
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x124>(v);
    v += dpp<0x128>(v);
    return v;
}
template <typename T>
__device__ __forceinline__ T row16_prod(T v) {
    v *= dpp<0xB1>(v);
    v *= dpp<0x4E>(v);
    v *= dpp<0x124>(v);
    v *= dpp<0x128>(v);
    return v;
}
__device__ __forceinline__ float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
// full-wave sum / product, result uniform across the wave
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v = row16_sum(v);
    return (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
}
template <typename T>
__device__ __forceinline__ T wave_prod(T v) {
    v = row16_prod(v);
    return (readlane(v, 0) * readlane(v, 16)) * (readlane(v, 32) * readlane(v, 48));
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Row of the 16 x 16 accumulator held in slot i by a lane with lk = lane / 16
// (column = lane % 16).  FP32 and BF16 16x16 MFMAs: row = 4 lk + i; the FP64
// 16x16x4 MFMA interleaves: row = 4 i + lk (measured on gfx950).
template <typename R>
__device__ __forceinline__ int acc_row(int lk, int i) {
    return sizeof(R) == 8 ? 4 * i + lk : 4 * lk + i;
}

// ---------------------------------------------------------------------------
// BF16 helpers: round-to-nearest-even conversion and a two-term split
// x ~= hi + lo with hi = bf16(x), lo = bf16(x - hi).
// ---------------------------------------------------------------------------
__host__ __device__ inline uint16_t f32_to_bf16_bits(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);  // inf / nan
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_bits_to_f32(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Philox stream tags
enum : uint32_t { TAG_METROPOLIS = 0, TAG_START = 1 };

}  // namespace nqs
